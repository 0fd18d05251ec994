"""Parity of the HIP path with the CPU oracle, through the C ABI (GPU only).

Every result is compared element by element, bit-exact (the output of a
permutation is unique): full arrays at sizes the oracle handles quickly (that
still span many tiles, plus sizes below one tile and below one wave), and the
full-size workloads of the benchmark either in full or on sampled outputs that
the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_07795_amd import binding as B
from synth import gen
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def run(n, rows, c, w, a, fn="permute", opts=None):
    x = G.to_device(a)
    y = G.empty_like_bytes(a)
    if fn == "permute":
        B.bmmc_permute(x, y, n, rows, c, w, G.stream())
    elif fn == "ex":
        B.bmmc_permute_ex(x, y, n, rows, c, w, opts, G.stream())
    elif fn == "naive":
        B.bmmc_permute_naive(x, y, n, rows, c, w, G.stream())
    G.sync()
    return G.to_host(y, a)


def check(n, rows, c, w, fn="permute", opts=None, seed=1):
    a = gen.data(n, w, seed)
    got = run(n, rows, c, w, a, fn, opts)
    want = O.permute(a, n, rows, c)
    assert np.array_equal(got, want), f"n={n} w={w} fn={fn} opts={opts}"


def test_device_present():
    assert torch.cuda.is_available()
    print("device:", torch.cuda.get_device_name(0), flush=True)


def test_bit_reversal_2p20_int32_full():
    """Bit reversal of 2^20 int32 filled from seed 0 (one tiled pass)."""
    n = 20
    rows = gen.bit_reversal_rows(n)
    p = B.bmmc_factorize(rows, 0, n)
    assert p.nfactors == 1
    a = gen.data(n, 4, 0)
    assert np.array_equal(run(n, rows, 0, 4, a), O.permute(a, n, rows, 0))


@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_random_2p26_int32_full(method):
    """Random BMMC on 2^26 int32, seed 0, full comparison: one general-tile
    pass (auto) and the paper's two tiled passes."""
    n = 26
    rows, c = gen.random_bmmc(n, 0)
    opts = {"method": method}
    assert B.bmmc_plan_ex(rows, c, n, 4, opts).nfactors == (1 if method == B.METHOD_AUTO else 2)
    a = gen.data(n, 4, 0)
    got = run(n, rows, c, 4, a, fn="ex", opts=opts)
    assert np.array_equal(got, O.permute(a, n, rows, c))


@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
@pytest.mark.parametrize("w", [4, 8])
@pytest.mark.parametrize("kind", ["random", "bitrev", "swap", "bpc", "cyclic", "reverse", "identity"])
@pytest.mark.parametrize("n", [1, 2, 3, 6, 9, 12, 13, 15, 18])
def test_small_sizes(kind, n, w, method):
    s = 31 * n + w
    rows, c = {
        "random": lambda: gen.random_bmmc(n, s),
        "bitrev": lambda: (gen.bit_reversal_rows(n), 0),
        "swap": lambda: (gen.block_swap_rows(n, n // 2), 0),
        "bpc": lambda: gen.random_bpc(n, s),
        "cyclic": lambda: (gen.cyclic_shift_rows(n), 1),
        "reverse": lambda: (gen.identity_rows(n), (1 << n) - 1),
        "identity": lambda: (gen.identity_rows(n), 0),
    }[kind]()
    check(n, rows, c, w, fn="ex", opts={"method": method})


@pytest.mark.parametrize("w", [1, 2, 16])
@pytest.mark.parametrize("n", [0, 1, 3, 5, 8, 11, 14, 17])
def test_other_widths(n, w):
    rows, c = gen.random_bmmc(n, 7 + n)
    check(n, rows, c, w)


@pytest.mark.parametrize("w", [4, 8, 16])
@pytest.mark.parametrize("n", [0, 5, 12, 16, 19])
def test_naive_kernel(n, w):
    rows, c = gen.random_bmmc(n, 3 * n)
    check(n, rows, c, w, fn="naive")


@pytest.mark.parametrize("n", [10, 14, 17, 20])
@pytest.mark.parametrize("w", [4, 8])
def test_onepass_method(n, w):
    rows, c = gen.random_bmmc(n, 11 * n)
    check(n, rows, c, w, fn="ex", opts={"method": B.METHOD_ONEPASS})


@pytest.mark.parametrize("opts", [
    {"threads": 512, "iters": 4}, {"threads": 1024, "iters": 2}, {"threads": 256, "iters": 8},
    {"threads": 256, "iters": 2}, {"threads": 1024, "iters": 4}, {"t": 5},
    {"swizzle": -1}, {"grid": 64}, {"grid": 1}, {"threads": 256, "iters": 16, "t": 7},
    {"run_in": 7, "run_out": 6, "threads": 512, "iters": 8, "tile_order": 2, "hints": 3},
    {"tile_order": 4 + 16 * 15, "grid": -1}, {"tile_order": 1 + 16 * 6, "grid": 96},
    {"hints": 3 | 8}, {"hints": 2 | 8, "threads": 512, "iters": 4}, {"hints": 4 | 8},
    {"threads": 1024, "iters": 4, "run_in": 6, "run_out": 8, "tile_order": 4 + 16 * 7, "hints": 3},
])
@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_shapes_and_grids(opts, method):
    n = 19
    rows, c = gen.random_bmmc(n, 99)
    check(n, rows, c, 4, fn="ex", opts={**opts, "method": method})


@pytest.mark.parametrize("opts", [{"threads": 256, "iters": 4}, {"threads": 512, "iters": 8},
                                  {"threads": 256, "iters": 16, "t": 6}])
def test_shapes_int64(opts):
    n = 18
    rows, c = gen.random_bmmc(n, 98)
    check(n, rows, c, 8, fn="ex", opts=opts)


def test_iota_payload_names_sources():
    n = 22
    rows, c = gen.random_bmmc(n, 5)
    a = gen.iota(n, 4)
    got = run(n, rows, c, 4, a)
    ys = O.index_map(rows, c, n).astype(np.int64)
    assert np.array_equal(got[ys], a)


def sampled_check(n, rows, c, w, got, a, count=1 << 16, seed=0):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    xs[:4] = [0, 1, (1 << n) - 2, (1 << n) - 1]
    ys = O.apply_many(rows, c, n, xs).astype(np.int64)
    assert np.array_equal(got[ys], a[xs.astype(np.int64)])


def shear_rows(n, w):
    """Identity plus three off-diagonal ones: the output bits above a 4 KiB
    block depend only on the same input bits (mixed among themselves), but
    one of those input bits also reaches a higher output bit and another a
    lower one."""
    blk = 12 - (w.bit_length() - 1)
    rows = gen.identity_rows(n)
    rows[20] |= 1 << blk
    rows[blk + 1] |= 1 << blk
    rows[5] |= 1 << (blk + 2)
    return rows


DEALT_KINDS = {
    "shear": lambda n, w: (shear_rows(n, w), 12345),
    "reverse": lambda n, w: (gen.identity_rows(n), (1 << n) - 1),
    "swap7": lambda n, w: (gen.block_swap_rows(n, 7), 0),
    "bitrev": lambda n, w: (gen.bit_reversal_rows(n), 0),
    "swap_half": lambda n, w: (gen.block_swap_rows(n, n // 2), 0),
    "bpc": lambda n, w: gen.random_bpc(n, n + w),
    "random": lambda n, w: gen.random_bmmc(n, n + w),
}


@pytest.mark.parametrize("small_tile", [False, True])
@pytest.mark.parametrize("w", [4, 8])
@pytest.mark.parametrize("kind", sorted(DEALT_KINDS))
def test_dealt_output_blocks(kind, w, small_tile):
    """Tile order + 256 (each tile writes 4 KiB blocks of one class where the
    matrix allows it, the plain choice elsewhere), on the library's shape and
    on the 16 KiB tile the per-matrix tuner offers with it: in full."""
    n = 22 if w == 4 else 21
    rows, c = DEALT_KINDS[kind](n, w)
    opts = {"tile_order": 256 + 4}
    if small_tile:
        opts.update(threads=512, iters=2, run_in=5 if w == 4 else 4, run_out=7)
    check(n, rows, c, w, fn="ex", opts=opts)


@pytest.mark.parametrize("case", ["random28_i32", "random27_i64", "bitrev28_i32", "swap28_i32",
                                  "swap27_i64", "random28_i32_tiled", "random27_i64_tiled",
                                  "reverse28_i32_dealt", "swap7_27_i64_dealt", "reverse28_i32", "xor27_i64",
                                  "shear28_i32", "shear27_i64"])
def test_full_size_sweep_sampled(case):
    """The 1 GiB sweep arrays in the benchmark's launch configuration (and in
    the paper's two-pass scheme), and the default call on matrices that keep
    their 4 KiB-block bits (dealt output blocks by default at this size),
    checked on 65536 sampled outputs computed one by one by the oracle."""
    n, w = (28, 4) if "i32" in case else (27, 8)
    if case.startswith("random"):
        rows, c = gen.random_bmmc(n, 1)
    elif case.startswith("bitrev"):
        rows, c = gen.bit_reversal_rows(n), 0
    elif case.startswith("reverse"):
        rows, c = gen.identity_rows(n), (1 << n) - 1
    elif case.startswith("xor"):
        rows, c = gen.identity_rows(n), gen.random_bmmc(n, 3)[1] | 1
    elif case.startswith("shear"):
        rows, c = shear_rows(n, w), 12345
    elif case.startswith("swap7"):
        rows, c = gen.block_swap_rows(n, 7), 0
    else:
        rows, c = gen.block_swap_rows(n, n // 2), 0
    a = gen.data(n, w, 1)
    if case.endswith("tiled"):
        got = run(n, rows, c, w, a, fn="ex", opts={"method": B.METHOD_TILED})
    elif case.endswith("dealt"):
        # dealt output blocks on the 16 KiB tile (the per-matrix tuner's candidate)
        got = run(n, rows, c, w, a, fn="ex", opts={"tile_order": 256 + 4, "threads": 512, "iters": 2,
                                                   "run_in": 5 if w == 4 else 4, "run_out": 7})
    else:
        got = run(n, rows, c, w, a)
    sampled_check(n, rows, c, w, got, a)


@pytest.mark.parametrize("n,w", [(25, 16), (28, 2)])
def test_default_call_dealt_other_widths(n, w):
    """The default call's dealt output blocks for 16- and 2-byte elements
    (512 MiB, the class options' shape): the reversal, on sampled outputs."""
    rows, c = gen.identity_rows(n), (1 << n) - 1
    a = gen.data(n, w, 6)
    got = run(n, rows, c, w, a)
    sampled_check(n, rows, c, w, got, a)


@pytest.mark.parametrize("kind", ["random", "bitrev"])
@pytest.mark.parametrize("n,w", [(22, 4), (23, 4), (24, 4), (21, 8), (22, 8), (23, 8), (27, 4), (26, 8)])
def test_size_dependent_defaults(n, w, kind):
    """The library's size-dependent defaults (explicit method, so no tuning
    file entry applies): in full up to 64 MiB, on sampled outputs above."""
    rows, c = gen.random_bmmc(n, 2 * n + w) if kind == "random" else (gen.bit_reversal_rows(n), 0)
    a = gen.data(n, w, 3)
    got = run(n, rows, c, w, a, fn="ex", opts={"method": B.METHOD_AUTO})
    if (1 << n) * w <= (64 << 20):
        assert np.array_equal(got, O.permute(a, n, rows, c))
    else:
        sampled_check(n, rows, c, w, got, a)


def test_copy_kernel():
    for nbytes in (16, 4096, 1 << 22, (1 << 20) + 5, 3):
        a = np.frombuffer(np.random.default_rng(nbytes).bytes(nbytes), dtype=np.uint8).copy()
        x = G.to_device(a)
        y = torch.zeros(nbytes, dtype=torch.uint8, device=G.dev())
        B.bmmc_copy(x, y, nbytes, G.stream())
        G.sync()
        assert np.array_equal(y.cpu().numpy(), a)


def test_same_result_on_side_stream():
    n = 20
    rows, c = gen.random_bmmc(n, 77)
    a = gen.data(n, 4, 2)
    x = G.to_device(a)
    y = G.empty_like_bytes(a)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.bmmc_permute(x, y, n, rows, c, 4, s)
    s.synchronize()
    assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c))


def test_host_threads_on_their_own_streams():
    """Four host threads call the library at once, each on a stream of its
    own, each with new matrices (plans made concurrently), both methods (the
    paper's scheme takes a scratch array per stream); every result checked."""
    import threading
    jobs = []
    for t in range(4):
        for k in range(12):
            n = 10 + (7 * t + 3 * k) % 9
            w = (4, 8)[(t + k) % 2]
            rows, c = gen.random_bmmc(n, 1000 * t + k)
            a = gen.data(n, w, 100 * t + k)
            jobs.append((t, n, w, rows, c, a, G.to_device(a), G.empty_like_bytes(a),
                         (B.METHOD_AUTO, B.METHOD_TILED)[k % 2]))
    G.sync()
    errors = []

    def work(t):
        try:
            s = torch.cuda.Stream()
            for (tt, n, w, rows, c, a, x, y, m) in jobs:
                if tt == t:
                    B.bmmc_permute_ex(x, y, n, rows, c, w, {"method": m}, s)
            s.synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for (t, n, w, rows, c, a, x, y, m) in jobs:
        assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c)), (t, n, w, m)


@pytest.mark.parametrize("method,per_call", [(B.METHOD_AUTO, 1), (B.METHOD_TILED, 2)])
def test_profile_reports_launches(method, per_call):
    n = 20
    rows, c = gen.random_bmmc(n, 9)
    a = gen.data(n, 4, 2)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    B.bmmc_profile_begin()
    for _ in range(3):
        B.bmmc_permute_ex(x, y, n, rows, c, 4, {"method": method}, G.stream())
    st = B.bmmc_profile_end()
    assert sum(v["launches"] for v in st.values()) == 3 * per_call
    assert all(v["total_ms"] > 0 for v in st.values())


@pytest.mark.parametrize("n,w", [(12, 4), (21, 4), (19, 8)])
def test_fused_sequence_equals_steps(n, w):
    """bmmc_permute_seq runs a fused sequence once; the oracle applies the
    steps one after the other."""
    seq = [gen.random_bmmc(n, 300 + k) for k in range(3)] + [(gen.bit_reversal_rows(n), 5)]
    a = gen.data(n, w, 12)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    B.bmmc_permute_seq(x, y, n, seq, w, G.stream())
    G.sync()
    want = a
    for rows, c in seq:
        want = O.permute(want, n, rows, c)
    assert np.array_equal(G.to_host(y, a), want)


def test_parm_split_and_merge_on_device():
    """parm mask f with f = reverse each half, built from two device BMMCs
    around a plain half reversal (Section 7.2), against the parm definition."""
    n, mask = 16, 0b1000100100010010
    rows, inv = B.bmmc_parm_matrix(mask, n)
    a = gen.data(n, 4, 21)
    x, t = G.to_device(a), G.empty_like_bytes(a)
    B.bmmc_permute(x, t, n, rows, 0, 4, G.stream())
    halves = t.view(torch.int32).view(2, -1).flip(1).contiguous().view(torch.uint8).view(-1)
    y = G.empty_like_bytes(a)
    B.bmmc_permute(halves, y, n, inv, 0, 4, G.stream())
    G.sync()
    sub = np.array([bin(v & mask).count("1") & 1 for v in range(1 << n)])
    want = a.copy()
    for s in (0, 1):
        idx = np.nonzero(sub == s)[0]
        want[idx] = a[idx][::-1]
    assert np.array_equal(G.to_host(y, a), want)


def test_permutes_captured_in_a_graph():
    """Library calls captured into a HIP graph (through torch's capture on the
    library's stream) and replayed with fresh inputs and eager work between
    replays: every replay equals the oracle."""
    n = 20
    cases = [(gen.bit_reversal_rows(n), 0), gen.random_bmmc(n, 41)]
    a = gen.data(n, 4, 0)
    x = G.to_device(a)
    ys = [G.empty_like_bytes(a) for _ in cases]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # plans made and kernels loaded before capture
        for (rows, c), y in zip(cases, ys):
            B.bmmc_permute(x, y, n, rows, c, 4, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream()
        for (rows, c), y in zip(cases, ys):
            B.bmmc_permute(x, y, n, rows, c, 4, cap)
    for rep in range(3):
        a = gen.data(n, 4, 100 + rep)
        x.copy_(torch.from_numpy(a.view(np.uint8)).to(G.dev()))
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (rows, c), y in zip(cases, ys):
            assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c)), rep


@pytest.mark.parametrize("n,w,method", [(32, 1, B.METHOD_AUTO), (32, 1, B.METHOD_TILED),
                                        (30, 4, B.METHOD_AUTO), (29, 8, B.METHOD_TILED)])
def test_maximum_sizes_sampled(n, w, method):
    """The largest index space (n = 32, 2^32 one-byte elements) and 4 GiB
    arrays of wider elements: 65536 sampled outputs, the first and last
    indices among them, against the oracle's index map."""
    print(f"max size n={n} w={w} method={method}", flush=True)
    rows, c = gen.random_bmmc(n, 3200 + n)
    g = torch.Generator(device="cuda")
    g.manual_seed(n * 10 + w)
    x = torch.randint(0, 256, ((1 << n) * w,), dtype=torch.uint8, device="cuda", generator=g)
    y = torch.empty_like(x)
    B.bmmc_permute_ex(x, y, n, rows, c, w, {"method": method}, G.stream())
    G.sync()
    rng = np.random.default_rng(n)
    xs = rng.integers(0, 1 << n, size=1 << 16, dtype=np.uint64)
    xs[:4] = [0, 1, (1 << n) - 2, (1 << n) - 1]
    ys = O.apply_many(rows, c, n, xs)
    xi = torch.from_numpy(xs.astype(np.int64)).to(G.dev())
    yi = torch.from_numpy(ys.astype(np.int64)).to(G.dev())
    assert torch.equal(y.view(-1, w)[yi], x.view(-1, w)[xi])
    del x, y
    torch.cuda.empty_cache()
