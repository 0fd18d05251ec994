"""Host logic of the GPU library, checked on the CPU (no device calls).

The library's planner and its host emulation of the kernels' addressing are
compared with the oracle (which shares no code with them): factor products,
the tiled condition, the paper's geometry examples, and full permutations run
lane by lane on the host.
"""
import json
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07795_amd import binding as B
from synth import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_examples.json")))


def header_functions():
    text = open(os.path.join(ROOT, "include", "bmmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bmmc_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 25
    L = B.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(B.exported_names())
    assert B.bmmc_version() >= 100


def test_strerror_and_errors():
    assert B.bmmc_strerror(0) == "ok"
    assert "singular" in B.bmmc_strerror(-2)
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_factorize([0b011, 0b110, 0b101], 0, 3)
    assert e.value.status == -2
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_factorize([1, 2, 1 << 5], 0, 3)  # bit beyond n
    assert e.value.status == -1
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_factorize(gen.identity_rows(3), 8, 3)  # complement bit beyond n
    assert e.value.status == -1
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_factorize(gen.identity_rows(33), 0, 33)
    assert e.value.status == -3
    with pytest.raises(B.BmmcError):
        B.bmmc_plan_ex(gen.identity_rows(4), 0, 4, 3)  # width 3
    # buffer validation happens before any device call
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_permute(0, 0, 4, gen.identity_rows(4), 0, 4)
    assert e.value.status == -1
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_permute(4096, 4096 + 32, 4, gen.identity_rows(4), 0, 4)  # overlap
    assert e.value.status == -4
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_permute(4096 + 4, 1 << 20, 4, gen.identity_rows(4), 0, 4)  # misaligned
    assert e.value.status == -1


def test_batched_validation_rejects_overlaps():
    rows = gen.identity_rows(4)
    base = 1 << 20
    ok = [(base, base + 4096, 4, 4, rows, 0), (base + 8192, base + 12288, 4, 4, rows, 0)]
    shared_input = [(base, base + 4096, 4, 4, rows, 0), (base, base + 8192, 4, 4, rows, 0)]
    clash = [(base, base + 4096, 4, 4, rows, 0), (base + 8192, base + 4096 + 16, 4, 4, rows, 0)]
    in_on_out = [(base, base + 4096, 4, 4, rows, 0), (base + 4096 + 32, base + 8192, 4, 4, rows, 0)]
    arr, keep, k = B.make_descs(clash)
    assert B.lib().bmmc_permute_batched(arr, k, None) == -4
    arr, keep, k = B.make_descs(in_on_out)
    assert B.lib().bmmc_permute_batched(arr, k, None) == -4
    # valid batches get past validation and then need a device (HIP error here)
    for items in (ok, shared_input):
        arr, keep, k = B.make_descs(items)
        assert B.lib().bmmc_permute_batched(arr, k, None) in (0, -6)
    # tile sizes other than 4, 8, 16 or 32 are refused before any device work
    for bad in (2, 12, 64):
        with pytest.raises(B.BmmcError) as e:
            B.bmmc_permute_batched(ok, None, {"iters": bad})
        assert e.value.status == -1


# ---------------------------------------------------------- tiled test

@pytest.mark.parametrize("n,seed", [(5, 0), (8, 1), (12, 2), (20, 3), (28, 4)])
def test_is_tiled_matches_oracle_definition(n, seed):
    mats = [gen.random_bmmc(n, seed)[0], gen.bit_reversal_rows(n), gen.block_swap_rows(n, n // 2),
            gen.random_bpc(n, seed)[0], gen.cyclic_shift_rows(n)]
    for rows in mats:
        m = O.dense(rows, n)
        for t in range(0, n + 1):
            ok, cols = O.is_tiled(m, t)
            got, mask = B.bmmc_is_tiled(rows, n, t)
            assert got == ok
            if ok:
                assert mask == cols


# ------------------------------------------------------- factorization

def check_ulp(rows, n):
    f = B.bmmc_factorize_ulp(rows, n)
    U, L, P = (O.dense(f[k], n) for k in ("U", "L", "P"))
    T1, T2 = O.dense(f["T1"], n), O.dense(f["T2"], n)
    A = O.dense(rows, n)
    R = O.dense(gen.bit_reversal_rows(n), n)
    assert np.array_equal(np.triu(U), U) and np.all(np.diag(U) == 1)
    assert np.array_equal(np.tril(L), L) and np.all(np.diag(L) == 1)
    assert np.all(P.sum(0) == 1) and np.all(P.sum(1) == 1)
    assert np.array_equal(O.mul(O.mul(U, L), P), A)
    assert np.array_equal(O.mul(U, R), T1)
    assert np.array_equal(O.mul(R, O.mul(L, P)), T2)
    assert np.array_equal(O.mul(T1, T2), A)
    for t in range(n + 1):
        ok1, cols1 = O.is_tiled(T1, t)
        ok2, _ = O.is_tiled(T2, t)
        assert ok1 and ok2
        assert cols1 == sum(1 << j for j in range(n - t, n))  # U.R on the top columns


@pytest.mark.parametrize("n", [1, 2, 3])
def test_ulp_brute_force_every_invertible_matrix(n):
    import itertools
    count = 0
    for rows in itertools.product(range(1 << n), repeat=n):
        if O.rank(O.dense(rows, n)) != n:
            continue
        count += 1
        check_ulp(list(rows), n)
    assert count == {1: 1, 2: 6, 3: 168}[n]


def test_ulp_n4_sample_of_all():
    import itertools
    seen = 0
    for k, rows in enumerate(itertools.product(range(16), repeat=4)):
        if k % 7:
            continue
        if O.rank(O.dense(rows, 4)) != 4:
            continue
        check_ulp(list(rows), 4)
        seen += 1
    assert seen > 2500


@pytest.mark.parametrize("n,seed", [(12, 1), (17, 2), (22, 3), (26, 4), (28, 5), (32, 6)])
def test_ulp_random(n, seed):
    check_ulp(gen.random_bmmc(n, seed)[0], n)


@pytest.mark.parametrize("n,seed,w", [(14, 1, 4), (20, 2, 4), (26, 0, 4), (28, 3, 4), (27, 4, 8), (24, 5, 16)])
def test_plan_factors(n, seed, w):
    """Planned factors compose to A, complement on the second, each tiled at t."""
    rows, c = gen.random_bmmc(n, seed)
    p = B.bmmc_factorize_t(rows, c, n, 0, w)
    assert p.nfactors == 2
    t = p.t
    (r0, c0), (r1, c1) = p.factor(0), p.factor(1)
    assert c0 == 0 and c1 == c
    T2, T1 = O.dense(r0, n), O.dense(r1, n)
    assert np.array_equal(O.mul(T1, T2), O.dense(rows, n))
    assert O.is_tiled(T1, t)[0] and O.is_tiled(T2, t)[0]
    for k in range(2):
        assert p.coordinate[k] == 1
        assert p.lds_conflict_score[k] == 0
        assert p.tile_bits[k] == {4: 12, 8: 12, 16: 11}[w]


def test_tiled_matrix_takes_one_pass():
    n = 20
    for rows in (gen.bit_reversal_rows(n), gen.block_swap_rows(n, 10), gen.random_bpc(n, 3)[0]):
        p = B.bmmc_factorize(rows, 5, n)
        assert p.nfactors == 1
        assert p.factor(0) == (rows, 5)


# ----------------------------------------------- geometry pins (paper values)

def pdep(value, mask):
    out, k = 0, 0
    for j in range(64):
        if (mask >> j) & 1:
            out |= ((value >> k) & 1) << j
            k += 1
    return out


def compress(index, mask):
    """Delete the bits of index outside mask (the stitch_tile_* view)."""
    out, k = 0, 0
    for j in range(64):
        if (mask >> j) & 1:
            out |= ((index >> j) & 1) << k
            k += 1
    return out


def test_stitch_examples_cyclic_shift():
    g = GOLDEN["stitch_cyclic_shift"]
    n, t = g["n"], g["t"]
    rows = gen.cyclic_shift_rows(n)
    # tile of exactly the paper's bits: 2t - n_over = 6 bits, no iterations
    p = B.bmmc_plan_ex(rows, 0, n, 16, {"t": t, "threads": 64, "iters": 1})
    assert p.nfactors == 1
    col, row, tb = p.col_mask[0], p.tile_rows_mask[0], p.tb_mask[0]
    assert p.n_over[0] == g["n_over"] and bin(tb).count("1") == g["n_tb"] and p.iter_mask[0] == 0
    assert col == (1 << t) - 1
    tile = col | row

    def stitch_col(c_, tb_, r_):
        return pdep(c_, col) | pdep(tb_, tb) | pdep(r_, row & ~col)

    def stitch_row(c_, tb_, r_):
        return pdep(r_, row) | pdep(tb_, tb) | pdep(c_, col & ~row)

    for ex in g["examples"]:
        b = lambda s: int(s, 2)
        if ex["fn"] == "stitch_col":
            got = stitch_col(b(ex["col"]), b(ex["tb"]), b(ex["row"]))
        elif ex["fn"] == "stitch_row":
            got = stitch_row(b(ex["col"]), b(ex["tb"]), b(ex["row"]))
        elif ex["fn"] == "stitch_tile_col":
            got = compress(stitch_col(b(ex["col"]), 0, b(ex["row"])), tile)
        else:
            got = compress(stitch_row(b(ex["col"]), 0, b(ex["row"])), tile)
        assert got == b(ex["result"]), ex


def test_appendix_geometry_bit_reverse():
    g = GOLDEN["appendix_bitrev15"]
    n, t = g["n"], g["t"]
    rows = gen.bit_reversal_rows(n)
    bits = lambda m: [j for j in range(n) if (m >> j) & 1]
    # tile of 2^10 = 1024 elements (no iteration bits)
    p = B.bmmc_plan_ex(rows, 0, n, 16, {"t": t, "threads": 1024, "iters": 1})
    assert bits(p.col_mask[0]) == g["col_bits"]
    assert bits(p.tile_rows_mask[0]) == g["row_bits"]
    assert bits(p.tb_mask[0]) == g["tb_bits"]
    assert p.n_over[0] == g["n_over"]
    assert 2 ** bin(p.tb_mask[0]).count("1") == g["blocks"]
    assert 2 ** p.tile_bits[0] == g["tile_elems"]
    # n_iter = 3: tile of 2^13 = 8192 elements
    it = g["iters"]
    p = B.bmmc_plan_ex(rows, 0, n, 16, {"t": t, "threads": 1024, "iters": 8})
    assert bits(p.iter_mask[0]) == it["iter_bits"]
    assert bits(p.tb_mask[0]) == it["tb_bits"]
    assert 2 ** bin(p.tb_mask[0]).count("1") == it["blocks"]
    assert 2 ** p.tile_bits[0] == it["tile_elems"]


# ------------------------------------------- host emulation vs the oracle

def emulate_check(n, rows, c, w, opts=None, data_seed=1):
    a = gen.data(n, w, data_seed)
    out = np.zeros_like(a)
    st = B.bmmc_emulate(a, out, n, rows, c, w, opts)
    assert np.array_equal(out, O.permute(a, n, rows, c))
    assert st["lds_slot_errors"] == 0
    return st


CASES = [
    ("random", lambda n, s: gen.random_bmmc(n, s)),
    ("bitrev", lambda n, s: (gen.bit_reversal_rows(n), 0)),
    ("swap", lambda n, s: (gen.block_swap_rows(n, n // 2), 0)),
    ("bpc", lambda n, s: gen.random_bpc(n, s)),
    ("cyclic", lambda n, s: (gen.cyclic_shift_rows(n), 1)),
    ("reverse", lambda n, s: (gen.identity_rows(n), (1 << n) - 1)),
]


@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n", [3, 8, 12, 13, 16, 18])
@pytest.mark.parametrize("w", [4, 8])
def test_emulation_matches_oracle(name, mk, n, w, method):
    rows, c = mk(n, n * 13 + w)
    st = emulate_check(n, rows, c, w, {"method": method})
    if n >= 8:
        # every wave access is one run of whole lines, and conflict-free LDS
        assert st["read_lines"] == st["read_lines_min"]
        assert st["write_lines"] == st["write_lines_min"]
        assert st["lds_conflicts32"] == 0 and st["lds_conflicts64"] == 0


@pytest.mark.parametrize("w", [1, 2, 16])
@pytest.mark.parametrize("n", [2, 5, 11, 15, 17])
def test_emulation_other_widths(w, n):
    rows, c = gen.random_bmmc(n, 100 + n)
    emulate_check(n, rows, c, w)


@pytest.mark.parametrize("method", [B.METHOD_ONEPASS, B.METHOD_NAIVE])
@pytest.mark.parametrize("n", [9, 14, 17])
def test_emulation_methods(method, n):
    rows, c = gen.random_bmmc(n, 7 * n)
    st = emulate_check(n, rows, c, 4, {"method": method})
    if method == B.METHOD_ONEPASS and n >= 13:
        d = B.bmmc_plan_ex(rows, c, n, 4, {"method": method}).tile_bits[0]
        assert st["tiles"] == 2 ** (n - d)  # one pass over all tiles
        assert st["read_lines"] == st["read_lines_min"]
        assert st["lds_conflicts64"] == 0


@pytest.mark.parametrize("opts", [
    {"threads": 512, "iters": 4}, {"threads": 1024, "iters": 2}, {"threads": 256, "iters": 8},
    {"threads": 256, "iters": 2}, {"t": 5}, {"t": 4, "threads": 256, "iters": 2},
    {"swizzle": -1}, {"threads": 256, "iters": 16, "t": 7},
    {"run_in": 7, "run_out": 5}, {"run_in": 5, "run_out": 7}, {"threads": 512, "run_in": 7, "run_out": 6},
    {"tile_order": 2}, {"tile_order": 3, "run_in": 7, "run_out": 5},
    {"tile_order": 10, "threads": 512, "iters": 8}, {"tile_order": 12, "threads": 1024, "iters": 4, "t": 6},
])
def test_emulation_shapes(opts):
    n = 17
    rows, c = gen.random_bmmc(n, 5)
    st = emulate_check(n, rows, c, 4, opts)
    if opts.get("swizzle", 0) >= 0:
        assert st["lds_conflicts64"] == 0


@pytest.mark.parametrize("order", [4 + 16, 1 + 16 * 6, 2 + 16 * 3, 4 + 16 * 15, 256 + 4, 256 + 4 + 16 * 7])
@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
@pytest.mark.parametrize("name,mk", [c for c in CASES if c[0] in ("random", "bitrev", "swap", "bpc")],
                         ids=["random", "bitrev", "swap", "bpc"])
@pytest.mark.parametrize("w", [4, 8])
def test_emulation_output_ordered_tiles(name, mk, w, method, order):
    """Tiles selected so that neighbouring tiles write neighbouring runs (or,
    with 256 added, each tile writes 4 KiB blocks of one class): the same
    permutation, every tile still reading and writing whole lines."""
    n = 17
    rows, c = mk(n, 3 * n + w)
    st = emulate_check(n, rows, c, w, {"method": method, "tile_order": order})
    assert st["read_lines"] == st["read_lines_min"]
    assert st["write_lines"] == st["write_lines_min"]


@pytest.mark.parametrize("order", [4 + 16 * 3, 4 + 16 * 15, 2 + 16 * 15, 256 + 4])
@pytest.mark.parametrize("n", [9, 12, 13, 14, 15])
def test_output_ordered_tiles_with_few_tile_bits(n, order):
    """k beyond the number of tile-selecting bits (the whole array in one
    tile, or one or two tiles) is clamped to what there is."""
    for rows, c in (gen.random_bmmc(n, 5 * n), (gen.bit_reversal_rows(n), 1)):
        st = emulate_check(n, rows, c, 4, {"tile_order": order})
        assert st["read_lines"] == st["read_lines_min"] and st["write_lines"] == st["write_lines_min"]


@pytest.mark.parametrize("w", [4, 8])
def test_dealt_output_blocks(w):
    """tile_order + 256: where no tile vector moves the output's 4 KiB-block
    bits (bit reversal, a transpose whose read runs land above those bits,
    the identity with any c), every tile writes blocks of one class, the
    class of tile t being t XOR k mod 8; where the matrix does not allow it
    (a random matrix, a transpose whose read runs land on those bits) the
    plan falls back to the plain choice.  Either way the same permutation."""
    n = 20
    cases = {"bitrev": (gen.bit_reversal_rows(n), 0), "swap7": (gen.block_swap_rows(n, 7), 0),
             "identity": (gen.identity_rows(n), 0x5A5A5), "swap_half": (gen.block_swap_rows(n, n // 2), 0),
             "random": gen.random_bmmc(n, 11)}
    for name, (rows, c) in cases.items():
        opts = {"threads": 256, "iters": 4}
        plain = emulate_check(n, rows, c, w, dict(opts, tile_order=4))
        dealt = emulate_check(n, rows, c, w, dict(opts, tile_order=256 + 4))
        assert dealt["write_lines"] == dealt["write_lines_min"]
        if name in ("bitrev", "swap7", "identity"):
            assert dealt["dealt_write_tiles"] == dealt["tiles"], name
            if name != "identity":
                assert plain["dealt_write_tiles"] < plain["tiles"], name
        else:
            # the read runs' images cover the block bits: the plain choice
            assert dealt["dealt_write_tiles"] == plain["dealt_write_tiles"], name


@pytest.mark.parametrize("w", [1, 2, 16])
def test_dealt_output_blocks_other_widths(w):
    """Dealt output blocks with 1-, 2- and 16-byte elements (the block bits
    sit 12 - log2(w) bits up): the reversal is dealt in every tile, and the
    permutation is exact for it, the bit reversal and a random matrix."""
    n = 18
    for name, (rows, c) in {"reverse": (gen.identity_rows(n), (1 << n) - 1),
                            "bitrev": (gen.bit_reversal_rows(n), 0),
                            "random": gen.random_bmmc(n, 3)}.items():
        st = emulate_check(n, rows, c, w, {"tile_order": 256 + 4})
        if name == "reverse":
            assert st["dealt_write_tiles"] == st["tiles"]


@pytest.mark.parametrize("n,w,a,d", [
    (21, 4, 6, 13),   # 8 MiB: the general tile's own default
    (22, 4, 5, 13),   # 16 MiB: 256 x 8 vectors, 2^5-element reads
    (24, 4, 6, 14),   # 64 MiB: 512 x 8
    (27, 4, 6, 14),   # 512 MiB: 1024 x 4
    (20, 8, 7, 12),   # 8 MiB
    (21, 8, 7, 12),   # 16 MiB: 256 x 8
    (23, 8, 5, 13),   # 64 MiB: 1024 x 4
    (26, 8, 5, 13),   # 512 MiB
])
def test_size_dependent_defaults(n, w, a, d):
    rows, c = gen.random_bmmc(n, 11)
    p = B.bmmc_plan_ex(rows, c, n, w, None)
    assert p.nfactors == 1 and p.tile_bits[0] == d
    assert bin(p.col_mask[0]).count("1") == a
    # given runs keep the general tile's default shape (2^13 4-byte elements)
    q = B.bmmc_plan_ex(rows, c, n, w, {"run_in": 7, "run_out": 5})
    assert bin(q.col_mask[0]).count("1") == 7
    assert q.tile_bits[0] == (13 if w == 4 else 12)


def test_auto_takes_one_pass_and_tiled_the_papers_two():
    """Auto: one pass for every A (a tiled pass, or one general tile);
    the tiled method: the paper's factorization, two passes unless A is tiled."""
    for n, w in [(14, 4), (20, 4), (26, 4), (27, 8), (24, 16), (20, 1), (20, 2)]:
        rows, c = gen.random_bmmc(n, n + w)
        auto = B.bmmc_plan_ex(rows, c, n, w, None)
        assert auto.nfactors == 1 and auto.coordinate[0] == 0
        tiled = B.bmmc_plan_ex(rows, c, n, w, {"method": B.METHOD_TILED})
        assert tiled.nfactors == 2 and tiled.coordinate[0] == 1 and tiled.coordinate[1] == 1
        assert B.bmmc_factorize(rows, c, n).nfactors == 2
        br = gen.bit_reversal_rows(n)
        for m in (B.METHOD_AUTO, B.METHOD_TILED):
            p = B.bmmc_plan_ex(br, 0, n, w, {"method": m})
            assert p.nfactors == 1 and p.coordinate[0] == 1


def test_emulation_iota_two_pass_n20():
    n = 20
    rows, c = gen.random_bmmc(n, 20)
    a = gen.iota(n, 4)
    out = np.zeros_like(a)
    st = B.bmmc_emulate(a, out, n, rows, c, 4, {"method": B.METHOD_TILED})
    assert st["tiles"] == 2 * 2 ** (n - 12)
    ys = O.index_map(rows, c, n)
    assert np.array_equal(out[ys.astype(np.int64)], a)


def test_plain_layout_has_conflicts_that_the_swizzle_removes():
    n = 16
    rows = gen.bit_reversal_rows(n)
    a = gen.data(n, 4, 0)
    out = np.zeros_like(a)
    plain = B.bmmc_emulate(a, out, n, rows, 0, 4, {"swizzle": -1})
    swz = B.bmmc_emulate(a, out, n, rows, 0, 4)
    assert plain["lds_conflicts32"] > 0
    assert swz["lds_conflicts32"] == 0 and swz["lds_conflicts64"] == 0


def test_tune_cache_classes_round_trip(tmp_path):
    """Tuned options are kept per matrix class (tiled or not) and survive a
    save / load; lookups pick the class of the matrix.  Sizes no other test
    tunes, so the process-wide cache is not disturbed."""
    n, w = 31, 2
    rnd, _ = gen.random_bmmc(n, 3)
    bpc, _ = gen.random_bpc(n, 4)
    assert B.bmmc_tune_lookup(n, w, rnd) is None
    path = tmp_path / "tune.jsonl"
    lines = [
        '{"kind": "plain", "n": 31, "w": 2, "method": 0, "class": 0, "used": 0, "threads": 512, "iters": 4, '
        '"t": 6, "run_in": 7, "run_out": 6, "hints": 2, "tile_order": 4, "grid": 0, "swizzle": 1, "ms": 1.5}',
        '{"kind": "plain", "n": 31, "w": 2, "method": 0, "class": 1, "used": 1, "threads": 256, "iters": 2, '
        '"t": 6, "run_in": 6, "run_out": 6, "hints": 3, "tile_order": 2, "grid": 0, "swizzle": 1, "ms": 1.25}',
    ]
    path.write_text("\n".join(lines) + "\n")
    assert B.bmmc_tune_load(str(path)) == 2
    g = B.bmmc_tune_lookup(n, w, rnd)
    assert (g["method"], g["threads"], g["run_in"], g["hints"]) == (0, 512, 7, 2)
    t = B.bmmc_tune_lookup(n, w, bpc)
    assert (t["method"], t["threads"], t["iters"], t["tile_order"]) == (1, 256, 2, 2)
    assert B.bmmc_tune_lookup(n, w, rnd, B.METHOD_TILED) is None
    out = tmp_path / "again.jsonl"
    B.bmmc_tune_save(str(out))
    saved = [l for l in out.read_text().splitlines() if '"n": 31, "w": 2' in l]
    assert len(saved) == 2 and '"class": 1, "used": 1' in saved[1]


def test_tune_cache_batch_lines_with_and_without_tile_order(tmp_path):
    """Batch entries load with cache hints and a tile order, in the older
    form without hints (hints 0), and in the oldest without a tile order
    (tile order 0); they are saved with both."""
    path = tmp_path / "batch.jsonl"
    lines = [
        '{"kind": "batch", "sig": "00000000000000a1", "workgroups": 512, "chunk_tiles": 2, "order": 0, '
        '"method": 0, "iters": 8, "tile_order": 116, "ms": 0.5}',
        '{"kind": "batch", "sig": "00000000000000a2", "workgroups": 1024, "chunk_tiles": 4, "order": 1, '
        '"method": 1, "iters": 4, "ms": 0.75}',
        '{"kind": "batch", "sig": "00000000000000a3", "workgroups": 256, "chunk_tiles": 1, "order": 0, '
        '"method": 0, "iters": 32, "tile_order": 2, "hints": 1, "ms": 0.25}',
    ]
    path.write_text("\n".join(lines) + "\n")
    assert B.bmmc_tune_load(str(path)) == 3
    out = tmp_path / "again.jsonl"
    B.bmmc_tune_save(str(out))
    saved = {l.split('"sig": "')[1][:16]: l for l in out.read_text().splitlines() if '"kind": "batch"' in l}
    assert '"tile_order": 116, "hints": 0' in saved["00000000000000a1"]
    assert '"tile_order": 0' in saved["00000000000000a2"] and '"chunk_tiles": 4' in saved["00000000000000a2"]
    assert '"tile_order": 2, "hints": 1' in saved["00000000000000a3"] and '"iters": 32' in saved["00000000000000a3"]


def test_tile_order_range_checked_when_planning():
    """Tile orders run from 0 to 511 (bit 8: dealt output blocks); planning
    refuses others with an argument error."""
    rows, c = gen.random_bmmc(14, 2)
    assert B.bmmc_plan_ex(rows, c, 14, 4, {"tile_order": 256 + 4}).nfactors == 1
    for bad in (-1, 512):
        with pytest.raises(B.BmmcError, match="tile_order"):
            B.bmmc_plan_ex(rows, c, 14, 4, {"tile_order": bad})


def test_batch_options_validated():
    """Options are checked before any device work (addresses are never
    dereferenced: the call fails first)."""
    rows, c = gen.random_bmmc(12, 1)
    item = (1 << 32, (1 << 32) + (1 << 20), 12, 4, rows, c)
    with pytest.raises(B.BmmcError, match="tile_order"):
        B.bmmc_permute_batched([item], None, {"tile_order": 512})
    with pytest.raises(B.BmmcError, match="iters"):
        B.bmmc_permute_batched([item], None, {"iters": 2})


def test_noalloc_batch_options_validated():
    """The allocation-free batched call checks its options before any device
    work: the two-pass method (whose scratch would have to be allocated) and
    bad knobs are refused, and its fixed table has the stated size."""
    rows, c = gen.random_bmmc(12, 1)
    item = (1 << 32, (1 << 32) + (1 << 20), 12, 4, rows, c)
    assert B.bmmc_noalloc_table_bytes() == 4 << 20
    with pytest.raises(B.BmmcError, match="TILED"):
        B.bmmc_permute_batched_noalloc([item], None, {"method": B.METHOD_TILED})
    with pytest.raises(B.BmmcError, match="iters"):
        B.bmmc_permute_batched_noalloc([item], None, {"iters": 2})
    with pytest.raises(B.BmmcError, match="tile_order"):
        B.bmmc_permute_batched_noalloc([item], None, {"tile_order": 512})
    B.bmmc_permute_batched_noalloc([], None)  # an empty batch is a no-op


@pytest.mark.skipif("BMMC_TUNE_CACHE" in os.environ, reason="another tuning file is named")
def test_packaged_tuning_results_are_loaded():
    """The library starts from its shipped gfx950 tuning results: the default
    workload's sizes have options for both matrix classes."""
    import json
    path = os.path.join(os.path.dirname(B.LIB_PATH), "tuning", "gfx950.jsonl")
    entries = [json.loads(l) for l in open(path) if l.strip()]
    assert any(e["kind"] == "plain" and e["n"] == 26 and e["w"] == 4 for e in entries)
    rnd = B.bmmc_tune_lookup(26, 4, gen.random_bmmc(26, 0)[0])
    bpc = B.bmmc_tune_lookup(26, 4, gen.bit_reversal_rows(26))
    assert rnd is not None and bpc is not None
    want = [e for e in entries if e["kind"] == "plain" and (e["n"], e["w"], e["method"], e["class"]) == (26, 4, 0, 0)][0]
    assert (rnd["threads"], rnd["iters"], rnd["run_in"], rnd["run_out"]) == \
        (want["threads"], want["iters"], want["run_in"], want["run_out"])


def test_header_is_plain_c_and_links(tmp_path):
    """include/bmmc.h compiles as C99 (no C++ or HIP types in the boundary) and
    a C program that calls host-only entry points links against the library."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include "bmmc.h"
int main(void) {
    uint64_t rows[4] = {8, 4, 2, 1};  /* bit reversal of 4 bits */
    bmmc_plan_t plan;
    if (bmmc_factorize(rows, 0, 4, &plan) != BMMC_OK) return 1;
    if (plan.nfactors != 1) return 2;
    uint64_t rows2[2] = {3, 3};
    if (bmmc_invert(rows2, 0, 2, rows2, &rows2[0]) != BMMC_ERR_SINGULAR) return 3;
    printf("%s\n", bmmc_strerror(BMMC_ERR_SINGULAR));
    return 0;
}
''')
    exe = tmp_path / "use"
    libdir = os.path.dirname(B.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe),
                        "-L", libdir, "-lbmmc", "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and "singular" in r.stdout
