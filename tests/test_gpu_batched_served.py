"""Batched and served forms on the GPU against the oracle, through the C ABI.

Each array's output must equal the oracle's, bit for bit, whether it runs in
one batched persistent launch, through graph replays, alone, or mixed with
other requests in the continuous-batching server.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_07795_amd import binding as B
from synth import gen
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def make_batch(sizes, widths, seed):
    arrays = []
    for k, (n, w) in enumerate(zip(sizes, widths)):
        rows, c = gen.random_bmmc(n, seed * 10007 + k)
        a = gen.data(n, w, seed * 10007 + k)
        arrays.append({"n": n, "w": w, "rows": rows, "c": c, "a": a,
                       "x": G.to_device(a), "y": G.empty_like_bytes(a)})
    return arrays


def items(arrays):
    return [(ar["x"], ar["y"], ar["n"], ar["w"], ar["rows"], ar["c"]) for ar in arrays]


def check_all(arrays):
    for k, ar in enumerate(arrays):
        got = G.to_host(ar["y"], ar["a"])
        want = O.permute(ar["a"], ar["n"], ar["rows"], ar["c"])
        assert np.array_equal(got, want), f"array {k}: n={ar['n']} w={ar['w']}"


@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
@pytest.mark.parametrize("use_graph", [1, -1])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("hints", [0, 3, 4])
def test_batched_mixed_sizes_and_widths(order, use_graph, hints, method):
    rng = np.random.default_rng(order)
    sizes = [int(v) for v in rng.integers(0, 19, size=48)]
    widths = [int(v) for v in rng.choice([4, 8, 16, 1, 2], size=48)]
    arrays = make_batch(sizes, widths, 3 + order)
    B.bmmc_permute_batched(items(arrays), G.stream(),
                           {"order": order, "use_graph": use_graph, "chunk_tiles": 1 + 2 * order,
                            "hints": hints, "method": method})
    G.sync()
    check_all(arrays)


@pytest.mark.parametrize("tile_order", [0, 2, 4 + 16 * 7])
@pytest.mark.parametrize("iters", [4, 8, 16, 32])
@pytest.mark.parametrize("chunk", [1, 4, 16])
def test_batched_chunks_and_grid(chunk, iters, tile_order):
    sizes = gen.batched_sizes(40, chunk, 10, 20)
    arrays = make_batch(sizes, [4, 8, 16, 4] * (len(sizes) // 4), chunk)
    B.bmmc_permute_batched(items(arrays), G.stream(), {"chunk_tiles": chunk, "workgroups": 64, "iters": iters,
                                                       "tile_order": tile_order})
    G.sync()
    check_all(arrays)


def test_batched_untuned_large_batch_defaults():
    """A batch of 512 MiB with no tuned entry and no options takes the
    128 KiB tiles (one per item); every array still bit-exact."""
    sizes = [22] * 8 + [21] * 8 + [23] * 8
    widths = [4] * 8 + [8] * 8 + [4] * 8
    arrays = make_batch(sizes, widths, 17)
    assert B.bmmc_tune_lookup_batched(items(arrays)) is None
    B.bmmc_permute_batched(items(arrays), G.stream())
    G.sync()
    check_all(arrays)


def test_batched_onepass_method():
    sizes = gen.batched_sizes(32, 9, 10, 21)
    arrays = make_batch(sizes, [4, 8] * 16, 9)
    B.bmmc_permute_batched(items(arrays), G.stream(), {"method": B.METHOD_ONEPASS})
    G.sync()
    check_all(arrays)


def test_graph_replays_with_fresh_data():
    """The same batch shape replayed from the cached graph, with new inputs
    and eager work in between; every replay is checked."""
    sizes = gen.batched_sizes(24, 5, 10, 19)
    arrays = make_batch(sizes, [4] * len(sizes), 5)
    for rep in range(4):
        for k, ar in enumerate(arrays):
            ar["a"] = gen.data(ar["n"], 4, 1000 * rep + k)
            ar["x"].copy_(torch.from_numpy(ar["a"].view(np.uint8)).to(G.dev()))
            ar["y"].zero_()
        torch.cuda.synchronize()
        B.bmmc_permute_batched(items(arrays), G.stream())
        G.sync()
        check_all(arrays)


def workload_batch():
    """The benchmark's batch: 1024 arrays, n uniform in [10, 22], int32, each
    with its own A and c (the benchmark's matrix seeds) and data of its own."""
    sizes = gen.batched_sizes(1024, 0, 10, 22)
    arrays = []
    for k, n in enumerate(sizes):
        rows, c = gen.random_bmmc(n, 1_000_003 + k)
        a = gen.data(n, 4, k)
        arrays.append({"n": n, "w": 4, "rows": rows, "c": c, "a": a,
                       "x": G.to_device(a), "y": G.empty_like_bytes(a)})
    return arrays


@pytest.mark.parametrize("iters", [4, 8, 16, 32])
@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_batch_of_1024_like_the_workload(method, iters):
    """The batched workload in every tile size and both methods: every one
    of the 1024 arrays compared in full."""
    arrays = workload_batch()
    B.bmmc_permute_batched(items(arrays), G.stream(), {"method": method, "iters": iters})
    G.sync()
    check_all(arrays)


def test_batch_of_1024_as_the_benchmark_runs_it():
    """The benchmark's calls on its batch: a resident batch with the tuned
    options of the tuning file (replayed twice with new data in between) and
    the one-shot batched call without options; every array in full."""
    arrays = workload_batch()
    tuned = B.bmmc_tune_lookup_batched(items(arrays))
    assert tuned is not None, "the tuning file has an entry for the benchmark's batch"
    pb = B.bmmc_batch_create(items(arrays), tuned)
    try:
        for rep in range(2):
            if rep:
                for k, ar in enumerate(arrays):
                    ar["a"] = gen.data(ar["n"], 4, 5000 + k)
                    ar["x"].copy_(torch.from_numpy(ar["a"].view(np.uint8)).to(G.dev()))
                    ar["y"].zero_()
                torch.cuda.synchronize()
            pb.launch(G.stream())
            G.sync()
            check_all(arrays)
    finally:
        pb.close()
    for ar in arrays:
        ar["y"].zero_()
    B.bmmc_permute_batched(items(arrays), G.stream())
    G.sync()
    check_all(arrays)


def test_batched_equals_separate_calls():
    sizes = gen.batched_sizes(16, 2, 12, 20)
    arrays = make_batch(sizes, [8] * 16, 2)
    B.bmmc_permute_batched(items(arrays), G.stream())
    torch.cuda.synchronize()
    for ar in arrays:
        z = G.empty_like_bytes(ar["a"])
        B.bmmc_permute(ar["x"], z, ar["n"], ar["rows"], ar["c"], ar["w"], G.stream())
        torch.cuda.synchronize()
        assert torch.equal(z, ar["y"])


def test_autotune_small_then_permute():
    opts, ms = B.bmmc_autotune(18, 4, B.METHOD_AUTO, G.stream(), 2)
    assert ms > 0 and opts["threads"] in (256, 512, 1024)
    a = gen.data(18, 4, 4)
    for rows, c in (gen.random_bmmc(18, 4), (gen.bit_reversal_rows(18), 3)):
        assert B.bmmc_tune_lookup(18, 4, rows) is not None  # each class tuned
        x, y = G.to_device(a), G.empty_like_bytes(a)
        B.bmmc_permute(x, y, 18, rows, c, 4, G.stream())  # now uses the tuned options
        G.sync()
        assert np.array_equal(G.to_host(y, a), O.permute(a, 18, rows, c))


def test_autotune_tiled_method_small():
    """The paper's two-pass scheme tuned below 64 MiB (its candidates timed as
    graph replays, scratch made before the capture); the tuned options then
    permute correctly."""
    n = 17
    opts, ms = B.bmmc_autotune(n, 8, B.METHOD_TILED, G.stream(), 2)
    assert ms > 0
    rows, c = gen.random_bmmc(n, 12)
    tuned = B.bmmc_tune_lookup(n, 8, rows, B.METHOD_TILED)
    assert tuned is not None and tuned["method"] == B.METHOD_TILED
    a = gen.data(n, 8, 12)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    B.bmmc_permute_ex(x, y, n, rows, c, 8, tuned, G.stream())
    G.sync()
    assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c))


def test_autotune_batched_small():
    sizes = gen.batched_sizes(20, 11, 10, 16)
    arrays = make_batch(sizes, [4] * 20, 11)
    opts, ms = B.bmmc_autotune_batched(items(arrays), G.stream(), 1)
    assert ms > 0 and opts["chunk_tiles"] >= 1
    for ar in arrays:
        ar["y"].zero_()
    B.bmmc_permute_batched(items(arrays), G.stream())  # tuned options
    G.sync()
    check_all(arrays)


@pytest.mark.parametrize("n,w", [(3, 4), (13, 16), (20, 4), (23, 8)])
def test_autotune_matrix_then_permute(n, w):
    """Per-matrix tuning (graph-timed below 64 MiB, plainly from 64 MiB):
    its output is the permutation, the setting is what later calls of this
    matrix use, they stay bit-exact, and clearing falls back to the class."""
    rows, c = gen.random_bmmc(n, 21)
    a = gen.data(n, w, 21)
    want = O.permute(a, n, rows, c)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    try:
        opts, ms = B.bmmc_autotune_matrix(x, y, n, rows, c, w, G.stream(), 2)
        G.sync()
        assert ms > 0 and np.array_equal(G.to_host(y, a), want)
        assert B.bmmc_tune_lookup(n, w, rows) == opts
        y.zero_()
        B.bmmc_permute(x, y, n, rows, c ^ 1, w, G.stream())  # same A, other c: same setting
        G.sync()
        assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c ^ 1))
    finally:
        B.bmmc_tune_clear_matrices()
    after = B.bmmc_tune_lookup(n, w, rows)
    assert after is None or after == B.bmmc_tune_lookup(n, w, gen.random_bmmc(n, 22)[0])


def test_autotune_matrix_errors():
    n, w = 12, 4
    a = gen.data(n, w, 3)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    singular = [1] * n
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_autotune_matrix(x, y, n, singular, 0, w, G.stream(), 1)
    assert e.value.status == -2
    r3 = gen.random_bmmc(n, 3)[0]
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_autotune_matrix(x, x, n, r3, 0, w, G.stream(), 1)
    assert e.value.status == -4
    # nothing stored for the matrix whose tuning failed: it gets its class's
    assert B.bmmc_tune_lookup(n, w, r3) == B.bmmc_tune_lookup(n, w, gen.random_bmmc(n, 4)[0])


# ------------------------------------------------------------------ server

@pytest.mark.parametrize("solo_log2", [0, 16, -1])
@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_server_mix_equals_alone_equals_oracle(method, use_graph, solo_log2):
    """solo_log2 16: requests of 64 KiB and more are planned as single-array
    calls (their own launches, tuned options) beside batched small ones."""
    reqs = gen.poisson_requests(60, 20000.0, 7, n_lo=8, n_hi=20)
    pool = {}
    srv = B.bmmc_server_create(1 << 30, streams=3, own_outputs=True, method=method, use_graph=use_graph,
                               solo_log2=solo_log2)
    try:
        t0 = B.bmmc_server_now_ns() + 2_000_000
        tickets = []
        for r in reqs:
            rows, c = gen.random_bmmc(r["n"], r["seed"])
            a = gen.data(r["n"], r["w"], r["seed"])
            x = G.to_device(a)
            pool[r["id"]] = (rows, c, a, x)
            tickets.append(B.bmmc_server_submit(srv, x, 0, r["n"], rows, c, r["w"],
                                                t0 + int(r["arrival"] * 1e9)))
        torch.cuda.synchronize()
        B.bmmc_server_drain(srv)
        mixed = {}
        for r, tk in zip(reqs, tickets):
            done, out = B.bmmc_server_poll(srv, tk)
            rows, c, a, x = pool[r["id"]]
            y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
            B.bmmc_copy(out, y, a.nbytes, G.stream())
            G.sync()
            got = G.to_host(y, a)
            assert np.array_equal(got, O.permute(a, r["n"], rows, c)), r
            mixed[r["id"]] = got
            B.bmmc_server_release(srv, tk)
        st = B.bmmc_server_stats(srv)
        assert st["completed"] == len(reqs) and st["rejected"] == 0
        assert st["p99_ms"] >= st["p50_ms"] > 0
    finally:
        B.bmmc_server_destroy(srv)
    # the same requests alone, one server each time
    srv = B.bmmc_server_create(1 << 28, streams=1, own_outputs=True, method=method)
    try:
        for r in reqs[:12]:
            rows, c, a, x = pool[r["id"]]
            tk = B.bmmc_server_submit(srv, x, 0, r["n"], rows, c, r["w"])
            done, out = B.bmmc_server_poll(srv, tk, wait=True)
            y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
            B.bmmc_copy(out, y, a.nbytes, G.stream())
            G.sync()
            assert np.array_equal(G.to_host(y, a), mixed[r["id"]])
            B.bmmc_server_release(srv, tk)
    finally:
        B.bmmc_server_destroy(srv)


@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_server_budget_admission_and_caller_outputs(method):
    """A budget that admits one large request at a time still completes all,
    in order; outputs provided by the caller."""
    n, w = 20, 4
    srv = B.bmmc_server_create(3 * (1 << n) * w + (1 << 20), streams=2, own_outputs=False,
                               method=method)
    try:
        work = []
        for k in range(6):
            rows, c = gen.random_bmmc(n, 50 + k)
            a = gen.data(n, w, 50 + k)
            x, y = G.to_device(a), G.empty_like_bytes(a)
            torch.cuda.synchronize()
            tk = B.bmmc_server_submit(srv, x, y, n, rows, c, w)
            work.append((tk, rows, c, a, x, y))
        B.bmmc_server_drain(srv)
        for tk, rows, c, a, x, y in work:
            B.bmmc_server_poll(srv, tk)
            assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c))
            B.bmmc_server_release(srv, tk)
        st = B.bmmc_server_stats(srv)
        assert st["peak_bytes"] <= 3 * (1 << n) * w + (1 << 20)
        with pytest.raises(B.BmmcError):  # can never fit
            B.bmmc_server_submit(srv, work[0][4], work[0][5], 22, gen.identity_rows(22), 0, 4)
    finally:
        B.bmmc_server_destroy(srv)


@pytest.mark.parametrize("iters", [4, 8, 16, 32])
@pytest.mark.parametrize("method", [B.METHOD_AUTO, B.METHOD_TILED])
def test_prepared_batch_replays(method, iters):
    """A resident batch (plans, table, scratch and graph made once) replayed
    with fresh inputs each time; every array checked each time."""
    rng = np.random.default_rng(31)
    sizes = [int(v) for v in rng.integers(0, 21, size=40)]
    widths = [int(v) for v in rng.choice([4, 8, 16, 2], size=40)]
    arrays = make_batch(sizes, widths, 31)
    pb = B.bmmc_batch_create(items(arrays), {"method": method, "iters": iters})
    try:
        for rep in range(3):
            for k, ar in enumerate(arrays):
                ar["a"] = gen.data(ar["n"], ar["w"], 500 * rep + k)
                ar["x"].copy_(torch.from_numpy(ar["a"].view(np.uint8).reshape(-1)).to(G.dev()))
                ar["y"].zero_()
            torch.cuda.synchronize()
            pb.launch(G.stream())
            G.sync()
            check_all(arrays)
    finally:
        pb.close()


def test_server_submit_many_in_arrival_order():
    """Requests marshalled once and submitted together, each with its own
    future arrival time, come out right."""
    reqs = gen.poisson_requests(24, 20000.0, 17, n_lo=10, n_hi=18)
    pool, items = {}, []
    for r in reqs:
        rows, c = gen.random_bmmc(r["n"], r["seed"])
        a = gen.data(r["n"], r["w"], r["seed"])
        x = G.to_device(a)
        pool[r["id"]] = (rows, c, a, x)
        items.append((x, None, r["n"], r["w"], rows, c))
    srv = B.bmmc_server_create(1 << 28, streams=2, own_outputs=True)
    try:
        t0 = B.bmmc_server_now_ns() + 5_000_000
        tickets = B.bmmc_server_submit_many(srv, B.DescBatch(items), [t0 + int(r["arrival"] * 1e9) for r in reqs])
        assert len(tickets) == len(reqs) and len(set(tickets)) == len(reqs)
        torch.cuda.synchronize()
        B.bmmc_server_drain(srv)
        for r, tk in zip(reqs, tickets):
            done, out = B.bmmc_server_poll(srv, tk)
            assert done >= t0 + int(r["arrival"] * 1e9)  # not before its arrival
            rows, c, a, x = pool[r["id"]]
            y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
            B.bmmc_copy(out, y, a.nbytes, G.stream())
            G.sync()
            assert np.array_equal(G.to_host(y, a), O.permute(a, r["n"], rows, c)), r
            B.bmmc_server_release(srv, tk)
    finally:
        B.bmmc_server_destroy(srv)


def test_server_stats_reset_after_warm_up():
    n, w = 16, 4
    srv = B.bmmc_server_create(1 << 28, streams=2, own_outputs=True)
    try:
        a = gen.data(n, w, 90)
        x = G.to_device(a)
        torch.cuda.synchronize()
        for k in range(3):
            rows, c = gen.random_bmmc(n, 90 + k)
            B.bmmc_server_submit(srv, x, 0, n, rows, c, w)
        B.bmmc_server_drain(srv)
        assert B.bmmc_server_stats(srv)["completed"] == 3
        B.bmmc_server_reset_stats(srv)
        st = B.bmmc_server_stats(srv)
        assert st["completed"] == 0 and st["p99_ms"] == 0
        rows, c = gen.random_bmmc(n, 99)
        tk = B.bmmc_server_submit(srv, x, 0, n, rows, c, w)
        done, out = B.bmmc_server_poll(srv, tk, wait=True)
        y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
        B.bmmc_copy(out, y, a.nbytes, G.stream())
        G.sync()
        assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c))
        B.bmmc_server_drain(srv)
        assert B.bmmc_server_stats(srv)["completed"] == 1
    finally:
        B.bmmc_server_destroy(srv)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_server_batched_launches_only(use_graph):
    """Forty requests arriving at the same instant, every launch batched (no
    single-array launches): every result equals the oracle's."""
    n_req = 40
    srv = B.bmmc_server_create(1 << 30, streams=2, own_outputs=True, use_graph=use_graph, direct_max=-1)
    try:
        work = []
        t0 = B.bmmc_server_now_ns() + 5_000_000
        for k in range(n_req):
            n, w = 10 + k % 9, (4, 8)[k % 2]
            rows, c = gen.random_bmmc(n, 700 + k)
            a = gen.data(n, w, 700 + k)
            x = G.to_device(a)
            work.append((n, w, rows, c, a, x))
        torch.cuda.synchronize()
        tickets = [B.bmmc_server_submit(srv, x, 0, n, rows, c, w, t0) for n, w, rows, c, a, x in work]
        B.bmmc_server_drain(srv)
        st = B.bmmc_server_stats(srv)
        assert st["completed"] == n_req and st["batches"] >= 1
        for tk, (n, w, rows, c, a, x) in zip(tickets, work):
            done, out = B.bmmc_server_poll(srv, tk)
            y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
            B.bmmc_copy(out, y, a.nbytes, G.stream())
            G.sync()
            assert np.array_equal(G.to_host(y, a), O.permute(a, n, rows, c))
            B.bmmc_server_release(srv, tk)
    finally:
        B.bmmc_server_destroy(srv)


def test_server_large_block_preserving_request():
    """A 512 MiB request whose matrix keeps its 4 KiB-block bits (the
    reversal), planned as a single-array call: the server plans it as the
    default call does (dealt output blocks on 16 KiB tiles); its output is
    the permutation on 65536 sampled outputs computed by the oracle."""
    n, w = 26, 8
    rows, c = gen.identity_rows(n), (1 << n) - 1
    a = gen.data(n, w, 4)
    x = G.to_device(a)
    srv = B.bmmc_server_create(2 << 30, streams=2, own_outputs=True, solo_log2=16)
    try:
        tk = B.bmmc_server_submit(srv, x, 0, n, rows, c, w)
        done, out = B.bmmc_server_poll(srv, tk, wait=True)
        y = torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev())
        B.bmmc_copy(out, y, a.nbytes, G.stream())
        G.sync()
        got = G.to_host(y, a)
        B.bmmc_server_release(srv, tk)
    finally:
        B.bmmc_server_destroy(srv)
    xs = np.random.default_rng(5).integers(0, 1 << n, size=1 << 16, dtype=np.uint64)
    xs[:2] = [0, (1 << n) - 1]
    ys = O.apply_many(rows, c, n, xs).astype(np.int64)
    assert np.array_equal(got[ys], a[xs.astype(np.int64)])
