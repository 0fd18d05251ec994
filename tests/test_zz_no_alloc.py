"""The allocation-free batched entry point against bmmc_permute_batched (GPU).

bmmc_permute_batched_noalloc keeps the batch's table, work items and queue
heads in the library's one fixed device array.  Its outputs must equal those
of bmmc_permute_batched bit for bit (a permutation's output is unique), on two
calls in a row, the second with a smaller batch, so that the second call
finds the first call's table and heads left in the array.
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
        rows, c = gen.random_bmmc(n, seed * 7919 + k)
        a = gen.data(n, w, seed * 7919 + k)
        arrays.append({"n": n, "w": w, "rows": rows, "c": c, "a": a, "x": G.to_device(a),
                       "y_ref": G.empty_like_bytes(a), "y": G.empty_like_bytes(a)})
    return arrays


def run_both(arrays, opts):
    """The existing entry point into y_ref, the allocation-free one into y."""
    ref = [(a["x"], a["y_ref"], a["n"], a["w"], a["rows"], a["c"]) for a in arrays]
    new = [(a["x"], a["y"], a["n"], a["w"], a["rows"], a["c"]) for a in arrays]
    for a in arrays:
        a["y"].fill_(0xA5)  # a kernel fill: the result must overwrite it
    B.bmmc_permute_batched(ref, G.stream(), opts)
    B.bmmc_permute_batched_noalloc(new, G.stream(), opts)
    G.sync()


def check(arrays, oracle_every=1):
    for k, a in enumerate(arrays):
        got = G.to_host(a["y"], a["a"])
        ref = G.to_host(a["y_ref"], a["a"])
        assert np.array_equal(got, ref), f"array {k}: n={a['n']} w={a['w']} differs from bmmc_permute_batched"
        if k % oracle_every == 0:
            want = O.permute(a["a"], a["n"], a["rows"], a["c"])
            assert np.array_equal(got, want), f"array {k}: n={a['n']} w={a['w']} differs from the oracle"


@pytest.mark.parametrize("opts", [None, {"iters": 4, "chunk_tiles": 4}, {"iters": 32, "chunk_tiles": 1},
                                  {"iters": 8, "chunk_tiles": 2, "method": B.METHOD_ONEPASS, "hints": 3}])
def test_noalloc_matches_batched_two_calls(opts):
    """A large mixed batch, then a smaller one: both equal the existing
    entry point's outputs (and the oracle's)."""
    print(f"noalloc two calls opts={opts}", flush=True)
    rng = np.random.default_rng(11)
    sizes1 = [int(v) for v in rng.integers(0, 21, size=96)] + [22, 22]
    widths1 = [int(v) for v in rng.choice([4, 8, 16, 1, 2], size=len(sizes1))]
    first = make_batch(sizes1, widths1, 1)
    run_both(first, opts)
    check(first)
    del first
    torch.cuda.empty_cache()
    sizes2 = [int(v) for v in rng.integers(8, 16, size=9)]
    second = make_batch(sizes2, [4] * len(sizes2), 2)
    run_both(second, opts)
    check(second)


def test_noalloc_workload_batch_then_small():
    """The 1024-array workload (n uniform in [10, 22], int32), then three
    arrays: every output equals the existing entry point's."""
    print("noalloc workload batch", flush=True)
    sizes = gen.batched_sizes(1024, 0, 10, 22)
    first = make_batch(sizes, [4] * len(sizes), 3)
    run_both(first, None)
    check(first, oracle_every=16)
    del first
    torch.cuda.empty_cache()
    second = make_batch([14, 19, 11], [4, 8, 4], 4)
    run_both(second, None)
    check(second)


def test_noalloc_refusals():
    """Two-pass method and a table beyond the fixed array are refused with
    an error; nothing is launched for them."""
    print("noalloc refusals", flush=True)
    arrays = make_batch([16, 18], [4, 4], 5)
    new = [(a["x"], a["y"], a["n"], a["w"], a["rows"], a["c"]) for a in arrays]
    with pytest.raises(B.BmmcError):
        B.bmmc_permute_batched_noalloc(new, G.stream(), {"method": B.METHOD_TILED})
    # 2^20-element arrays cut into tiles of 2^12 elements, one per item:
    # 256 items of 16 bytes each per array, so the items alone of this many
    # arrays overflow the table
    cap = B.bmmc_noalloc_table_bytes()
    count = cap // (256 * 16) + 1
    a = gen.data(20, 4, 6)
    x = G.to_device(a)
    outs = [torch.empty(a.nbytes, dtype=torch.uint8, device=G.dev()) for _ in range(count)]
    rows, c = gen.random_bmmc(20, 6)
    big = [(x, o, 20, 4, rows, c) for o in outs]
    with pytest.raises(B.BmmcError):
        B.bmmc_permute_batched_noalloc(big, G.stream(), {"iters": 4, "chunk_tiles": 1})
    G.sync()
