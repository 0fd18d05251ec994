"""Parity of the exact configurations the benchmark times, in full (GPU only).

The benchmark's calls take the options of the shipped tuning file (a call
without options looks them up by size and matrix class), not the size
defaults the method-only tests get.  Each case here runs the call the
benchmark makes, on the benchmark's own input, and compares every output
element with the oracle (bit-exact: a permutation's output is unique).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_07795_amd import binding as B
from synth import gen
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def full_check(n, w, rows, c, seed, call):
    """call(x, y) runs the permutation; the whole output is compared."""
    print(f"full check n={n} w={w} seed={seed}", flush=True)
    a = gen.data(n, w, seed)
    x, y = G.to_device(a), G.empty_like_bytes(a)
    call(x, y)
    G.sync()
    got = G.to_host(y, a)
    del x, y
    torch.cuda.empty_cache()
    want = O.permute(a, n, rows, c)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} outputs differ, first at {int(bad[0])}"


def test_default_call_2p26_int32_seed0():
    """The benchmark's step: the random BMMC of seed 0 on 2^26 int32 (data of
    seed 0), by bmmc_permute with no options (the tuning-file plan) and by
    bmmc_permute_ex with the options the benchmark looks up."""
    n, w = 26, 4
    rows, c = gen.random_bmmc(n, 0)
    tuned = B.bmmc_tune_lookup(n, w, rows, B.METHOD_AUTO)
    assert tuned is not None, "the tuning file has an entry for the benchmark's workload"
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute(x, y, n, rows, c, w, G.stream()))
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute_ex(x, y, n, rows, c, w, tuned, G.stream()))


def test_tuned_two_pass_2p26_int32_seed0():
    """The paper's scheme as the benchmark times it: two tiled passes with
    the tuned options of BMMC_METHOD_TILED."""
    n, w = 26, 4
    rows, c = gen.random_bmmc(n, 0)
    tuned = B.bmmc_tune_lookup(n, w, rows, B.METHOD_TILED)
    assert tuned is not None
    assert B.bmmc_plan_ex(rows, c, n, w, tuned).nfactors == 2
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute_ex(x, y, n, rows, c, w, tuned, G.stream()))


@pytest.mark.parametrize("seed", range(1, 8))
def test_default_call_2p26_other_seeds(seed):
    """The other random matrices the benchmark times (seeds 1-7)."""
    n, w = 26, 4
    rows, c = gen.random_bmmc(n, seed)
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute(x, y, n, rows, c, w, G.stream()))


@pytest.mark.parametrize("case", ["random28", "random27x8", "bitrev28", "bitrev27x8", "swap28", "swap27x8"])
def test_sweep_arrays_full(case):
    """The 1 GiB sweep arrays as the benchmark's --workload runs them: the
    call without options, seed 0 matrix and data, whole output compared."""
    n, w = (28, 4) if case.endswith("28") else (27, 8)
    if case.startswith("random"):
        rows, c = gen.random_bmmc(n, 0)
    elif case.startswith("bitrev"):
        rows, c = gen.bit_reversal_rows(n), 0
    else:
        rows, c = gen.block_swap_rows(n, n // 2), 0
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute(x, y, n, rows, c, w, G.stream()))


@pytest.mark.parametrize("case", ["random28", "random27x8"])
def test_sweep_arrays_two_pass_full(case):
    """The paper's scheme on the 1 GiB random arrays with its tuned options."""
    n, w = (28, 4) if case == "random28" else (27, 8)
    rows, c = gen.random_bmmc(n, 0)
    tuned = B.bmmc_tune_lookup(n, w, rows, B.METHOD_TILED) or {"method": B.METHOD_TILED}
    full_check(n, w, rows, c, 0, lambda x, y: B.bmmc_permute_ex(x, y, n, rows, c, w, tuned, G.stream()))
