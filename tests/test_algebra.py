"""Host BMMC algebra of the library (composition, inverse, parm matrices)
against the oracle and the paper's printed matrices (no GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07795_amd import binding as B
from synth import gen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def printed_rows(matrix):
    return [sum(1 << j for j, ch in enumerate(r) if ch == "1") for r in matrix]


def parm_target(x, n, mask):
    """Section 7.2 by counting: sub-array x.mask, order kept inside it."""
    sub = lambda v: bin(v & mask).count("1") & 1
    s = sub(x)
    return (s << (n - 1)) | sum(1 for v in range(x) if sub(v) == s)


@pytest.mark.parametrize("name", ["parm_0011", "parm_110"])
def test_parm_matrix_is_the_printed_one(name):
    g = GOLDEN[name]
    rows, inv = B.bmmc_parm_matrix(g["mask"], g["n"])
    assert rows == printed_rows(g["matrix"])
    n = g["n"]
    assert np.array_equal(O.mul(O.dense(rows, n), O.dense(inv, n)), np.eye(n, dtype=np.uint8))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_parm_matrix_every_mask(n):
    for mask in range(1, 1 << n):
        rows, inv = B.bmmc_parm_matrix(mask, n)
        for x in range(1 << n):
            y = O.apply(rows, 0, n, x)
            assert y == parm_target(x, n, mask)
            assert O.apply(inv, 0, n, y) == x


def test_parm_matrix_rejects_bad_masks():
    with pytest.raises(B.BmmcError):
        B.bmmc_parm_matrix(0, 4)
    with pytest.raises(B.BmmcError):
        B.bmmc_parm_matrix(1 << 4, 4)


@pytest.mark.parametrize("n,seed", [(3, 0), (7, 1), (12, 2), (20, 3), (32, 4)])
def test_compose_is_sequential_application(n, seed):
    ra, c = gen.random_bmmc(n, seed)
    rb, d = gen.random_bmmc(n, seed + 77)
    rab, e = B.bmmc_compose(ra, c, rb, d, n)
    xs = np.random.default_rng(seed).integers(0, 1 << n, size=500, dtype=np.uint64)
    two = O.apply_many(ra, c, n, O.apply_many(rb, d, n, xs))
    assert np.array_equal(O.apply_many(rab, e, n, xs), two)


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (16, 2), (30, 3)])
def test_invert_undoes(n, seed):
    rows, c = gen.random_bmmc(n, seed)
    ri, ci = B.bmmc_invert(rows, c, n)
    xs = np.random.default_rng(seed).integers(0, 1 << n, size=500, dtype=np.uint64)
    assert np.array_equal(O.apply_many(ri, ci, n, O.apply_many(rows, c, n, xs)), xs)
    assert np.array_equal(O.dense(ri, n), O.inverse(O.dense(rows, n)))
    with pytest.raises(B.BmmcError) as e:
        B.bmmc_invert([0b11, 0b11], 0, 2)
    assert e.value.status == -2


def test_parm_identity_through_matrices():
    """parm mask f = bmmc(A^-1) . parm 2^(n-1) f . bmmc(A) (Section 3), with f
    reversing each half: checked element by element on the oracle."""
    n, mask = 6, 0b101001
    rows, inv = B.bmmc_parm_matrix(mask, n)
    a = np.arange(1 << n, dtype=np.uint32) * 7 + 3
    half = 1 << (n - 1)
    # right-hand side: permute, reverse each contiguous half, permute back
    t = O.permute(a, n, rows, 0)
    t = np.concatenate([t[:half][::-1], t[half:][::-1]])
    rhs = O.permute(t, n, inv, 0)
    # left-hand side: split by x.mask directly, reverse each sub-array, stitch
    sub = np.array([bin(x & mask).count("1") & 1 for x in range(1 << n)])
    lhs = a.copy()
    for s in (0, 1):
        idx = np.nonzero(sub == s)[0]
        lhs[idx] = a[idx][::-1]
    assert np.array_equal(lhs, rhs)
