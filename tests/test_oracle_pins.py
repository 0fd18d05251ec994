"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each test ties the oracle to something it does not compute itself: values the
paper prints (tests/golden/paper_examples.json), library routines (numpy
reshape / transpose / flip), closed forms (|GL(n,2)|), the parm definition of
Section 7.2, and brute-force properties on tiny n.  A dropped term, a swapped
index, a transposed matrix, a gather instead of a scatter or a wrong bit order
in the oracle fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth import gen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def printed_rows(matrix):
    """Rows of a matrix printed as strings (character j of string i is a_ij)."""
    return [sum(1 << j for j, ch in enumerate(r) if ch == "1") for r in matrix]


def printed_vec(s):
    """Column vector printed top to bottom (c_0 first)."""
    return sum(1 << i for i, ch in enumerate(s) if ch == "1")


# ------------------------------------------------------------ paper values

def test_bitrev_7_to_14():
    g = GOLDEN["bitrev4"]
    rows = printed_rows(g["matrix"])
    for x, y in g["pairs"]:
        assert O.apply(rows, printed_vec(g["c"]), g["n"], x) == y
    # the generator's anti-diagonal matrix is the printed one
    assert gen.bit_reversal_rows(4) == rows


def test_transpose_6_to_9():
    g = GOLDEN["transpose4x4"]
    rows = printed_rows(g["matrix"])
    for x, y in g["pairs"]:
        assert O.apply(rows, 0, g["n"], x) == y
    # y_i = x_((i + 2) mod 4) for all x
    for x in range(16):
        y = O.apply(rows, 0, 4, x)
        for i in range(4):
            assert (y >> i) & 1 == (x >> ((i + 2) % 4)) & 1


def test_complement_reverses_array():
    g = GOLDEN["reverse16"]
    rows, c = printed_rows(g["matrix"]), printed_vec(g["c"])
    assert [O.apply(rows, c, 4, x) for x in range(16)] == [15 - x for x in range(16)]
    data = gen.data(4, 4, 7)
    assert np.array_equal(O.permute(data, 4, rows, c), data[::-1])


def test_cyclic_shift_example():
    g = GOLDEN["cyclic_shift5"]
    rows = gen.bpc_rows(g["p"])
    assert rows == gen.cyclic_shift_rows(5)
    for xs, ys in g["pairs_binary"]:
        assert O.apply(rows, 0, g["n"], int(xs, 2)) == int(ys, 2)


def parm_target(x, n, mask):
    """Section 7.2 definition, computed by counting: the element at x belongs
    to sub-array (x . mask) and keeps its order inside that sub-array; it lands
    at sub-array * 2^(n-1) + sub-index."""
    sub = lambda v: bin(v & mask).count("1") & 1
    s = sub(x)
    idx = sum(1 for v in range(x) if sub(v) == s)
    return (s << (n - 1)) | idx


def test_parm_0011_matrix_matches_parm_definition():
    g = GOLDEN["parm_0011"]
    rows = printed_rows(g["matrix"])
    n, mask = g["n"], g["mask"]
    got = [O.apply(rows, 0, n, x) for x in range(1 << n)]
    assert got == [parm_target(x, n, mask) for x in range(1 << n)]


def test_parm_110_printed_table_and_scatter_direction():
    g = GOLDEN["parm_110"]
    rows = printed_rows(g["matrix"])
    n = g["n"]
    for x, sub_array, sub_index in g["table"]:
        y = (sub_array << (n - 1)) | sub_index
        assert O.apply(rows, 0, n, x) == y
        assert parm_target(x, n, g["mask"]) == y
    # Scatter: permuting xs with (A, 0) puts xs0 first and xs1 second, order kept.
    xs = np.arange(100, 108, dtype=np.uint32)
    out = O.permute(xs, n, rows, 0)
    table = sorted(g["table"], key=lambda r: (r[1], r[2]))
    assert list(out) == [100 + r[0] for r in table]


def test_appendix_naive_bit_moves():
    g = GOLDEN["appendix_bitrev15"]
    rows = gen.bit_reversal_rows(g["n"])
    for src, dst in g["naive_bit_moves"]:
        assert O.apply(rows, 0, g["n"], 1 << src) == 1 << dst


# ------------------------------------------------------- library routines

def bpc_by_numpy(a, n, p, c):
    """out for the BPC y_{p(j)} = x_j XOR c_{p(j)}, built only from numpy's
    reshape / transpose / flip.  Axis k of the [2]*n view is bit n-1-k."""
    inv = [0] * n
    for j in range(n):
        inv[p[j]] = j
    t = a.reshape([2] * n).transpose([n - 1 - inv[n - 1 - k] for k in range(n)])
    for k in range(n):
        if (c >> (n - 1 - k)) & 1:
            t = np.flip(t, axis=k)
    return np.ascontiguousarray(t).reshape(-1)


@pytest.mark.parametrize("n,seed", [(1, 0), (3, 1), (6, 2), (9, 3), (12, 4), (14, 5)])
def test_random_bpc_equals_numpy(n, seed):
    p = gen.random_perm(n, seed)
    rows, c = gen.random_bpc(n, seed)
    assert rows == gen.bpc_rows(p)
    a = gen.data(n, 4, seed)
    assert np.array_equal(O.permute(a, n, rows, c), bpc_by_numpy(a, n, p, c))


@pytest.mark.parametrize("n,k", [(4, 2), (8, 3), (10, 5), (13, 6), (14, 9)])
def test_block_swap_is_matrix_transpose(n, k):
    a = gen.data(n, 4, n * 31 + k)
    want = a.reshape(1 << (n - k), 1 << k).T.copy().reshape(-1)
    assert np.array_equal(O.permute(a, n, gen.block_swap_rows(n, k), 0), want)


@pytest.mark.parametrize("n", [2, 5, 11])
def test_bit_reversal_numpy(n):
    a = gen.data(n, 8, n)
    want = a.reshape([2] * n).transpose(list(range(n))[::-1]).reshape(-1)
    assert np.array_equal(O.permute(a, n, gen.bit_reversal_rows(n), 0), want)


def test_element_widths_are_opaque():
    n = 7
    rows, c = gen.random_bmmc(n, 11)
    ys = O.index_map(rows, c, n)
    for w in (1, 2, 4, 8, 16):
        a = gen.data(n, w, 3)
        out = O.permute(a, n, rows, c)
        assert np.array_equal(out[ys.astype(np.int64)], a)


# ---------------------------------------------------- closed forms, brute force

def all_rows(n):
    return itertools.product(range(1 << n), repeat=n)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_gl_count_and_rank_is_injectivity(n):
    """rank(A) = n exactly when x -> A.x is injective; the number of such
    matrices is prod_{k<n} (2^n - 2^k)."""
    count = 0
    for rows in all_rows(n):
        m = O.dense(rows, n)
        inj = len({O.matvec(m, x) for x in range(1 << n)}) == (1 << n)
        full = O.rank(m) == n
        assert inj == full
        count += full
    closed = 1
    for k in range(n):
        closed *= (1 << n) - (1 << k)
    assert count == closed == {1: 1, 2: 6, 3: 168, 4: 20160}[n]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_fast_and_summed_forms_agree_everywhere(n):
    for rows in all_rows(n):
        for c in range(1 << n):
            for x in range(1 << n):
                assert O.apply(rows, c, n, x) == O.apply_sum(rows, c, n, x)


def test_fast_form_n4_and_bijection_every_invertible_matrix():
    n = 4
    seen = 0
    for rows in all_rows(n):
        if O.rank(O.dense(rows, n)) != n:
            continue
        seen += 1
        c = seen % 16
        ys = O.index_map(rows, c, n)
        assert sorted(ys.tolist()) == list(range(16))
        if seen % 97 == 0:
            assert all(O.apply_sum(rows, c, n, x) == int(ys[x]) for x in range(16))
    assert seen == 20160


@pytest.mark.parametrize("n,seed", [(5, 1), (10, 2), (16, 3), (20, 4)])
def test_bijection_iota(n, seed):
    rows, c = gen.random_bmmc(n, seed)
    out = O.permute(gen.iota(n, 4), n, rows, c)
    assert np.array_equal(np.sort(out), np.arange(1 << n, dtype=np.uint32))


def test_identity_is_copy():
    a = gen.data(10, 4, 1)
    assert np.array_equal(O.permute(a, 10, gen.identity_rows(10), 0), a)


# ------------------------------------------------------- algebraic invariants

@pytest.mark.parametrize("n,seed", [(3, 0), (8, 1), (12, 2), (17, 3)])
def test_inverse_undoes(n, seed):
    """(A^-1, A^-1 c) undoes (A, c); A A^-1 = I."""
    rows, c = gen.random_bmmc(n, seed)
    m = O.dense(rows, n)
    mi = O.inverse(m)
    assert np.array_equal(O.mul(m, mi), np.eye(n, dtype=np.uint8))
    assert np.array_equal(O.mul(mi, m), np.eye(n, dtype=np.uint8))
    ci = O.matvec(mi, c)
    a = gen.data(n, 4, seed)
    assert np.array_equal(O.permute(O.permute(a, n, rows, c), n, O.packed(mi), ci), a)


def test_singular_has_no_inverse():
    rows = [0b011, 0b110, 0b101]  # row 2 = row 0 + row 1
    assert O.rank(O.dense(rows, 3)) == 2
    assert O.inverse(O.dense(rows, 3)) is None


@pytest.mark.parametrize("n,seed", [(4, 0), (9, 1), (13, 2)])
def test_composition_rule(n, seed):
    """bmmc(A, c) after bmmc(B, d) = bmmc(AB, A d + c)  (Section 3)."""
    ra, c = gen.random_bmmc(n, seed)
    rb, d = gen.random_bmmc(n, seed + 100)
    A, B = O.dense(ra, n), O.dense(rb, n)
    AB = O.packed(O.mul(A, B))
    e = O.matvec(A, d) ^ c
    a = gen.data(n, 4, seed)
    two = O.permute(O.permute(a, n, rb, d), n, ra, c)
    assert np.array_equal(two, O.permute(a, n, AB, e))


def test_mul_is_composition_of_maps():
    n = 5
    for s in range(20):
        ra, _ = gen.random_bmmc(n, s)
        rb, _ = gen.random_bmmc(n, s + 50)
        AB = O.packed(O.mul(O.dense(ra, n), O.dense(rb, n)))
        for x in range(1 << n):
            assert O.apply(AB, 0, n, x) == O.apply(ra, 0, n, O.apply(rb, 0, n, x))


# ----------------------------------------------------------- tiled condition

def preimage_is_coordinate(rows, n, t):
    """Geometric form of the tiled condition: the inputs that land in the first
    2^t outputs are exactly the sums of a set J of t unit vectors."""
    pre = [x for x in range(1 << n) if O.apply(rows, 0, n, x) < (1 << t)]
    J = [j for j in range(n) if O.apply(rows, 0, n, 1 << j) < (1 << t)]
    if len(J) != t:
        return False, 0
    span = set()
    for bits in range(1 << t):
        span.add(sum(1 << J[k] for k in range(t) if (bits >> k) & 1))
    return set(pre) == span, sum(1 << j for j in J)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_tiled_condition_brute_force(n):
    for rows in all_rows(n):
        m = O.dense(rows, n)
        if O.rank(m) != n:
            continue
        for t in range(n + 1):
            ok, cols = O.is_tiled(m, t)
            geo, gcols = preimage_is_coordinate(rows, n, t)
            assert ok == geo
            if ok:
                assert cols == gcols


@pytest.mark.parametrize("n,seed", [(6, 0), (10, 1), (13, 2)])
def test_every_bpc_is_tiled(n, seed):
    """Section 5.1: a BPC is always tiled; the columns are the tile row bits."""
    p = gen.random_perm(n, seed)
    m = O.dense(gen.bpc_rows(p), n)
    for t in range(n + 1):
        ok, cols = O.is_tiled(m, t)
        assert ok
        assert cols == sum(1 << j for j in range(n) if p[j] < t)


# ------------------------------------------- sorting network (Section 7.1)

def _parm_py(mask, f, xs):
    """parm by its definition: sub-array of index i = parity of i & mask,
    order kept inside each sub-array, f applied to each, stitched back."""
    sub = [bin(i & mask).count("1") & 1 for i in range(len(xs))]
    parts = [[x for x, s in zip(xs, sub) if s == k] for k in (0, 1)]
    done = [iter(f(p)) for p in parts]
    return [next(done[s]) for s in sub]


def _vcolumn_py(n, xs):
    if n == 0:
        return xs
    if n == 1:
        return xs if xs[0] <= xs[1] else [xs[1], xs[0]]
    return _parm_py(3, lambda s: _vcolumn_py(n - 1, s), xs)


def _merge_py(n, xs):
    if n == 0:
        return xs
    ys = _vcolumn_py(n, xs)
    return _parm_py(1 << (n - 1), lambda s: _merge_py(n - 1, s), ys)


def _sortnet_py(n, xs):
    if n == 0:
        return xs
    ys = _parm_py(1, lambda s: _sortnet_py(n - 1, s), xs)
    return _merge_py(n, ys)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_papers_network_sorts_every_zero_one_input(n):
    """The 0-1 principle over every 0-1 input: the network of Section 7.1,
    written out by its recursion, gives the oracle's sorted keys."""
    for bits in itertools.product([0, 1], repeat=1 << n):
        a = np.array(bits, dtype=np.int32)
        assert np.array_equal(np.array(_sortnet_py(n, list(bits)), dtype=np.int32), O.sort_keys(a))


@pytest.mark.parametrize("n,seed", [(5, 0), (6, 1), (7, 2)])
def test_papers_network_on_integers_with_duplicates(n, seed):
    a = np.random.default_rng(seed).integers(-20, 20, size=1 << n).astype(np.int32)
    assert np.array_equal(np.array(_sortnet_py(n, a.tolist()), dtype=np.int32), O.sort_keys(a))


@pytest.mark.parametrize("signed", [True, False])
@pytest.mark.parametrize("n,seed", [(0, 0), (4, 1), (12, 2), (16, 3)])
def test_sort_oracle_is_an_ordered_rearrangement(n, seed, signed):
    """Ascending in the key order and the same multiset of keys: the unique
    result of sorting."""
    rng = np.random.default_rng(seed)
    a = rng.integers(-(1 << 31), 1 << 31, size=1 << n, dtype=np.int64).astype(np.int32)
    a[: len(a) // 4] = a[0]  # duplicates
    out = O.sort_keys(a, signed)
    k = out.view(np.int32 if signed else np.uint32).astype(np.int64)
    assert np.all(k[1:] >= k[:-1])
    va, ca = np.unique(a, return_counts=True)
    vo, co = np.unique(out, return_counts=True)
    assert np.array_equal(va, vo) and np.array_equal(ca, co)
    if not signed and n >= 4:
        # negative int32 keys are large unsigned keys: they come last
        neg = np.nonzero(out < 0)[0]
        assert len(neg) == 0 or neg[0] == len(out) - len(neg)
