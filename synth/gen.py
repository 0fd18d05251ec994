"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws numbers: it contains none of the permutation's
arithmetic (no index map, no factorization, no kernel logic).  Both the GPU
path's callers and the oracle's callers take their inputs from here, so the two
sides see identical bytes.

Random numbers come from splitmix64 (S. Vigna's published generator: add the
constant 0x9E3779B97F4A7C15 to the state, then mix with two xor-shift-multiply
rounds and a final xor-shift).  Its k-th output (k = 0, 1, ...) for seed s is
mix(s + (k + 1) * 0x9E3779B97F4A7C15), which makes it counter-based and
vectorizable.

Streams (one per purpose):
  * matrix / complement: seed s, rows drawn first, then c;
  * data: seed s ^ 0xD1B54A32D192ED03.

Matrices are returned as ``rows``: a list of n ints, bit j of rows[i] being the
entry a_ij (row i gives output bit i, bit 0 is the least significant).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
DATA_SEED_XOR = 0xD1B54A32D192ED03
_M64 = (1 << 64) - 1


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential splitmix64 stream."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & _M64
        return _mix(self.state)

    def below(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection (no modulo bias)."""
        if bound <= 1:
            return 0
        limit = (1 << 64) - ((1 << 64) % bound)
        while True:
            v = self.next()
            if v < limit:
                return v % bound

    def uniform(self) -> float:
        """Uniform float in (0, 1] from the top 53 bits."""
        return ((self.next() >> 11) + 1) * (1.0 / (1 << 53))


def splitmix64_array(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the stream seeded with ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & _M64) + k * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


_DTYPES = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def data(n: int, w: int, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """2^n elements of w bytes, uniform random, from the data stream of ``seed``.

    w in {1, 2, 4, 8}: element i is the low 8w bits of draw i.
    w = 16: element i is draws 2i (low half) and 2i+1 (high half).
    The result has shape (2^n,) for w <= 8 and (2^n, 2) uint64 for w = 16.
    """
    s = seed ^ DATA_SEED_XOR
    size = 1 << n
    if w == 16:
        out = np.empty((size, 2), dtype=np.uint64)
        flat = out.reshape(-1)

        def fill(a):
            m = min(chunk, 2 * size - a)
            flat[a:a + m] = splitmix64_array(s, m, a)
        _each_chunk(fill, 2 * size, chunk)
        return out
    if w not in _DTYPES:
        raise ValueError("element width must be 1, 2, 4, 8 or 16 bytes")
    out = np.empty(size, dtype=_DTYPES[w])

    def fill(a):
        m = min(chunk, size - a)
        out[a:a + m] = splitmix64_array(s, m, a).astype(_DTYPES[w])
    _each_chunk(fill, size, chunk)
    return out


def _each_chunk(fill, total: int, chunk: int):
    """fill(a) for a = 0, chunk, 2 chunk, ... < total; large arrays on a few
    threads (numpy's elementwise work releases the GIL; every chunk depends
    only on its own offsets, so the result is the same)."""
    starts = range(0, total, chunk)
    if len(starts) <= 2:
        for a in starts:
            fill(a)
        return
    import concurrent.futures as cf
    import os
    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        list(ex.map(fill, starts))


def iota(n: int, w: int) -> np.ndarray:
    """in[i] = i (an extra correctness payload: every value names its source)."""
    if w == 16:
        out = np.zeros((1 << n, 2), dtype=np.uint64)
        out[:, 0] = np.arange(1 << n, dtype=np.uint64)
        return out
    return np.arange(1 << n, dtype=np.uint64).astype(_DTYPES[w])


def _independent_of(basis: dict, v: int) -> bool:
    """True when v is outside the span of the rows kept so far (rejection test
    for the matrix sampler; basis maps a leading bit to a stored row)."""
    while v:
        top = v.bit_length() - 1
        if top not in basis:
            basis[top] = v
            return True
        v ^= basis[top]
    return False


def random_bmmc(n: int, seed: int):
    """(rows, c): a uniformly random invertible n x n matrix over F_2 and a
    uniformly random n-bit complement.

    Rows are drawn one at a time from the stream and a row is rejected when it
    lies in the span of the rows already accepted; the result is uniform over
    the invertible matrices.  c is the next draw after the last accepted row.
    """
    rng = SplitMix64(seed)
    mask = (1 << n) - 1
    rows, basis = [], {}
    while len(rows) < n:
        r = rng.next() & mask
        if _independent_of(basis, r):
            rows.append(r)
    c = rng.next() & mask if n > 0 else 0
    return rows, c


def random_perm(n: int, seed: int):
    """Uniform permutation p of {0..n-1} (Fisher-Yates)."""
    rng = SplitMix64(seed)
    p = list(range(n))
    for i in range(n - 1, 0, -1):
        j = rng.below(i + 1)
        p[i], p[j] = p[j], p[i]
    return p


def bpc_rows(p):
    """Matrix of the bit permutation with y_{p(j)} = x_j: a 1 at (p(j), j)."""
    n = len(p)
    rows = [0] * n
    for j in range(n):
        rows[p[j]] |= 1 << j
    return rows


def random_bpc(n: int, seed: int):
    """(rows, c) of a uniformly random BPC: random bit permutation, random c."""
    p = random_perm(n, seed)
    rng = SplitMix64(seed ^ GOLDEN)
    c = rng.next() & ((1 << n) - 1) if n > 0 else 0
    return bpc_rows(p), c


def bit_reversal_rows(n: int):
    """Anti-diagonal identity: entry (i, j) is 1 exactly when i + j = n - 1."""
    return [1 << (n - 1 - i) for i in range(n)]


def identity_rows(n: int):
    return [1 << i for i in range(n)]


def block_swap_rows(n: int, k: int):
    """Bit permutation sending the low k bits to the top and the rest down:
    p(j) = j + n - k for j < k, p(j) = j - k for j >= k."""
    return bpc_rows([(j + n - k) if j < k else (j - k) for j in range(n)])


def cyclic_shift_rows(n: int):
    """p(i) = i - 1 for i > 0 and p(0) = n - 1."""
    return bpc_rows([(i - 1) if i > 0 else (n - 1) for i in range(n)])


# ----------------------------------------------------------- workload mixes

def batched_sizes(count: int, seed: int, lo: int = 10, hi: int = 22):
    """n for each array of a batch: lo + (draw mod (hi - lo + 1))."""
    rng = SplitMix64(seed)
    span = hi - lo + 1
    return [lo + (rng.next() % span) for _ in range(count)]


def poisson_requests(count: int, rate: float, seed: int, n_lo: int = 12, n_hi: int = 26,
                     widths=(4, 8)):
    """Open-loop Poisson request stream: list of dicts with arrival time (s),
    n, element width and a per-request matrix seed.  Inter-arrival times are
    -ln(U)/rate."""
    rng = SplitMix64(seed)
    t = 0.0
    reqs = []
    for k in range(count):
        t += -math.log(rng.uniform()) / rate
        n = n_lo + rng.below(n_hi - n_lo + 1)
        w = widths[rng.below(len(widths))]
        reqs.append({"id": k, "arrival": t, "n": n, "w": w, "seed": rng.next()})
    return reqs
