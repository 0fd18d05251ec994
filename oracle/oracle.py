"""Python face of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liboracle.so`` (built from
``bmmc_oracle.c`` with gcc) and never touches the GPU library.

Definitions (paper, Section 3): y = A.x XOR c over F_2 with y_i = sum_j a_ij x_j
+ c_i mod 2, bit 0 the least significant; the permutation is the scatter
out[A.x XOR c] = in[x] (Section 4.1 kernel, Section 7.2).  Matrices cross this
interface as ``rows``: a sequence of n ints, bit j of rows[i] being a_ij.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64, i32, i64 = ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
        vp = ctypes.c_void_p
        L.oracle_apply.restype = u64
        L.oracle_apply.argtypes = [vp, u64, i32, u64]
        L.oracle_apply_sum.restype = u64
        L.oracle_apply_sum.argtypes = [vp, u64, i32, u64]
        L.oracle_apply_many.restype = None
        L.oracle_apply_many.argtypes = [vp, u64, i32, vp, vp, i64]
        L.oracle_permute.restype = i32
        L.oracle_permute.argtypes = [vp, vp, i32, vp, u64, i32, i32]
        L.oracle_threads.restype = i32
        L.oracle_threads.argtypes = [i32]
        L.oracle_mul.restype = None
        L.oracle_mul.argtypes = [vp, vp, vp, i32]
        L.oracle_rank.restype = i32
        L.oracle_rank.argtypes = [vp, i32, i32]
        L.oracle_inverse.restype = i32
        L.oracle_inverse.argtypes = [vp, vp, i32]
        L.oracle_is_tiled.restype = i32
        L.oracle_is_tiled.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


def _rows_arr(rows, n):
    a = np.zeros(max(n, 1), dtype=np.uint64)
    for i in range(n):
        a[i] = int(rows[i])
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- index map

def apply(rows, c: int, n: int, x: int) -> int:
    """A.x XOR c for one index (Section 3, per-bit form)."""
    r = _rows_arr(rows, n)
    return int(lib().oracle_apply(_ptr(r), c, n, x))


def apply_sum(rows, c: int, n: int, x: int) -> int:
    """Same map with the double sum written out entry by entry."""
    r = _rows_arr(rows, n)
    return int(lib().oracle_apply_sum(_ptr(r), c, n, x))


def apply_many(rows, c: int, n: int, xs) -> np.ndarray:
    r = _rows_arr(rows, n)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    ys = np.empty_like(xs)
    lib().oracle_apply_many(_ptr(r), c, n, _ptr(xs), _ptr(ys), xs.size)
    return ys


def index_map(rows, c: int, n: int) -> np.ndarray:
    """y for every x in [0, 2^n)."""
    return apply_many(rows, c, n, np.arange(1 << n, dtype=np.uint64))


def permute(inp: np.ndarray, n: int, rows, c: int, nthreads: int = 0) -> np.ndarray:
    """out[A.x XOR c] = in[x]; elements are the rows of ``inp`` viewed as bytes."""
    inp = np.ascontiguousarray(inp)
    if inp.shape[0] != (1 << n):
        raise ValueError("input must hold 2^n elements")
    w = inp.itemsize * (int(np.prod(inp.shape[1:])) if inp.ndim > 1 else 1)
    out = np.empty_like(inp)
    r = _rows_arr(rows, n)
    rc = lib().oracle_permute(_ptr(inp), _ptr(out), n, _ptr(r), c, w, nthreads)
    if rc != 0:
        raise ValueError("oracle_permute rejected its arguments")
    return out


def threads(nthreads: int = 0) -> int:
    return int(lib().oracle_threads(nthreads))


# ---------------------------------------------------------------- dense F_2

def dense(rows, n: int) -> np.ndarray:
    """n x n uint8 matrix, entry (i, j) = bit j of rows[i]."""
    m = np.zeros((n, n), dtype=np.uint8)
    for i in range(n):
        for j in range(n):
            m[i, j] = (int(rows[i]) >> j) & 1
    return m


def packed(m: np.ndarray):
    """Inverse of ``dense``."""
    n = m.shape[0]
    return [sum(int(m[i, j]) << j for j in range(n)) for i in range(n)]


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    n = a.shape[0]
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros((n, n), dtype=np.uint8)
    lib().oracle_mul(_ptr(a), _ptr(b), _ptr(out), n)
    return out


def rank(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return int(lib().oracle_rank(_ptr(a), a.shape[0], a.shape[1]))


def inverse(a: np.ndarray):
    n = a.shape[0]
    a = np.ascontiguousarray(a, dtype=np.uint8)
    out = np.zeros((n, n), dtype=np.uint8)
    if lib().oracle_inverse(_ptr(a), _ptr(out), n) != 0:
        return None
    return out


def is_tiled(a: np.ndarray, t: int):
    """(tiled?, column mask) per the Section 5.1 condition."""
    n = a.shape[0]
    a = np.ascontiguousarray(a, dtype=np.uint8)
    cols = ctypes.c_uint64(0)
    ok = lib().oracle_is_tiled(_ptr(a), n, t, ctypes.byref(cols))
    return bool(ok), int(cols.value)


def matvec(a: np.ndarray, x: int) -> int:
    """A.x over F_2 with the dense matrix (no complement)."""
    n = a.shape[0]
    y = 0
    for i in range(n):
        s = 0
        for j in range(n):
            s ^= int(a[i, j]) & ((x >> j) & 1)
        y |= s << i
    return y


def sort_keys(keys: np.ndarray, signed: bool = True) -> np.ndarray:
    """Section 7.1: the even/odd merge sort written with parm (a balanced
    periodic merger of V-shaped columns) sorts its input into ascending
    order, so its result is the sorted keys; a library sort is that step.
    keys: 4-byte keys compared as int32 (signed) or uint32; returned with the
    input's dtype."""
    a = np.ascontiguousarray(keys)
    if a.dtype.itemsize != 4:
        raise ValueError("4-byte keys expected")
    v = a.view(np.int32 if signed else np.uint32)
    return np.sort(v, kind="stable").view(a.dtype)
