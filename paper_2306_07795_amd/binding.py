"""ctypes binding of libbmmc.so: the C entry points under the same names.

Argument marshalling only: every step of a permutation runs in the library's
HIP kernels.  Device buffers are passed as integers (device addresses) or as
objects with ``data_ptr()`` (e.g. torch tensors); streams as integers or as
objects with a ``cuda_stream`` attribute (torch streams).  A non-zero status
raises ``BmmcError`` carrying the library's message.  If the library has not
been built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmmc.so")

MAX_BITS = 32
METHOD_AUTO, METHOD_TILED, METHOD_ONEPASS, METHOD_NAIVE = 0, 1, 2, 3
KEY_I32, KEY_U32 = 0, 1
SORTNET_PASSES, SORTNET_DIRECT = 0, 1

_c = ctypes
_u64, _i32, _i64, _vp, _dbl = _c.c_uint64, _c.c_int, _c.c_int64, _c.c_void_p, _c.c_double


class BmmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bmmc status {status}: {message}")
        self.status = status


class Options(_c.Structure):
    _fields_ = [("method", _i32), ("t", _i32), ("threads", _i32), ("iters", _i32),
                ("swizzle", _i32), ("grid", _i32), ("run_in", _i32), ("run_out", _i32),
                ("hints", _i32), ("tile_order", _i32), ("reserved", _i32 * 2)]


class Plan(_c.Structure):
    _fields_ = [("n", _i32), ("t", _i32), ("nfactors", _i32), ("elem_bytes", _i32),
                ("rows", (_u64 * 64) * 2), ("c", _u64 * 2), ("col_mask", _u64 * 2),
                ("tile_rows_mask", _u64 * 2), ("iter_mask", _u64 * 2), ("tb_mask", _u64 * 2),
                ("n_over", _i32 * 2), ("tile_bits", _i32 * 2), ("coordinate", _i32 * 2),
                ("lds_conflict_score", _i32 * 2)]

    def factor(self, k: int):
        """(rows, c) of factor k as Python ints."""
        return [int(self.rows[k][i]) for i in range(self.n)], int(self.c[k])


class Desc(_c.Structure):
    _fields_ = [("in_", _vp), ("out", _vp), ("n", _i32), ("elem_bytes", _i32),
                ("A_rows", _c.POINTER(_u64)), ("c", _u64)]


class BatchOptions(_c.Structure):
    _fields_ = [("workgroups", _i32), ("chunk_tiles", _i32), ("order", _i32),
                ("use_graph", _i32), ("method", _i32), ("hints", _i32), ("iters", _i32),
                ("tile_order", _i32)]


class KernelStat(_c.Structure):
    _fields_ = [("name", _c.c_char * 48), ("launches", _i32), ("total_ms", _dbl), ("bytes", _dbl)]


class EmuStats(_c.Structure):
    _fields_ = [(f, _i64) for f in (
        "tiles", "read_instr", "write_instr", "read_lines", "write_lines", "read_lines_min",
        "write_lines_min", "lds_instr", "lds_conflicts32", "lds_conflicts64", "lds_slot_errors",
        "dealt_write_tiles")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerStats(_c.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("rejected", _i64), ("batches", _i64),
                ("bytes_moved", _dbl), ("busy_s", _dbl), ("p50_ms", _dbl), ("p99_ms", _dbl),
                ("mean_ms", _dbl), ("max_ms", _dbl), ("in_use_bytes", _i64), ("peak_bytes", _i64),
                ("mean_batch", _dbl), ("mean_plan_ms", _dbl), ("mean_wait_ms", _dbl), ("mean_run_ms", _dbl),
                ("reserved", _dbl * 1)]


class ServerOptions(_c.Structure):
    _fields_ = [("budget_bytes", _i64), ("streams", _i32), ("max_batch", _i32),
                ("own_outputs", _i32), ("method", _i32), ("use_graph", _i32), ("direct_max", _i32),
                ("solo_log2", _i32), ("reserved", _i32 * 1)]


_lib = None


def lib():
    """Load libbmmc.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_07795_amd.build`")
    # PyTorch ships its own copy of the HIP runtime.  Loaded after this
    # library, it would be a second runtime in the process, and this
    # library's would then find no device; loaded first, both share it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = _c.CDLL(LIB_PATH)
    P = _c.POINTER
    sig = {
        "bmmc_strerror": (_c.c_char_p, [_i32]),
        "bmmc_last_error": (_c.c_char_p, []),
        "bmmc_version": (_i32, []),
        "bmmc_is_tiled": (_i32, [P(_u64), _i32, _i32, P(_u64)]),
        "bmmc_factorize": (_i32, [P(_u64), _u64, _i32, P(Plan)]),
        "bmmc_factorize_t": (_i32, [P(_u64), _u64, _i32, _i32, _i32, P(Plan)]),
        "bmmc_emulate": (_i32, [_vp, _vp, _i32, P(_u64), _u64, _i32, P(Options), P(EmuStats)]),
        "bmmc_compose": (_i32, [P(_u64), _u64, P(_u64), _u64, _i32, P(_u64), P(_u64)]),
        "bmmc_invert": (_i32, [P(_u64), _u64, _i32, P(_u64), P(_u64)]),
        "bmmc_parm_matrix": (_i32, [_u64, _i32, P(_u64), P(_u64)]),
        "bmmc_permute_seq": (_i32, [_vp, _vp, _i32, _i32, P(_u64), P(_u64), _i32, _vp]),
        "bmmc_sortnet_stages": (_i32, [_i32, P(_u64), _i32, P(_i32)]),
        "bmmc_sortnet": (_i32, [_vp, _vp, _i32, _i32, _i32, _vp]),
        "bmmc_sortnet_emulate": (_i32, [_vp, _vp, _i32, _i32, P(_i32)]),
        "bmmc_sortnet_passes": (_i32, [_i32, P(_i32), P(_i32)]),
        "bmmc_plan_ex": (_i32, [P(_u64), _u64, _i32, _i32, P(Options), P(Plan)]),
        "bmmc_factorize_ulp": (_i32, [P(_u64), _i32, P(_u64), P(_u64), P(_u64), P(_u64), P(_u64)]),
        "bmmc_permute": (_i32, [_vp, _vp, _i32, P(_u64), _u64, _i32, _vp]),
        "bmmc_permute_ex": (_i32, [_vp, _vp, _i32, P(_u64), _u64, _i32, P(Options), _vp]),
        "bmmc_permute_naive": (_i32, [_vp, _vp, _i32, P(_u64), _u64, _i32, _vp]),
        "bmmc_copy": (_i32, [_vp, _vp, _c.c_size_t, _vp]),
        "bmmc_copy_ex": (_i32, [_vp, _vp, _c.c_size_t, _i32, _i32, _vp]),
        "bmmc_permute_batched": (_i32, [P(Desc), _i32, _vp]),
        "bmmc_permute_batched_ex": (_i32, [P(Desc), _i32, P(BatchOptions), _vp]),
        "bmmc_batch_create": (_i32, [P(Desc), _i32, P(BatchOptions), P(_vp)]),
        "bmmc_batch_launch": (_i32, [_vp, _vp]),
        "bmmc_batch_destroy": (_i32, [_vp]),
        "bmmc_profile_begin": (_i32, []),
        "bmmc_profile_end": (_i32, [P(KernelStat), _i32]),
        "bmmc_autotune_batched": (_i32, [P(Desc), _i32, _vp, _i32, P(BatchOptions), P(_dbl)]),
        "bmmc_autotune": (_i32, [_i32, _i32, _i32, _vp, _i32, P(Options), P(_dbl)]),
        "bmmc_autotune_matrix": (_i32, [_vp, _vp, _i32, P(_u64), _u64, _i32, _vp, _i32, P(Options), P(_dbl)]),
        "bmmc_tune_clear_matrices": (_i32, []),
        "bmmc_tune_save": (_i32, [_c.c_char_p]),
        "bmmc_tune_lookup": (_i32, [_i32, _i32, _i32, P(_u64), P(Options)]),
        "bmmc_tune_lookup_batched": (_i32, [P(Desc), _i32, P(BatchOptions)]),
        "bmmc_tune_load": (_i32, [_c.c_char_p]),
        "bmmc_server_create": (_i32, [P(ServerOptions), P(_vp)]),
        "bmmc_server_destroy": (_i32, [_vp]),
        "bmmc_server_submit": (_i32, [_vp, P(Desc), _i64, P(_i64)]),
        "bmmc_server_poll": (_i32, [_vp, _i64, _i32, P(_i64), P(_vp)]),
        "bmmc_server_release": (_i32, [_vp, _i64]),
        "bmmc_server_drain": (_i32, [_vp]),
        "bmmc_server_stats": (_i32, [_vp, P(ServerStats)]),
        "bmmc_server_now_ns": (_i64, []),
        "bmmc_server_reset_stats": (_i32, [_vp]),
        "bmmc_serve_direct": (_i32, [P(Desc), P(_i64), _i32, _i32, P(ServerStats)]),
        "bmmc_permute_batched_noalloc": (_i32, [P(Desc), _i32, P(BatchOptions), _vp]),
        "bmmc_noalloc_table_bytes": (_c.c_size_t, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_names():
    return [
        "bmmc_strerror", "bmmc_last_error", "bmmc_version", "bmmc_is_tiled", "bmmc_factorize",
        "bmmc_factorize_t", "bmmc_plan_ex", "bmmc_factorize_ulp", "bmmc_emulate",
        "bmmc_compose", "bmmc_invert", "bmmc_parm_matrix", "bmmc_permute_seq", "bmmc_permute", "bmmc_permute_ex", "bmmc_permute_naive",
        "bmmc_copy", "bmmc_copy_ex", "bmmc_permute_batched", "bmmc_permute_batched_ex",
        "bmmc_batch_create", "bmmc_batch_launch", "bmmc_batch_destroy",
        "bmmc_profile_begin", "bmmc_profile_end", "bmmc_autotune_batched", "bmmc_autotune",
        "bmmc_tune_save", "bmmc_tune_load", "bmmc_server_create", "bmmc_server_destroy",
        "bmmc_server_submit", "bmmc_server_poll", "bmmc_server_release", "bmmc_server_drain",
        "bmmc_server_stats", "bmmc_server_now_ns", "bmmc_sortnet_stages", "bmmc_sortnet",
        "bmmc_tune_lookup", "bmmc_sortnet_emulate", "bmmc_sortnet_passes", "bmmc_tune_lookup_batched",
        "bmmc_server_reset_stats", "bmmc_autotune_matrix", "bmmc_tune_clear_matrices",
        "bmmc_serve_direct", "bmmc_permute_batched_noalloc", "bmmc_noalloc_table_bytes",
    ]


# ------------------------------------------------------------- marshalling

def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if hasattr(x, "ctypes"):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take a device address from {type(x)!r}")


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s or None
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream) or None
    raise TypeError(f"cannot take a stream from {type(s)!r}")


def _rows(A_rows, n):
    arr = (_u64 * max(n, 1))()
    for i in range(n):
        arr[i] = int(A_rows[i])
    return arr


def _check(status: int):
    if status < 0:
        raise BmmcError(status, lib().bmmc_last_error().decode(errors="replace"))
    return status


def _options(opts):
    if opts is None:
        return None
    if isinstance(opts, Options):
        return _c.byref(opts)
    o = Options()
    for k, v in dict(opts).items():
        setattr(o, k, int(v))
    return _c.byref(o)


# ------------------------------------------------------------ entry points

def bmmc_strerror(status: int) -> str:
    return lib().bmmc_strerror(status).decode()


def bmmc_version() -> int:
    return lib().bmmc_version()


def bmmc_is_tiled(A_rows, n: int, t: int):
    """(tiled?, tile row mask)."""
    mask = _u64(0)
    r = _check(lib().bmmc_is_tiled(_rows(A_rows, n), n, t, _c.byref(mask)))
    return bool(r), int(mask.value)


def bmmc_factorize(A_rows, c: int, n: int) -> Plan:
    p = Plan()
    _check(lib().bmmc_factorize(_rows(A_rows, n), c, n, _c.byref(p)))
    return p


def bmmc_factorize_t(A_rows, c: int, n: int, t: int, elem_bytes: int = 4) -> Plan:
    p = Plan()
    _check(lib().bmmc_factorize_t(_rows(A_rows, n), c, n, t, elem_bytes, _c.byref(p)))
    return p


def bmmc_plan_ex(A_rows, c: int, n: int, elem_bytes: int = 4, opts=None) -> Plan:
    p = Plan()
    _check(lib().bmmc_plan_ex(_rows(A_rows, n), c, n, elem_bytes, _options(opts), _c.byref(p)))
    return p


def bmmc_factorize_ulp(A_rows, n: int):
    """dict of U, L, P, T1, T2 (lists of n row words) with A = U.L.P = T1.T2."""
    outs = {k: (_u64 * max(n, 1))() for k in ("U", "L", "P", "T1", "T2")}
    _check(lib().bmmc_factorize_ulp(_rows(A_rows, n), n, outs["U"], outs["L"], outs["P"],
                                    outs["T1"], outs["T2"]))
    return {k: [int(v[i]) for i in range(n)] for k, v in outs.items()}


def bmmc_compose(A_rows, c: int, B_rows, d: int, n: int):
    """(rows, c) of bmmc(A, c) after bmmc(B, d)."""
    out = (_u64 * max(n, 1))()
    oc = _u64(0)
    _check(lib().bmmc_compose(_rows(A_rows, n), c, _rows(B_rows, n), d, n, out, _c.byref(oc)))
    return [int(out[i]) for i in range(n)], int(oc.value)


def bmmc_invert(A_rows, c: int, n: int):
    out = (_u64 * max(n, 1))()
    oc = _u64(0)
    _check(lib().bmmc_invert(_rows(A_rows, n), c, n, out, _c.byref(oc)))
    return [int(out[i]) for i in range(n)], int(oc.value)


def bmmc_parm_matrix(mask: int, n: int):
    """(A, A^-1) rows for parm with this mask."""
    a = (_u64 * max(n, 1))()
    ai = (_u64 * max(n, 1))()
    _check(lib().bmmc_parm_matrix(mask, n, a, ai))
    return [int(a[i]) for i in range(n)], [int(ai[i]) for i in range(n)]


def bmmc_permute_seq(inp, out, n: int, seq, elem_bytes: int, stream=None):
    """seq: list of (rows, c), applied first to last, fused into one permutation."""
    count = len(seq)
    rows = (_u64 * max(count * n, 1))()
    cs = (_u64 * max(count, 1))()
    for k, (r, c) in enumerate(seq):
        for i in range(n):
            rows[k * n + i] = int(r[i])
        cs[k] = int(c)
    _check(lib().bmmc_permute_seq(_ptr(inp), _ptr(out), n, count, rows, cs, elem_bytes, _stream(stream)))


def bmmc_sortnet_stages(n: int):
    """The compiled network: list of S + 1 matrices (rows), S = n(n+1)/2
    compare-exchange columns between them."""
    count = _c.c_int(0)
    _check(lib().bmmc_sortnet_stages(n, None, 0, _c.byref(count)))
    rows = (_u64 * max(count.value * n, 1))()
    _check(lib().bmmc_sortnet_stages(n, rows, count.value, _c.byref(count)))
    return [[int(rows[s * n + i]) for i in range(n)] for s in range(count.value)]


def bmmc_sortnet_passes(n: int):
    """(passes, most columns in one pass) of the compiled network."""
    p, c = _c.c_int(0), _c.c_int(0)
    _check(lib().bmmc_sortnet_passes(n, _c.byref(p), _c.byref(c)))
    return p.value, c.value


def bmmc_sortnet_emulate(inp, out, n: int, key_type: int = KEY_I32) -> int:
    """Host emulation of the network's passes on numpy arrays; returns the
    number of passes."""
    count = _c.c_int(0)
    _check(lib().bmmc_sortnet_emulate(_ptr(inp), _ptr(out), n, key_type, _c.byref(count)))
    return count.value


def bmmc_sortnet(inp, out, n: int, key_type: int = KEY_I32, method: int = SORTNET_PASSES, stream=None):
    _check(lib().bmmc_sortnet(_ptr(inp), _ptr(out), n, key_type, method, _stream(stream)))


def bmmc_emulate(inp, out, n: int, A_rows, c: int, elem_bytes: int, opts=None) -> dict:
    """Host emulation of the kernels; inp/out are host buffers (numpy arrays)."""
    st = EmuStats()
    _check(lib().bmmc_emulate(_ptr(inp), _ptr(out), n, _rows(A_rows, n), c, elem_bytes,
                              _options(opts), _c.byref(st)))
    return st.as_dict()


def bmmc_permute(inp, out, n: int, A_rows, c: int, elem_bytes: int, stream=None):
    _check(lib().bmmc_permute(_ptr(inp), _ptr(out), n, _rows(A_rows, n), c, elem_bytes,
                              _stream(stream)))


def bmmc_permute_ex(inp, out, n: int, A_rows, c: int, elem_bytes: int, opts=None, stream=None):
    _check(lib().bmmc_permute_ex(_ptr(inp), _ptr(out), n, _rows(A_rows, n), c, elem_bytes,
                                 _options(opts), _stream(stream)))


def bmmc_permute_naive(inp, out, n: int, A_rows, c: int, elem_bytes: int, stream=None):
    _check(lib().bmmc_permute_naive(_ptr(inp), _ptr(out), n, _rows(A_rows, n), c, elem_bytes,
                                    _stream(stream)))


def bmmc_copy(inp, out, nbytes: int, stream=None):
    _check(lib().bmmc_copy(_ptr(inp), _ptr(out), nbytes, _stream(stream)))


def bmmc_copy_ex(inp, out, nbytes: int, vpt: int = 4, hints: int = 0, stream=None):
    _check(lib().bmmc_copy_ex(_ptr(inp), _ptr(out), nbytes, vpt, hints, _stream(stream)))


class DescBatch:
    """The descriptors of a batch marshalled once, for repeated calls (every
    batched entry point accepts one in place of the list of items)."""

    def __init__(self, items):
        self.arr, self.keep, self.count = make_descs(items)


def make_descs(items):
    """items: iterable of (in, out, n, elem_bytes, A_rows, c), or a DescBatch.
    Returns a ctypes array of Desc plus the row storage it points into (keep
    both alive) and the count.  All rows go into one uint64 buffer."""
    import numpy as np
    if isinstance(items, DescBatch):
        return items.arr, items.keep, items.count
    items = list(items)
    count = len(items)
    arr = (Desc * max(count, 1))()
    total = sum(int(it[2]) for it in items)
    rows = np.zeros(max(total, 1), dtype=np.uint64)
    base = rows.ctypes.data
    off = 0
    for k, (i, o, n, w, r, c) in enumerate(items):
        n = int(n)
        if n:
            rows[off:off + n] = np.asarray([int(v) for v in r[:n]], dtype=np.uint64)
        d = arr[k]
        d.in_ = _ptr(i)
        d.out = _ptr(o)
        d.n = n
        d.elem_bytes = w
        d.A_rows = _c.cast(_c.c_void_p(base + 8 * off), _c.POINTER(_u64))
        d.c = c
        off += n
    return arr, rows, count


def _batch_options(opts):
    if opts is None:
        return None
    if isinstance(opts, BatchOptions):
        return _c.byref(opts)
    o = BatchOptions()
    for k, v in dict(opts).items():
        setattr(o, k, int(v))
    return _c.byref(o)


class PreparedBatch:
    """A batch resident on the device (bmmc_batch_create); launch() replays
    its graph.  The caller keeps the arrays alive until close()."""

    def __init__(self, items, opts=None):
        arr, keep, count = make_descs(items)
        h = _vp()
        _check(lib().bmmc_batch_create(arr, count, _batch_options(opts), _c.byref(h)))
        self.handle = h.value

    def launch(self, stream=None):
        _check(lib().bmmc_batch_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            _check(lib().bmmc_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bmmc_batch_create(items, opts=None) -> PreparedBatch:
    return PreparedBatch(items, opts)


def bmmc_permute_batched(items, stream=None, opts=None):
    arr, keep, count = make_descs(items)
    if opts is None:
        _check(lib().bmmc_permute_batched(arr, count, _stream(stream)))
    else:
        _check(lib().bmmc_permute_batched_ex(arr, count, _batch_options(opts), _stream(stream)))
    del keep


def bmmc_permute_batched_noalloc(items, stream=None, opts=None):
    """bmmc_permute_batched without device allocation (the library's fixed
    table; calls on one device must not overlap)."""
    arr, keep, count = make_descs(items)
    _check(lib().bmmc_permute_batched_noalloc(arr, count, _batch_options(opts), _stream(stream)))
    del keep


def bmmc_noalloc_table_bytes() -> int:
    return int(lib().bmmc_noalloc_table_bytes())


def bmmc_profile_begin():
    _check(lib().bmmc_profile_begin())


def bmmc_profile_end(max_kernels: int = 64):
    arr = (KernelStat * max_kernels)()
    k = _check(lib().bmmc_profile_end(arr, max_kernels))
    return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                   "bytes": arr[i].bytes} for i in range(k)}


def bmmc_autotune(n: int, elem_bytes: int, method: int = METHOD_AUTO, stream=None, reps: int = 5):
    """Time the tile shapes for random permutations of this size; the best is
    cached and used by later calls.  Returns (options dict, best ms)."""
    o = Options()
    ms = _dbl(0)
    _check(lib().bmmc_autotune(n, elem_bytes, method, _stream(stream), reps, _c.byref(o),
                               _c.byref(ms)))
    return {f: getattr(o, f) for f, _ in Options._fields_ if f != "reserved"}, ms.value


def bmmc_autotune_matrix(inp, out, n: int, A_rows, c: int, elem_bytes: int, stream=None, reps: int = 3):
    """Time settings for this very matrix on these buffers; the best is kept
    for later calls with this matrix.  Returns (options dict, ms per call)."""
    o = Options()
    ms = _dbl(0)
    _check(lib().bmmc_autotune_matrix(_ptr(inp), _ptr(out), n, _rows(A_rows, n), c, elem_bytes, _stream(stream),
                                      reps, _c.byref(o), _c.byref(ms)))
    return {f: getattr(o, f) for f, _ in Options._fields_ if f != "reserved"}, ms.value


def bmmc_tune_clear_matrices():
    _check(lib().bmmc_tune_clear_matrices())


def bmmc_tune_lookup(n: int, elem_bytes: int, A_rows, method: int = METHOD_AUTO):
    """The tuned options of `method` for this matrix, else for its class
    (dict), or None when nothing is tuned for it."""
    o = Options()
    r = lib().bmmc_tune_lookup(n, elem_bytes, method, _rows(A_rows, n), _c.byref(o))
    if r < 0:
        _check(r)
    if r == 0:
        return None
    return {f: getattr(o, f) for f, _ in Options._fields_ if f != "reserved"}


def bmmc_tune_lookup_batched(items):
    """The tuned batch options for batches of this size histogram (dict), or
    None."""
    arr, keep, count = make_descs(items)
    o = BatchOptions()
    r = _check(lib().bmmc_tune_lookup_batched(arr, count, _c.byref(o)))
    del keep
    if r == 0:
        return None
    return {f: getattr(o, f) for f, _ in BatchOptions._fields_ if f != "reserved"}


def bmmc_autotune_batched(items, stream=None, reps: int = 3):
    arr, keep, count = make_descs(items)
    o = BatchOptions()
    ms = _dbl(0)
    _check(lib().bmmc_autotune_batched(arr, count, _stream(stream), reps, _c.byref(o), _c.byref(ms)))
    del keep
    return {f: getattr(o, f) for f, _ in BatchOptions._fields_ if f != "reserved"}, ms.value


def bmmc_tune_save(path: str):
    _check(lib().bmmc_tune_save(path.encode()))


def bmmc_tune_load(path: str):
    return _check(lib().bmmc_tune_load(path.encode()))


# ---------------------------------------------------------------- serving

def bmmc_server_create(budget_bytes: int, streams: int = 4, max_batch: int = 0,
                       own_outputs: int = 1, method: int = METHOD_AUTO, use_graph: int = 0,
                       direct_max: int = 0, solo_log2: int = 0):
    """own_outputs: 0 caller passes out, 1 server allocates and keeps it until
    release, 2 server allocates and drops it at completion."""
    o = ServerOptions()
    o.budget_bytes = budget_bytes
    o.streams = streams
    o.max_batch = max_batch
    o.own_outputs = int(own_outputs)
    o.method = method
    o.use_graph = int(use_graph)
    o.direct_max = int(direct_max)
    o.solo_log2 = int(solo_log2)
    h = _vp()
    _check(lib().bmmc_server_create(_c.byref(o), _c.byref(h)))
    return h.value


def bmmc_server_reset_stats(handle):
    _check(lib().bmmc_server_reset_stats(handle))


def bmmc_server_destroy(handle):
    _check(lib().bmmc_server_destroy(handle))


def bmmc_server_submit(handle, inp, out, n: int, A_rows, c: int, elem_bytes: int,
                       arrival_ns: int = 0) -> int:
    arr, keep, _ = make_descs([(inp, out, n, elem_bytes, A_rows, c)])
    ticket = _i64(0)
    _check(lib().bmmc_server_submit(handle, arr, arrival_ns, _c.byref(ticket)))
    del keep
    return int(ticket.value)


def bmmc_server_submit_many(handle, descs: "DescBatch", arrival_ns) -> list:
    """Submit every descriptor of a DescBatch (marshalled beforehand), the
    k-th arriving at arrival_ns[k]; one library call each, tickets in order."""
    L = lib()
    ticket = _i64(0)
    out = []
    for k in range(descs.count):
        _check(L.bmmc_server_submit(handle, _c.byref(descs.arr[k]), int(arrival_ns[k]), _c.byref(ticket)))
        out.append(int(ticket.value))
    return out


def bmmc_server_poll(handle, ticket: int, wait: bool = False):
    """None while pending; else (completion time ns, output device address)."""
    done = _i64(0)
    out = _vp()
    st = lib().bmmc_server_poll(handle, ticket, 1 if wait else 0, _c.byref(done), _c.byref(out))
    if st == -9:  # BMMC_ERR_BUSY
        return None
    _check(st)
    return int(done.value), int(out.value or 0)


def bmmc_server_release(handle, ticket: int):
    _check(lib().bmmc_server_release(handle, ticket))


def bmmc_server_drain(handle):
    _check(lib().bmmc_server_drain(handle))


def bmmc_server_stats(handle) -> dict:
    s = ServerStats()
    _check(lib().bmmc_server_stats(handle, _c.byref(s)))
    return {f: (getattr(s, f) if f != "reserved" else None) for f, _ in ServerStats._fields_
            if f != "reserved"}


def bmmc_server_now_ns() -> int:
    return int(lib().bmmc_server_now_ns())


def bmmc_serve_direct(descs: "DescBatch", arrival_ns, streams: int = 4) -> dict:
    """The unbatched baseline: each request k as its own bmmc_permute call at
    arrival_ns[k] on stream k mod `streams` (one issuing thread per stream);
    statistics as bmmc_server_stats."""
    arr, keep, count = make_descs(descs)
    arrivals = (_i64 * max(count, 1))(*[int(v) for v in arrival_ns])
    s = ServerStats()
    _check(lib().bmmc_serve_direct(arr, arrivals, count, streams, _c.byref(s)))
    del keep
    return {f: getattr(s, f) for f, _ in ServerStats._fields_ if f != "reserved"}
