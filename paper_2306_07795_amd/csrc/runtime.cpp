// C entry points for planning and the single-array device path, plus the
// runtime pieces they share (plan cache, per-stream scratch, profiling).
#include "runtime.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <tuple>
#include <map>

#include "kernels.hpp"

namespace bmmc {

static thread_local std::string g_last_error;

int set_error(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    return set_error(BMMC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool PlanKey::operator==(const PlanKey& o) const {
    if (n != o.n || w != o.w || method != o.method || t != o.t || a != o.a || b != o.b || nt != o.nt ||
        iters != o.iters || swizzle != o.swizzle || tb_mix != o.tb_mix || iter_mix != o.iter_mix || c != o.c)
        return false;
    for (int i = 0; i < n; i++)
        if (rows[i] != o.rows[i]) return false;
    return true;
}

size_t PlanKeyHash::operator()(const PlanKey& k) const {
    uint64_t h = 0xcbf29ce484222325ull;
    auto mixin = [&](uint64_t v) {
        h ^= v;
        h *= 0x100000001b3ull;
        h ^= h >> 29;
    };
    mixin((uint64_t)k.n | ((uint64_t)k.w << 8) | ((uint64_t)k.method << 16) | ((uint64_t)k.t << 24) |
          ((uint64_t)k.nt << 32) | ((uint64_t)k.iters << 48) | ((uint64_t)k.swizzle << 60) |
          ((uint64_t)(k.tb_mix & 1) << 62) | ((uint64_t)k.iter_mix << 63));
    mixin(k.c ^ ((uint64_t)k.a << 56) ^ ((uint64_t)k.b << 48) ^ ((uint64_t)(k.tb_mix >> 4) << 40));
    for (int i = 0; i < k.n; i++) mixin(k.rows[i]);
    return (size_t)h;
}

DeviceState* device_state(int* status) {
    static std::mutex mu;
    static DeviceState* states[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) {
        *status = hip_fail(e == hipSuccess ? hipErrorInvalidDevice : e, "hipGetDevice");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!states[dev]) {
        auto* s = new DeviceState();
        s->device = dev;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        s->cu_count = cus;
        if (const char* x = std::getenv("BMMC_XCDS")) s->xcds = std::atoi(x) > 0 ? std::atoi(x) : 8;
        states[dev] = s;
    }
    *status = BMMC_OK;
    return states[dev];
}

int get_plan(DeviceState* ds, const uint64_t* rows, uint64_t c, int n, int w, const PlanOptions& o,
             std::shared_ptr<const Plan>* out) {
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    if (n > 0 && !rows) return set_error(BMMC_ERR_ARG, "A_rows is NULL");
    PlanKey key;
    std::memset(&key, 0, sizeof(key));
    key.n = n;
    key.w = w;
    key.method = o.method;
    key.t = o.t;
    key.a = o.a;
    key.b = o.b;
    key.nt = o.shape_given ? o.shape.nt : 0;
    key.iters = o.shape_given ? o.shape.iters : 0;
    key.swizzle = o.swizzle;
    key.tb_mix = o.tb_mix;
    key.iter_mix = o.iter_mix;
    key.c = c;
    for (int i = 0; i < n; i++) key.rows[i] = rows[i];
    {
        std::lock_guard<std::mutex> lk(ds->mu);
        auto it = ds->plans.find(key);
        if (it != ds->plans.end()) {
            *out = it->second;
            return BMMC_OK;
        }
    }
    auto plan = std::make_shared<Plan>();
    int st = make_plan(rows, c, n, w, o, plan.get());
    if (st != BMMC_OK) {
        switch (st) {
            case BMMC_ERR_SINGULAR: return set_error(st, "A is singular over F_2");
            case BMMC_ERR_ARG: return set_error(st, "bad argument: width %d, or bits of A or c at positions >= n = %d", w, n);
            case BMMC_ERR_RANGE: return set_error(st, "tile geometry out of range (n = %d, t = %d, w = %d)", n, o.t, w);
            default: return set_error(st, "planner failed (%d)", st);
        }
    }
    // A full cache is emptied by swapping it out under the lock and freeing
    // its plans after the lock is released: launches on other threads wait
    // for this lock, and freeing thousands of plans takes milliseconds.
    decltype(ds->plans) old;
    {
        std::lock_guard<std::mutex> lk(ds->mu);
        if (ds->plans.size() > 8192) old.swap(ds->plans);
        ds->plans[key] = plan;
    }
    *out = plan;
    return BMMC_OK;
}

int get_scratch(DeviceState* ds, hipStream_t stream, size_t bytes, void** out) {
    auto& s = ds->scratch[stream];
    if (s.bytes < bytes) {
        if (s.ptr) {
            // earlier work on this stream may still read the old buffer
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            hipFree(s.ptr);
            s.ptr = nullptr;
            s.bytes = 0;
        }
        hipError_t e = hipMalloc(&s.ptr, bytes);
        if (e != hipSuccess) {
            s.ptr = nullptr;
            (void)hipGetLastError();
            return set_error(BMMC_ERR_NOMEM, "scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
        }
        s.bytes = bytes;
    }
    *out = s.ptr;
    return BMMC_OK;
}

LaunchScope::LaunchScope(DeviceState* d, hipStream_t s, const char* name, double bytes, bool one_kernel)
    : ds(d), stream(s) {
    if (!ds->profiling) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return;
    }
    ProfileEvent pe;
    pe.name = name;
    pe.bytes = bytes;
    for (hipEvent_t* slot : {&pe.start, &pe.stop}) {
        if (!ds->event_pool.empty()) {
            *slot = ds->event_pool.back();
            ds->event_pool.pop_back();
        } else if (hipEventCreate(slot) != hipSuccess) {
            return;
        }
    }
    ds->events.push_back(pe);
    if (one_kernel) {
        set_kernel_events(pe.start, pe.stop);
        bound = true;
    } else {
        hipEventRecord(pe.start, stream);
        stop = pe.stop;
    }
}

LaunchScope::~LaunchScope() {
    if (bound) {
        if (kernel_events_pending()) {
            // nothing was launched (an error before the launch): drop the entry
            set_kernel_events(nullptr, nullptr);
            ds->event_pool.push_back(ds->events.back().start);
            ds->event_pool.push_back(ds->events.back().stop);
            ds->events.pop_back();
        }
    } else if (stop) {
        hipEventRecord(stop, stream);
    }
}

// Library defaults of the general one-pass tile (BMMC_METHOD_AUTO and
// _ONEPASS) for 4- and 8-byte arrays larger than 8 MiB, by size: measured
// on gfx950 over random matrices and bit permutations of 2^21..2^28
// elements.  Up to 256 MiB an array fits the last-level cache, where
// non-temporal stores with cached loads and, from 32 MiB, a persistent grid
// of twice the resident work-groups are best; beyond it both sides stream
// through HBM with non-temporal loads and stores.  The tiles are ordered so
// that neighbouring tiles write neighbouring runs.
namespace {
struct SizeDefault {
    int w;
    size_t lo, hi;  // lo < bytes <= hi
    int nt, iters, a, b, hints, order;
    bool persistent;
};
const SizeDefault kSizeDefaults[] = {
    {4, (size_t)8 << 20, (size_t)32 << 20, 256, 8, 5, 8, 2, 4 + 16 * 6, false},
    {4, (size_t)32 << 20, (size_t)256 << 20, 512, 8, 6, 7, 2, 4 + 16 * 15, true},
    {4, (size_t)256 << 20, ~(size_t)0, 1024, 4, 6, 8, 3, 4 + 16 * 7, false},
    {8, (size_t)8 << 20, (size_t)32 << 20, 256, 8, 7, 5, 2, 4 + 16 * 15, false},
    {8, (size_t)32 << 20, (size_t)256 << 20, 1024, 4, 5, 7, 2, 1 + 16 * 8, true},
    {8, (size_t)256 << 20, ~(size_t)0, 1024, 4, 5, 7, 3, 4 + 16 * 6, false},
};
}  // namespace

// Resident work-groups per CU of a tiled kernel shape, asked of the runtime
// once per shape (the answer does not change) rather than on every call.
static int cached_occupancy(int w, int nt, int iters) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> known;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find({w, nt, iters});
    if (it != known.end()) return it->second;
    const int occ = tiled_occupancy(w, nt, iters, 0);
    known[{w, nt, iters}] = occ;
    return occ;
}

bmmc_options_t effective_options(const DeviceState* ds, int n, int w, const bmmc_options_t* o) {
    bmmc_options_t e;
    if (o)
        e = *o;
    else
        std::memset(&e, 0, sizeof(e));
    if (e.method != BMMC_METHOD_AUTO && e.method != BMMC_METHOD_ONEPASS) return e;
    const size_t bytes = ((size_t)1 << n) * (size_t)w;
    const SizeDefault* d = nullptr;
    for (const SizeDefault& s : kSizeDefaults)
        if (s.w == w && bytes > s.lo && bytes <= s.hi) {
            d = &s;
            break;
        }
    if (!d) return e;
    // the runs and the tile shape go together: only when none is given
    const bool shape_free = !e.threads && !e.iters && !e.t && !e.run_in && !e.run_out;
    if (shape_free) {
        e.threads = d->nt;
        e.iters = d->iters;
        e.run_in = d->a;
        e.run_out = d->b;
        e.t = d->a < d->b ? d->a : d->b;
    }
    if (!e.hints) e.hints = d->hints;
    if (!e.tile_order) e.tile_order = d->order;
    if (!e.grid && d->persistent && ds && ds->cu_count > 0) {
        KernelShape ks = general_shape(w);  // the general tile's shape unless given
        ks.nt = e.threads ? e.threads : ks.nt;
        ks.iters = e.iters ? e.iters : ks.iters;
        const int occ = cached_occupancy(w, ks.nt, ks.iters);
        if (occ > 0) e.grid = 2 * ds->cu_count * occ;
    }
    return e;
}

bool keeps_block_bits(const uint64_t* rows, int n, int w) {
    int blk = 12;
    for (int wb = w; wb > 1; wb >>= 1) blk--;
    if (blk < 0 || blk + 3 > n || !rows) return false;
    // rows of the block bits within the block columns (A invertible makes
    // that 3 x 3 block invertible)
    for (int i = blk; i < blk + 3; i++)
        if (rows[i] & ~(7ull << blk)) return false;
    return true;
}

void dealt_default(bmmc_options_t* e, const uint64_t* rows, int n, int w) {
    const size_t bytes = ((size_t)1 << n) * (size_t)w;
    if (bytes <= kDealtFrom || !keeps_block_bits(rows, n, w)) return;
    e->tile_order = 256 + 4;  // dealt output blocks, plain order
    if (w == 4 || w == 8) {
        // 16 KiB tiles (512 threads x 2 vectors), one work-group each,
        // non-temporal loads and cached stores: the fastest dealt setting
        // measured for these matrices beyond the last-level cache
        e->threads = 512;
        e->iters = 2;
        e->run_in = w == 4 ? 5 : 4;
        e->run_out = 7;
        e->t = e->run_in;
        e->hints = 1;
        e->grid = -1;
    }
}

int tile_order_mix(int t) {
    if (!t) return -1;
    return ((t & 4) ? 0 : ((t >> 1) & 1)) | (((t >> 4) & 15) << 4) | (t & 256);
}

PlanOptions plan_options(const bmmc_options_t* o, int w) {
    PlanOptions p;
    p.shape = default_shape(w);
    if (!o) return p;
    p.method = o->method;
    if (o->t) p.t = o->t;
    if (o->run_in) p.a = o->run_in;
    if (o->run_out) p.b = o->run_out;
    p.swizzle = o->swizzle < 0 ? 0 : 1;
    p.tb_mix = tile_order_mix(o->tile_order);
    p.iter_mix = (o->tile_order >> 3) & 1;
    if (o->threads > 0 || o->iters > 0) {
        // a shape given in part takes the rest from the default of its kind
        const bool general = o->method == BMMC_METHOD_ONEPASS || o->method == BMMC_METHOD_AUTO;
        p.shape = general ? general_shape(w) : default_shape(w);
        p.shape_given = true;
    }
    if (o->threads > 0) p.shape.nt = o->threads;
    if (o->iters > 0) p.shape.iters = o->iters;
    return p;
}

int resolve_hints(const bmmc_options_t* o, size_t bytes) {
    const int h = o ? o->hints : 0;
    const int scratch_cached = h & 8;
    const int base = h & ~8;
    // default: non-temporal loads and stores from 64 MiB; a two-pass plan's
    // scratch through the caches while it fits the 256 MB last-level cache
    if (base == 0)
        return (bytes >= ((size_t)64 << 20) ? 3 : 0) | (bytes <= ((size_t)256 << 20) ? 8 : 0) | scratch_cached;
    if (base & 4) return scratch_cached;
    return (base & 3) | scratch_cached;
}

int resolve_order(const bmmc_options_t* o) {
    const int t = o ? o->tile_order : 0;
    if (t == 0 || (t & 4)) return 0;
    return t & 1;  // XCD-contiguous tiles; the mixing bit lives in the plan
}

// Name of the tiled kernel instance (template arguments), shared by both
// passes of a plan.
static void kernel_name(char* buf, size_t len, const Plan& p, int hints) {
    snprintf(buf, len, "k_tiled<%d,%d,%d,%d>", p.w, p.shape.nt, p.shape.iters, hints);
}

int enqueue_plan(DeviceState* ds, const Plan& plan, const void* in, void* out, hipStream_t stream,
                 uint32_t grid, int hints, int order, void* scratch) {
    const size_t bytes = ((size_t)1 << plan.n) * (size_t)plan.w;
    hipError_t e;
    if (plan.npass == 0) {
        LaunchScope ls(ds, stream, "k_copy<4,0>", 2.0 * bytes);
        e = launch_copy(in, out, bytes, stream);
        return e == hipSuccess ? BMMC_OK : hip_fail(e, "copy launch");
    }
    if (plan.naive) {
        NaiveArgs na;
        std::memset(&na, 0, sizeof(na));
        na.n = (uint32_t)plan.n;
        na.c = (uint32_t)plan.c;
        for (int j = 0; j < plan.n; j++) na.col[j] = (uint32_t)plan.A.col(j);
        LaunchScope ls(ds, stream, "k_naive", 2.0 * bytes);
        e = launch_naive(plan.w, plan.n, in, out, na, stream);
        return e == hipSuccess ? BMMC_OK : hip_fail(e, "naive launch");
    }
    const KernelShape& ks = plan.shape;
    if (!tiled_kernel_available(plan.w, ks.nt, ks.iters, hints & 3))
        return set_error(BMMC_ERR_RANGE, "no tiled kernel for w=%d threads=%d iters=%d hints=%d", plan.w, ks.nt,
                         ks.iters, hints & 3);
    void* mid = scratch;
    if (plan.npass == 2 && !mid) {
        int st = get_scratch(ds, stream, bytes, &mid);
        if (st != BMMC_OK) return st;
    }
    char name[64];
    for (int k = 0; k < plan.npass; k++) {
        const PassTables& tab = plan.pass[k].tab;
        const void* src = (k == 0) ? in : mid;
        void* dst = (k == plan.npass - 1) ? out : mid;
        const uint32_t ntiles = 1u << tab.ntb;
        // hints bit 8 (two passes): the scratch array goes through the
        // caches -- cached stores in the first pass, cached loads in the
        // second -- so that the second pass finds what fits of it there
        int hk = hints & 3;
        if ((hints & 8) && plan.npass == 2) hk &= (k == 0) ? 1 : 2;
        kernel_name(name, sizeof(name), plan, hk);
        LaunchScope ls(ds, stream, name, 2.0 * bytes);
        e = launch_tiled(plan.w, ks.nt, ks.iters, hk, src, dst, tab, ntiles, grid,
                         (order & 1) ? (uint32_t)ds->xcds : 0u, stream);
        if (e != hipSuccess) return hip_fail(e, "tiled launch");
    }
    return BMMC_OK;
}

int validate_buffers(const void* in, const void* out, size_t bytes) {
    if (!in || !out) return set_error(BMMC_ERR_ARG, "in/out must not be NULL");
    if (((uintptr_t)in | (uintptr_t)out) & 15u) return set_error(BMMC_ERR_ARG, "in/out must be 16-byte aligned");
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a < b + bytes && b < a + bytes) return set_error(BMMC_ERR_ALIAS, "in and out overlap");
    return BMMC_OK;
}

static void fill_public_plan(const Plan& p, bmmc_plan_t* out) {
    std::memset(out, 0, sizeof(*out));
    out->n = p.n;
    out->t = p.t;
    out->elem_bytes = p.w;
    out->nfactors = p.npass;
    for (int k = 0; k < p.npass && k < 2; k++) {
        const PassPlan& pp = p.pass[k];
        if (p.naive) {
            for (int i = 0; i < p.n; i++) out->rows[k][i] = p.A.r[i];
            out->c[k] = p.c;
            continue;
        }
        for (int i = 0; i < p.n; i++) out->rows[k][i] = pp.T.r[i];
        out->c[k] = pp.c;
        out->col_mask[k] = pp.col_mask;
        out->tile_rows_mask[k] = pp.row_mask;
        out->iter_mask[k] = pp.iter_mask;
        out->tb_mask[k] = pp.tb_mask;
        out->n_over[k] = pp.n_over;
        out->tile_bits[k] = pp.d;
        out->coordinate[k] = pp.coordinate ? 1 : 0;
        out->lds_conflict_score[k] = pp.lds_score;
    }
}

int plan_single_array(DeviceState* ds, const bmmc_desc_t& d, int method, BatchArray* out) {
    bmmc_options_t o;
    std::memset(&o, 0, sizeof(o));
    o.method = method;
    // the options tuned for this matrix, else for its class, else the
    // defaults (with the default call's dealt output blocks where they apply)
    const bool own = method == BMMC_METHOD_AUTO && matrix_options(d.n, d.elem_bytes, d.A_rows, &o);
    if (!own) tuned_options(d.n, d.elem_bytes, method, matrix_class(d.A_rows, d.n), &o);
    bmmc_options_t eff = effective_options(ds, d.n, d.elem_bytes, &o);
    if (!own && method == BMMC_METHOD_AUTO) dealt_default(&eff, d.A_rows, d.n, d.elem_bytes);
    const int st = get_plan(ds, d.A_rows, d.c, d.n, d.elem_bytes, plan_options(&eff, d.elem_bytes), &out->plan);
    if (st != BMMC_OK) return st;
    out->in = d.in;
    out->out = d.out;
    out->scratch = nullptr;
    out->bytes = ((size_t)1 << d.n) * (size_t)d.elem_bytes;
    out->single = true;
    out->grid = (uint32_t)eff.grid;
    out->hints = resolve_hints(&eff, out->bytes);
    out->order = resolve_order(&eff);
    return BMMC_OK;
}

}  // namespace bmmc

using namespace bmmc;

extern "C" {

const char* bmmc_strerror(int status) {
    switch (status) {
        case BMMC_OK: return "ok";
        case BMMC_ERR_ARG: return "invalid argument";
        case BMMC_ERR_SINGULAR: return "matrix is singular over F_2";
        case BMMC_ERR_RANGE: return "size or tile parameter out of range";
        case BMMC_ERR_ALIAS: return "input and output overlap";
        case BMMC_ERR_NOMEM: return "out of memory";
        case BMMC_ERR_HIP: return "HIP runtime error";
        case BMMC_ERR_INTERNAL: return "internal planner error";
        case BMMC_ERR_NOTFOUND: return "unknown handle or ticket";
        case BMMC_ERR_BUSY: return "not finished";
        default: return "unknown status";
    }
}

const char* bmmc_last_error(void) { return g_last_error.c_str(); }

int bmmc_version(void) { return BMMC_VERSION; }

int bmmc_is_tiled(const uint64_t* A_rows, int n, int t, uint64_t* rows_mask_out) {
    if (n < 0 || n > 64 || t < 0 || t > n) return set_error(BMMC_ERR_RANGE, "n or t out of range");
    if (n > 0 && !A_rows) return set_error(BMMC_ERR_ARG, "A_rows is NULL");
    BitMat A;
    A.n = n;
    for (int i = 0; i < n; i++) A.r[i] = A_rows[i] & low_mask(n);
    if (rank(A) != n) return set_error(BMMC_ERR_SINGULAR, "A is singular over F_2");
    const uint64_t S = tiled_row_mask(A, t);
    if (rows_mask_out) *rows_mask_out = S;
    return popcount64(S) == t ? 1 : 0;
}

int bmmc_factorize_t(const uint64_t* A_rows, uint64_t c, int n, int t, int elem_bytes,
                     bmmc_plan_t* plan_out) {
    if (!plan_out) return set_error(BMMC_ERR_ARG, "plan_out is NULL");
    PlanOptions o;
    int w = elem_bytes > 0 ? elem_bytes : 4;
    o.method = kMethodTiled;  // the factorization of Section 5
    o.t = t;
    Plan p;
    int st = make_plan(A_rows, c, n, w, o, &p);
    if (st != BMMC_OK) return set_error(st, "planning failed: %s", bmmc_strerror(st));
    fill_public_plan(p, plan_out);
    return BMMC_OK;
}

int bmmc_plan_ex(const uint64_t* A_rows, uint64_t c, int n, int elem_bytes, const bmmc_options_t* opts,
                 bmmc_plan_t* plan_out) {
    if (!plan_out) return set_error(BMMC_ERR_ARG, "plan_out is NULL");
    if (!(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16))
        return set_error(BMMC_ERR_ARG, "elem_bytes = %d not in {1,2,4,8,16}", elem_bytes);
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    if (opts && (opts->tile_order < 0 || opts->tile_order > 511))
        return set_error(BMMC_ERR_ARG, "tile_order outside [0, 511]");
    const bmmc_options_t eff = effective_options(nullptr, n, elem_bytes, opts);
    PlanOptions o = plan_options(&eff, elem_bytes);
    Plan p;
    int st = make_plan(A_rows, c, n, elem_bytes, o, &p);
    if (st != BMMC_OK) return set_error(st, "planning failed: %s", bmmc_strerror(st));
    fill_public_plan(p, plan_out);
    return BMMC_OK;
}

int bmmc_factorize_ulp(const uint64_t* A_rows, int n, uint64_t* U, uint64_t* L, uint64_t* P, uint64_t* T1,
                       uint64_t* T2) {
    if (n < 1 || n > 64) return set_error(BMMC_ERR_RANGE, "n = %d outside [1, 64]", n);
    if (!A_rows) return set_error(BMMC_ERR_ARG, "A_rows is NULL");
    BitMat A;
    A.n = n;
    for (int i = 0; i < n; i++) {
        if (A_rows[i] & ~low_mask(n)) return set_error(BMMC_ERR_ARG, "row %d has bits at positions >= n", i);
        A.r[i] = A_rows[i];
    }
    BitMat u, l, pm, t1, t2;
    if (!factorize_ulp(A, &u, &l, &pm, &t1, &t2)) return set_error(BMMC_ERR_SINGULAR, "A is singular over F_2");
    for (int i = 0; i < n; i++) {
        if (U) U[i] = u.r[i];
        if (L) L[i] = l.r[i];
        if (P) P[i] = pm.r[i];
        if (T1) T1[i] = t1.r[i];
        if (T2) T2[i] = t2.r[i];
    }
    return BMMC_OK;
}

int bmmc_factorize(const uint64_t* A_rows, uint64_t c, int n, bmmc_plan_t* plan_out) {
    return bmmc_factorize_t(A_rows, c, n, 0, 4, plan_out);
}

int bmmc_permute_ex(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                    int elem_bytes, const bmmc_options_t* opts, void* stream) {
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    if (!(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16))
        return set_error(BMMC_ERR_ARG, "elem_bytes = %d not in {1,2,4,8,16}", elem_bytes);
    if (opts && (opts->tile_order < 0 || opts->tile_order > 511))
        return set_error(BMMC_ERR_ARG, "tile_order outside [0, 511]");
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    int st = validate_buffers(in, out, bytes);
    if (st != BMMC_OK) return st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    bmmc_options_t tuned;
    bool by_class = false;  // options of the matrix's class or the defaults, not the caller's or the matrix's own
    if (!opts) {
        by_class = !matrix_options(n, elem_bytes, A_rows, &tuned);
        if (!by_class || tuned_options(n, elem_bytes, BMMC_METHOD_AUTO, matrix_class(A_rows, n), &tuned))
            opts = &tuned;
    }
    bmmc_options_t eff = effective_options(ds, n, elem_bytes, opts);
    if (by_class) dealt_default(&eff, A_rows, n, elem_bytes);
    opts = &eff;
    PlanOptions po = plan_options(opts, elem_bytes);
    std::shared_ptr<const Plan> plan;
    st = get_plan(ds, A_rows, c, n, elem_bytes, po, &plan);
    if (st != BMMC_OK) return st;
    std::lock_guard<std::mutex> lk(ds->mu);
    return enqueue_plan(ds, *plan, in, out, (hipStream_t)stream, (uint32_t)opts->grid,
                        resolve_hints(opts, bytes), resolve_order(opts));
}

int bmmc_permute(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                 int elem_bytes, void* stream) {
    return bmmc_permute_ex(in, out, n, A_rows, c, elem_bytes, nullptr, stream);
}

int bmmc_permute_naive(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                       int elem_bytes, void* stream) {
    bmmc_options_t o;
    std::memset(&o, 0, sizeof(o));
    o.method = BMMC_METHOD_NAIVE;
    return bmmc_permute_ex(in, out, n, A_rows, c, elem_bytes, &o, stream);
}

int bmmc_copy_ex(const void* in, void* out, size_t bytes, int vpt, int hints, void* stream) {
    int st = validate_buffers(in, out, bytes);
    if (st != BMMC_OK) return st;
    if (!(vpt == 1 || vpt == 2 || vpt == 4 || vpt == 8) || hints < 0 || hints > 3)
        return set_error(BMMC_ERR_ARG, "vpt must be 1, 2, 4 or 8 and hints 0..3");
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    std::lock_guard<std::mutex> lk(ds->mu);
    char name[32];
    snprintf(name, sizeof(name), "k_copy<%d,%d>", vpt, hints);
    LaunchScope ls(ds, (hipStream_t)stream, name, 2.0 * (double)bytes);
    hipError_t e = launch_copy(in, out, bytes, (hipStream_t)stream, vpt, hints);
    return e == hipSuccess ? BMMC_OK : hip_fail(e, "copy launch");
}

int bmmc_copy(const void* in, void* out, size_t bytes, void* stream) {
    const bool big = bytes >= ((size_t)64 << 20);
    return bmmc_copy_ex(in, out, bytes, big ? 2 : 4, big ? 2 : 0, stream);
}

int bmmc_profile_begin(void) {
    int st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    std::lock_guard<std::mutex> lk(ds->mu);
    ds->profiling = true;
    ds->events.clear();
    ds->events.reserve(1 << 16);
    return BMMC_OK;
}

int bmmc_profile_end(bmmc_kernel_stat_t* out, int max) {
    int st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    std::lock_guard<std::mutex> lk(ds->mu);
    ds->profiling = false;
    std::vector<bmmc_kernel_stat_t> acc;
    for (auto& ev : ds->events) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.stop) == hipSuccess) hipEventElapsedTime(&ms, ev.start, ev.stop);
        bmmc_kernel_stat_t* slot = nullptr;
        for (auto& a : acc)
            if (ev.name == a.name) slot = &a;
        if (!slot) {
            bmmc_kernel_stat_t s;
            std::memset(&s, 0, sizeof(s));
            snprintf(s.name, sizeof(s.name), "%s", ev.name.c_str());
            acc.push_back(s);
            slot = &acc.back();
        }
        slot->launches++;
        slot->total_ms += ms;
        slot->bytes += ev.bytes;
        ds->event_pool.push_back(ev.start);
        ds->event_pool.push_back(ev.stop);
    }
    ds->events.clear();
    int k = 0;
    for (auto& a : acc) {
        if (k >= max) break;
        out[k++] = a;
    }
    return k;
}

}  // extern "C"
