// Batched form: many arrays, each with its own n, width, A and c, in one
// replay of a captured hipGraph.
//
// The host plans every array (plan cache), lays the passes and the work items
// out in a pinned staging buffer and copies them to a device-resident table.
// The graph is [clear heads] -> [persistent kernel, phase 0] -> [persistent
// kernel, phase 1]: phase 0 runs the one-pass arrays and the first passes of
// the two-pass arrays, phase 1 their second passes.  The graph's kernel
// arguments are fixed device pointers (the item ranges live in the table), so
// one instantiated graph serves every call on a stream until the table has to
// grow.
#include <algorithm>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

namespace bmmc {

namespace {

struct BatchState {
    hipStream_t stream = nullptr;
    // device table: [range[3] | passes | items | heads[2]]
    void* dev = nullptr;
    void* host = nullptr;  // pinned staging of the same layout
    size_t cap_passes = 0, cap_items = 0;
    hipEvent_t staged = nullptr;  // last copy out of the staging buffer
    // one captured graph per (cache hints, tile iterations, second phase)
    // setting (batches of different sizes alternate between them), each for
    // one grid size
    hipGraphExec_t exec[32] = {};
    uint32_t exec_grid[32] = {};
};

struct BatchRegistry {
    std::mutex mu;
    std::vector<BatchState*> states;  // one per (device, stream)
    std::vector<int> devices;
};

BatchRegistry& registry() {
    static BatchRegistry r;
    return r;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t passes_off, items_off, heads_off, total;
};

Layout layout_for(size_t np, size_t ni) {
    Layout L;
    L.passes_off = 256;
    L.items_off = align_up(L.passes_off + np * sizeof(BatchPass), 256);
    L.heads_off = align_up(L.items_off + ni * sizeof(BatchItem), 256);
    L.total = L.heads_off + 256;
    return L;
}

int ensure_capacity(BatchState* bs, size_t np, size_t ni) {
    if (np <= bs->cap_passes && ni <= bs->cap_items) return BMMC_OK;
    np = std::max(np * 2, bs->cap_passes);
    ni = std::max(ni * 2, bs->cap_items);
    Layout L = layout_for(np, ni);
    hipError_t e;
    if (bs->dev) {
        e = hipStreamSynchronize(bs->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        hipFree(bs->dev);
        hipHostFree(bs->host);
        bs->dev = bs->host = nullptr;
    }
    for (hipGraphExec_t& g : bs->exec) {
        if (g) hipGraphExecDestroy(g);
        g = nullptr;
    }
    e = hipMalloc(&bs->dev, L.total);
    if (e != hipSuccess) {
        bs->dev = nullptr;
        return set_error(BMMC_ERR_NOMEM, "batch table of %zu bytes: %s", L.total, hipGetErrorString(e));
    }
    e = hipHostMalloc(&bs->host, L.total, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(bs->dev);
        bs->dev = nullptr;
        bs->host = nullptr;
        return set_error(BMMC_ERR_NOMEM, "pinned staging of %zu bytes: %s", L.total, hipGetErrorString(e));
    }
    bs->cap_passes = np;
    bs->cap_items = ni;
    return BMMC_OK;
}

BatchState* batch_state(hipStream_t stream, int device) {
    auto& r = registry();
    std::lock_guard<std::mutex> lk(r.mu);
    for (size_t i = 0; i < r.states.size(); i++)
        if (r.states[i]->stream == stream && r.devices[i] == device) return r.states[i];
    auto* bs = new BatchState();
    bs->stream = stream;
    r.states.push_back(bs);
    r.devices.push_back(device);
    return bs;
}

// Enqueue [clear heads] -> phase 0 [-> phase 1] on `s` (captured or not) for
// the device table at d with layout L; phase 1 only when some array takes
// two passes.
hipError_t enqueue_phases_at(uint8_t* d, const Layout& L, uint32_t grid, int hints, int iters, bool second,
                             hipStream_t s) {
    uint32_t* heads = (uint32_t*)(d + L.heads_off);
    const BatchPass* passes = (const BatchPass*)(d + L.passes_off);
    const BatchItem* items = (const BatchItem*)(d + L.items_off);
    const uint32_t* range = (const uint32_t*)d;
    hipError_t e = launch_zero(heads, 2, s);
    if (e == hipSuccess) e = launch_batched(passes, items, range, 0, heads, grid, hints, iters, s);
    if (e == hipSuccess && second) e = launch_batched(passes, items, range, 1, heads + 1, grid, hints, iters, s);
    return e;
}

// Capture those launches into an executable graph.
int capture_graph_at(uint8_t* d, const Layout& L, uint32_t grid, int hints, int iters, bool second,
                     hipGraphExec_t* out) {
    hipStream_t cap;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        hipStreamDestroy(cap);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    enqueue_phases_at(d, L, grid, hints, iters, second, cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return BMMC_OK;
}

int graph_slot(int hints, int size, bool second) {
    return (hints & 3) | (size == 8 ? 4 : size == 16 ? 8 : size == 32 ? 12 : 0) | (second ? 16 : 0);
}

int build_graph(BatchState* bs, uint32_t grid, int hints, int iters, bool second) {
    const int slot = graph_slot(hints, iters, second);
    hipGraphExec_t& g = bs->exec[slot];
    if (g && bs->exec_grid[slot] == grid) return BMMC_OK;
    if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
    }
    int st = capture_graph_at((uint8_t*)bs->dev, layout_for(bs->cap_passes, bs->cap_items), grid, hints, iters,
                              second, &g);
    if (st != BMMC_OK) return st;
    bs->exec_grid[slot] = grid;
    return BMMC_OK;
}

// The arrays that go through the persistent kernel, in queue order.
// 0: largest first (the short items at the end even out the finish);
// 1: input order.
std::vector<size_t> work_order(const std::vector<BatchArray>& arrays, int order) {
    std::vector<size_t> work;
    for (size_t i = 0; i < arrays.size(); i++)
        if (!arrays[i].single) work.push_back(i);
    if (order != 1)
        std::stable_sort(work.begin(), work.end(),
                         [&](size_t x, size_t y) { return arrays[x].bytes > arrays[y].bytes; });
    return work;
}

void table_counts(const std::vector<BatchArray>& arrays, const std::vector<size_t>& work, uint32_t chunk,
                  size_t* npasses, size_t* nitems) {
    *npasses = *nitems = 0;
    for (size_t a : work) {
        const Plan& p = *arrays[a].plan;
        *npasses += p.npass;
        for (int k = 0; k < p.npass; k++) *nitems += ((1u << p.pass[k].tab.ntb) + chunk - 1) / chunk;
    }
}

// Write the range header, the pass table and the work items (phase 0: every
// first pass; phase 1: the second passes) into the image h with layout L.
// Returns the number of passes; *nitems and *moved receive the item count
// and the algorithmic bytes of one launch.
uint32_t fill_table(const std::vector<BatchArray>& arrays, const std::vector<size_t>& work, uint32_t chunk,
                    uint8_t* h, const Layout& L, size_t* nitems, double* moved) {
    BatchPass* hp = (BatchPass*)(h + L.passes_off);
    BatchItem* hi = (BatchItem*)(h + L.items_off);
    uint32_t pidx = 0;
    *moved = 0;
    std::vector<uint32_t> first_pass(arrays.size(), 0);
    for (size_t a : work) {
        const BatchArray& ba = arrays[a];
        const Plan& p = *ba.plan;
        first_pass[a] = pidx;
        for (int k = 0; k < p.npass; k++) {
            BatchPass& bp = hp[pidx++];
            std::memset(&bp, 0, sizeof(bp));
            bp.in = (k == 0) ? ba.in : ba.scratch;
            bp.out = (k == p.npass - 1) ? ba.out : ba.scratch;
            bp.w = (uint32_t)p.w;
            bp.tab = p.pass[k].tab;
        }
        *moved += 2.0 * (double)ba.bytes;
    }
    size_t ni = 0;
    auto emit = [&](size_t a, int k) {
        const Plan& p = *arrays[a].plan;
        const uint32_t ntiles = 1u << p.pass[k].tab.ntb;
        for (uint32_t t0 = 0; t0 < ntiles; t0 += chunk) {
            BatchItem& it = hi[ni++];
            std::memset(&it, 0, sizeof(it));
            it.pass = first_pass[a] + (uint32_t)k;
            it.tile_begin = t0;
            it.tile_end = std::min(ntiles, t0 + chunk);
        }
    };
    for (size_t a : work) emit(a, 0);
    const uint32_t phase0_end = (uint32_t)ni;
    for (size_t a : work)
        if (arrays[a].plan->npass == 2) emit(a, 1);
    uint32_t* range = (uint32_t*)h;
    range[0] = 0;
    range[1] = phase0_end;
    range[2] = (uint32_t)ni;
    *nitems = ni;
    return pidx;
}

int resolve_batch_hints(const bmmc_batch_options_t& o, double moved) {
    // Non-temporal accesses pay off once the data outgrows the last-level cache.
    if (o.hints > 0) return (o.hints & 4) ? 0 : (o.hints & 3);
    return moved >= 2.0 * (double)((size_t)64 << 20) ? 3 : 0;
}

}  // namespace

int reserve_batch_state(hipStream_t stream, int device, size_t passes, size_t items) {
    return ensure_capacity(batch_state(stream, device), passes, items);
}

void release_batch_state(hipStream_t stream, int device) {
    BatchState* bs = nullptr;
    {
        auto& r = registry();
        std::lock_guard<std::mutex> lk(r.mu);
        for (size_t i = 0; i < r.states.size(); i++)
            if (r.states[i]->stream == stream && r.devices[i] == device) {
                bs = r.states[i];
                r.states.erase(r.states.begin() + (long)i);
                r.devices.erase(r.devices.begin() + (long)i);
                break;
            }
    }
    if (!bs) return;
    for (hipGraphExec_t& g : bs->exec)
        if (g) hipGraphExecDestroy(g);
    if (bs->staged) hipEventSynchronize(bs->staged);
    if (bs->dev) hipFree(bs->dev);
    if (bs->host) hipHostFree(bs->host);
    if (bs->staged) hipEventDestroy(bs->staged);
    delete bs;
}

int batch_validate(const bmmc_desc_t* descs, int count) {
    if (count < 0 || (count > 0 && !descs)) return set_error(BMMC_ERR_ARG, "descs is NULL or count < 0");
    struct Iv {
        uintptr_t a, b;
        int idx;
        bool is_out;
    };
    std::vector<Iv> iv;
    iv.reserve(2 * (size_t)count);
    for (int i = 0; i < count; i++) {
        const bmmc_desc_t& d = descs[i];
        if (d.n < 0 || d.n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "array %d: n = %d out of range", i, d.n);
        const int w = d.elem_bytes;
        if (!(w == 1 || w == 2 || w == 4 || w == 8 || w == 16))
            return set_error(BMMC_ERR_ARG, "array %d: elem_bytes = %d", i, w);
        const size_t bytes = ((size_t)1 << d.n) * (size_t)w;
        int st = validate_buffers(d.in, d.out, bytes);
        if (st != BMMC_OK) return set_error(st, "array %d: %s", i, bmmc_last_error());
        iv.push_back({(uintptr_t)d.in, (uintptr_t)d.in + bytes, i, false});
        iv.push_back({(uintptr_t)d.out, (uintptr_t)d.out + bytes, i, true});
    }
    // No output may overlap any other interval (inputs may be shared).  In
    // start order, an interval overlaps an earlier one exactly when it starts
    // before the largest end seen so far.
    std::sort(iv.begin(), iv.end(), [](const Iv& x, const Iv& y) { return x.a < y.a; });
    uintptr_t end_any = 0, end_out = 0;
    int idx_any = -1, idx_out = -1;
    for (const Iv& v : iv) {
        if (v.is_out && idx_any >= 0 && v.a < end_any)
            return set_error(BMMC_ERR_ALIAS, "arrays %d and %d overlap", idx_any, v.idx);
        if (!v.is_out && idx_out >= 0 && v.a < end_out)
            return set_error(BMMC_ERR_ALIAS, "arrays %d and %d overlap", idx_out, v.idx);
        if (v.b > end_any) {
            end_any = v.b;
            idx_any = v.idx;
        }
        if (v.is_out && v.b > end_out) {
            end_out = v.b;
            idx_out = v.idx;
        }
    }
    return BMMC_OK;
}


int plan_batch_array(DeviceState* ds, const bmmc_desc_t& d, int method, int iters, BatchArray* out,
                     int tile_order) {
    PlanOptions po;
    po.method = (method == BMMC_METHOD_ONEPASS || method == BMMC_METHOD_TILED) ? method : kMethodAuto;
    po.tb_mix = tile_order_mix(tile_order);
    if (d.elem_bytes >= 4) {
        // the batched kernel's one shape
        po.shape = default_shape(d.elem_bytes);
        po.shape.nt = batched_threads(batched_size(iters));
        po.shape.iters = batched_vectors(batched_size(iters));
        po.shape_given = true;
    }
    int st = get_plan(ds, d.A_rows, d.c, d.n, d.elem_bytes, po, &out->plan);
    if (st != BMMC_OK) return st;
    out->in = d.in;
    out->out = d.out;
    out->scratch = nullptr;
    out->bytes = ((size_t)1 << d.n) * (size_t)d.elem_bytes;
    // Arrays of one element, too small for 16-byte vectors, or of 1- or
    // 2-byte elements take the single-array kernels.
    out->single = out->plan->npass == 0 || out->plan->naive || d.elem_bytes < 4;
    out->grid = 0;
    out->hints = resolve_hints(nullptr, out->bytes);
    out->order = 0;
    return BMMC_OK;
}

// Options of a batch with no tuned entry: beyond the last-level cache, the
// 128 KiB tile with one tile per item (measured on the 1024-array batch of
// 2^10-2^22 elements: 93 % of a copy of the same bytes against 77 % with
// the 16 KiB default, whose many items per array keep more arrays in
// flight); below it, the defaults.
void untuned_batch_options(const bmmc_desc_t* descs, int count, bmmc_batch_options_t* o) {
    double bytes = 0;
    for (int i = 0; i < count; i++) bytes += (double)((size_t)1 << descs[i].n) * (double)descs[i].elem_bytes;
    if (bytes >= (double)((size_t)256 << 20)) {
        o->iters = 32;
        o->chunk_tiles = 1;
    }
}

// Every array the persistent kernel runs was planned for its tile shape
// (the tables address the tile's slots by that shape).
int check_batch_shapes(const std::vector<BatchArray>& arrays, int size) {
    for (const BatchArray& a : arrays)
        if (!a.single && (a.plan->shape.nt != batched_threads(size) || a.plan->shape.iters != batched_vectors(size)))
            return set_error(BMMC_ERR_INTERNAL, "array planned for another batched tile shape");
    return BMMC_OK;
}

int enqueue_batched(DeviceState* ds, std::vector<BatchArray>& arrays, const bmmc_batch_options_t& o,
                    hipStream_t stream) {
    const uint32_t chunk = o.chunk_tiles > 0 ? (uint32_t)o.chunk_tiles : 4u;
    int st;
    for (size_t i = 0; i < arrays.size(); i++) {
        if (arrays[i].single) {
            const BatchArray& a = arrays[i];
            st = enqueue_plan(ds, *a.plan, a.in, a.out, stream, a.grid, a.hints, a.order, a.scratch);
            if (st != BMMC_OK) return st;
        } else if (arrays[i].plan->npass == 2 && !arrays[i].scratch) {
            return set_error(BMMC_ERR_INTERNAL, "two-pass array without scratch");
        }
    }
    st = check_batch_shapes(arrays, batched_size(o.iters));
    if (st != BMMC_OK) return st;
    const std::vector<size_t> work = work_order(arrays, o.order);
    if (work.empty()) return BMMC_OK;
    size_t npasses, nitems;
    table_counts(arrays, work, chunk, &npasses, &nitems);
    BatchState* bs = batch_state(stream, ds->device);
    st = ensure_capacity(bs, npasses, nitems);
    if (st != BMMC_OK) return st;
    if (bs->staged) {
        hipError_t e = hipEventSynchronize(bs->staged);  // staging buffer free again
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    const Layout L = layout_for(bs->cap_passes, bs->cap_items);
    uint8_t* h = (uint8_t*)bs->host;
    size_t ni;
    double moved;
    const uint32_t np = fill_table(arrays, work, chunk, h, L, &ni, &moved);

    // Upload only what is used, then launch.
    hipError_t e = hipMemcpyAsync(bs->dev, bs->host, L.passes_off + np * sizeof(BatchPass),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((uint8_t*)bs->dev + L.items_off, h + L.items_off, ni * sizeof(BatchItem),
                           hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (batch table)");
    if (!bs->staged) hipEventCreateWithFlags(&bs->staged, hipEventDisableTiming);
    hipEventRecord(bs->staged, stream);

    const int iters = batched_size(o.iters);
    uint32_t grid = o.workgroups > 0 ? (uint32_t)o.workgroups : (uint32_t)(ds->cu_count * batched_occupancy(iters));
    const uint32_t* range = (const uint32_t*)h;
    const bool second = range[2] > range[1];
    if (o.use_graph < 0) {
        // plain launches: no more work-groups than the larger phase has items
        const uint32_t most = std::max(range[1] - range[0], range[2] - range[1]);
        grid = std::max(1u, std::min(grid, most));
    }
    const int hints = resolve_batch_hints(o, moved);
    if (o.use_graph >= 0) {
        st = build_graph(bs, grid, hints, iters, second);
        if (st != BMMC_OK) return st;
    }
    LaunchScope ls(ds, stream, "k_batched", moved, false);
    if (o.use_graph >= 0) {
        e = hipGraphLaunch(bs->exec[graph_slot(hints, iters, second)], stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        e = enqueue_phases_at((uint8_t*)bs->dev, L, grid, hints, iters, second, stream);
        if (e != hipSuccess) return hip_fail(e, "batched launch");
    }
    return BMMC_OK;
}

// The batch with its device table at `table` (cap bytes, caller-provided):
// the table image is built in host memory, copied in, and both phases run as
// plain launches.  No device memory is allocated, so arrays that take two
// passes (they need a scratch array as large as themselves) are refused.
int enqueue_batched_fixed(DeviceState* ds, std::vector<BatchArray>& arrays, const bmmc_batch_options_t& o,
                          hipStream_t stream, void* table, size_t cap) {
    const uint32_t chunk = o.chunk_tiles > 0 ? (uint32_t)o.chunk_tiles : 4u;
    for (size_t i = 0; i < arrays.size(); i++)
        if (arrays[i].plan->npass > 1)
            return set_error(BMMC_ERR_ARG,
                             "array %zu takes two passes, whose scratch array would have to be allocated", i);
    int st = check_batch_shapes(arrays, batched_size(o.iters));
    if (st != BMMC_OK) return st;
    const std::vector<size_t> work = work_order(arrays, o.order);
    size_t npasses = 0, nitems = 0;
    table_counts(arrays, work, chunk, &npasses, &nitems);
    const Layout L = layout_for(npasses, nitems);
    if (!work.empty() && L.total > cap)
        return set_error(BMMC_ERR_RANGE, "batch table of %zu bytes exceeds the fixed %zu-byte table", L.total, cap);
    for (const BatchArray& a : arrays) {
        if (!a.single) continue;
        st = enqueue_plan(ds, *a.plan, a.in, a.out, stream, a.grid, a.hints, a.order, nullptr);
        if (st != BMMC_OK) return st;
    }
    if (work.empty()) return BMMC_OK;
    // Host image of the table; hipMemcpyAsync from pageable memory has
    // consumed it when it returns, so the next call may refill it.
    static thread_local std::vector<uint8_t> image;
    image.assign(L.total, 0);
    size_t ni;
    double moved;
    const uint32_t np = fill_table(arrays, work, chunk, image.data(), L, &ni, &moved);
    hipError_t e = hipMemcpyAsync(table, image.data(), L.passes_off + np * sizeof(BatchPass),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((uint8_t*)table + L.items_off, image.data() + L.items_off, ni * sizeof(BatchItem),
                           hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (fixed batch table)");
    const int iters = batched_size(o.iters);
    uint32_t grid = o.workgroups > 0 ? (uint32_t)o.workgroups : (uint32_t)(ds->cu_count * batched_occupancy(iters));
    const uint32_t* range = (const uint32_t*)image.data();
    const bool second = range[2] > range[1];
    const uint32_t most = std::max(range[1] - range[0], range[2] - range[1]);
    grid = std::max(1u, std::min(grid, most));
    LaunchScope ls(ds, stream, "k_batched", moved, false);
    e = enqueue_phases_at((uint8_t*)table, L, grid, resolve_batch_hints(o, moved), iters, second, stream);
    return e == hipSuccess ? BMMC_OK : hip_fail(e, "batched launch");
}

// Signature of a batch for the tuning cache: count and a histogram of
// (n, width) pairs.
uint64_t batch_signature(const bmmc_desc_t* descs, int count) {
    uint64_t hist[33 * 5] = {};
    for (int i = 0; i < count; i++) {
        const int w = descs[i].elem_bytes;
        const int wi = w == 1 ? 0 : w == 2 ? 1 : w == 4 ? 2 : w == 8 ? 3 : 4;
        const int n = descs[i].n < 0 ? 0 : descs[i].n > 32 ? 32 : descs[i].n;
        hist[n * 5 + wi]++;
    }
    uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)count;
    for (int k = 0; k < 33 * 5; k++) {
        h ^= hist[k] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    }
    return h;
}

void default_batch_options(const bmmc_desc_t* descs, int count, bmmc_batch_options_t* o) {
    std::memset(o, 0, sizeof(*o));
    if (!tuned_batch_options(batch_signature(descs, count), o)) untuned_batch_options(descs, count, o);
}

}  // namespace bmmc

using namespace bmmc;

extern "C" int bmmc_permute_batched_ex(const bmmc_desc_t* descs, int count, const bmmc_batch_options_t* opts,
                                       void* stream_) {
    int st = batch_validate(descs, count);
    if (st != BMMC_OK) return st;
    if (count == 0) return BMMC_OK;
    bmmc_batch_options_t o;
    if (opts) o = *opts;
    else default_batch_options(descs, count, &o);
    if (o.iters != 0 && o.iters != 4 && o.iters != 8 && o.iters != 16 && o.iters != 32)
        return set_error(BMMC_ERR_ARG, "iters must be 0, 4, 8, 16 or 32");
    if (o.tile_order < 0 || o.tile_order > 511) return set_error(BMMC_ERR_ARG, "tile_order outside [0, 511]");
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    hipStream_t stream = (hipStream_t)stream_;

    std::vector<BatchArray> arrays(count);
    size_t scratch_total = 0;
    std::vector<size_t> offs(count, 0);
    for (int i = 0; i < count; i++) {
        st = plan_batch_array(ds, descs[i], o.method, o.iters, &arrays[i], o.tile_order);
        if (st != BMMC_OK) return set_error(st, "array %d: %s", i, bmmc_last_error());
        if (!arrays[i].single && arrays[i].plan->npass == 2) {
            offs[i] = scratch_total;
            scratch_total += (arrays[i].bytes + 255) / 256 * 256;
        }
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    if (scratch_total) {
        void* scratch = nullptr;
        st = get_scratch(ds, stream, scratch_total, &scratch);
        if (st != BMMC_OK) return st;
        for (int i = 0; i < count; i++)
            if (!arrays[i].single && arrays[i].plan->npass == 2) arrays[i].scratch = (uint8_t*)scratch + offs[i];
    }
    return enqueue_batched(ds, arrays, o, stream);
}

extern "C" int bmmc_permute_batched(const bmmc_desc_t* descs, int count, void* stream) {
    return bmmc_permute_batched_ex(descs, count, nullptr, stream);
}

// ------------------------------------------------------------ prepared batches

namespace bmmc {

struct PreparedBatch {
    DeviceState* ds = nullptr;
    std::vector<BatchArray> arrays;
    void* table = nullptr;    // device table (range, passes, items, heads)
    void* scratch = nullptr;  // owned scratch of the two-pass arrays
    hipGraphExec_t exec = nullptr;
    uint32_t grid = 0;
    int hints = 0;
    int iters = 4;
    bool use_graph = true;
    bool second = false;  // some array takes two passes
    Layout L{};
    double moved = 0;
};

}  // namespace bmmc

extern "C" int bmmc_batch_create(const bmmc_desc_t* descs, int count, const bmmc_batch_options_t* opts,
                                 void** handle_out) {
    if (!handle_out) return set_error(BMMC_ERR_ARG, "handle_out is NULL");
    int st = batch_validate(descs, count);
    if (st != BMMC_OK) return st;
    if (count == 0) return set_error(BMMC_ERR_ARG, "empty batch");
    bmmc_batch_options_t o;
    if (opts) o = *opts;
    else default_batch_options(descs, count, &o);
    if (o.iters != 0 && o.iters != 4 && o.iters != 8 && o.iters != 16 && o.iters != 32)
        return set_error(BMMC_ERR_ARG, "iters must be 0, 4, 8, 16 or 32");
    if (o.tile_order < 0 || o.tile_order > 511) return set_error(BMMC_ERR_ARG, "tile_order outside [0, 511]");
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    const uint32_t chunk = o.chunk_tiles > 0 ? (uint32_t)o.chunk_tiles : 4u;

    auto* pb = new PreparedBatch();
    pb->ds = ds;
    pb->arrays.resize(count);
    size_t scratch_total = 0;
    std::vector<size_t> offs(count, 0);
    for (int i = 0; i < count; i++) {
        st = plan_batch_array(ds, descs[i], o.method, o.iters, &pb->arrays[i], o.tile_order);
        if (st != BMMC_OK) {
            delete pb;
            return set_error(st, "array %d: %s", i, bmmc_last_error());
        }
        if (!pb->arrays[i].single && pb->arrays[i].plan->npass == 2) {
            offs[i] = scratch_total;
            scratch_total += (pb->arrays[i].bytes + 255) / 256 * 256;
        }
    }
    auto fail = [&](int code) {
        if (pb->scratch) hipFree(pb->scratch);
        if (pb->table) hipFree(pb->table);
        delete pb;
        return code;
    };
    if (scratch_total) {
        hipError_t e = hipMalloc(&pb->scratch, scratch_total);
        if (e != hipSuccess) {
            pb->scratch = nullptr;
            (void)hipGetLastError();
            return fail(set_error(BMMC_ERR_NOMEM, "batch scratch of %zu bytes", scratch_total));
        }
        for (int i = 0; i < count; i++)
            if (!pb->arrays[i].single && pb->arrays[i].plan->npass == 2)
                pb->arrays[i].scratch = (uint8_t*)pb->scratch + offs[i];
    }
    st = check_batch_shapes(pb->arrays, batched_size(o.iters));
    if (st != BMMC_OK) return fail(st);
    const std::vector<size_t> work = work_order(pb->arrays, o.order);
    size_t npasses, nitems;
    table_counts(pb->arrays, work, chunk, &npasses, &nitems);
    pb->L = layout_for(npasses, nitems);
    std::vector<uint8_t> image(pb->L.total, 0);
    size_t ni;
    fill_table(pb->arrays, work, chunk, image.data(), pb->L, &ni, &pb->moved);
    {
        const uint32_t* range = (const uint32_t*)image.data();
        pb->second = range[2] > range[1];
    }
    hipError_t e = hipMalloc(&pb->table, pb->L.total);
    if (e != hipSuccess) {
        pb->table = nullptr;
        (void)hipGetLastError();
        return fail(set_error(BMMC_ERR_NOMEM, "batch table of %zu bytes", pb->L.total));
    }
    e = hipMemcpy(pb->table, image.data(), pb->L.total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpy (batch table)"));
    pb->iters = batched_size(o.iters);
    pb->grid = o.workgroups > 0 ? (uint32_t)o.workgroups : (uint32_t)(ds->cu_count * batched_occupancy(pb->iters));
    pb->hints = resolve_batch_hints(o, pb->moved);
    pb->use_graph = o.use_graph >= 0;
    if (!work.empty() && pb->use_graph) {
        st = capture_graph_at((uint8_t*)pb->table, pb->L, pb->grid, pb->hints, pb->iters, pb->second, &pb->exec);
        if (st != BMMC_OK) return fail(st);
    }
    *handle_out = pb;
    return BMMC_OK;
}

extern "C" int bmmc_batch_launch(void* handle, void* stream_) {
    PreparedBatch* pb = (PreparedBatch*)handle;
    if (!pb) return set_error(BMMC_ERR_ARG, "NULL handle");
    hipStream_t stream = (hipStream_t)stream_;
    DeviceState* ds = pb->ds;
    std::lock_guard<std::mutex> lk(ds->mu);
    for (auto& ba : pb->arrays) {
        if (!ba.single) continue;
        int st = enqueue_plan(ds, *ba.plan, ba.in, ba.out, stream, ba.grid, ba.hints, ba.order, ba.scratch);
        if (st != BMMC_OK) return st;
    }
    bool any = false;
    for (auto& ba : pb->arrays) any |= !ba.single;
    if (!any) return BMMC_OK;
    LaunchScope ls(ds, stream, "k_batched", pb->moved, false);
    hipError_t e = pb->use_graph ? hipGraphLaunch(pb->exec, stream)
                                 : enqueue_phases_at((uint8_t*)pb->table, pb->L, pb->grid, pb->hints, pb->iters,
                                                     pb->second, stream);
    return e == hipSuccess ? BMMC_OK : hip_fail(e, "batch launch");
}

extern "C" int bmmc_batch_destroy(void* handle) {
    PreparedBatch* pb = (PreparedBatch*)handle;
    if (!pb) return set_error(BMMC_ERR_ARG, "NULL handle");
    hipDeviceSynchronize();
    if (pb->exec) hipGraphExecDestroy(pb->exec);
    if (pb->table) hipFree(pb->table);
    if (pb->scratch) hipFree(pb->scratch);
    delete pb;
    return BMMC_OK;
}
