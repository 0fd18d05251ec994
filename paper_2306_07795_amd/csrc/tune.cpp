// Autotuner: times candidate tile shapes and launch parameters on the device
// and caches the fastest, per (n, width, method, matrix class) for single
// arrays -- class 0: matrices that are not tiled (general one-pass tiles or
// two passes), class 1: tiled matrices such as bit permutations -- and per
// batch signature for batched launches.  The cache can be saved to and loaded
// from a JSON-lines file; BMMC_TUNE_CACHE names a file loaded on first use.
// Options tuned for one matrix (bmmc_autotune_matrix) are kept in memory
// only and take precedence over its class's.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <dlfcn.h>

#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

namespace bmmc {

namespace {

struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    std::map<std::tuple<int, int, int, int>, std::pair<bmmc_options_t, double>> plain;
    std::map<uint64_t, std::pair<bmmc_batch_options_t, double>> batch;
    // per matrix: key {n, width, rows...}; `nmatrix` lets calls skip the
    // lookup while the map is empty
    std::map<std::vector<uint64_t>, bmmc_options_t> matrix;
    std::atomic<size_t> nmatrix{0};
};

constexpr size_t kMaxMatrixEntries = 4096;

std::vector<uint64_t> matrix_key(int n, int w, const uint64_t* rows) {
    std::vector<uint64_t> k((size_t)n + 2);
    k[0] = (uint64_t)n;
    k[1] = (uint64_t)w;
    for (int i = 0; i < n; i++) k[(size_t)i + 2] = rows[i] & low_mask(n);
    return k;
}

TuneCache& cache() {
    static TuneCache c;
    return c;
}

int load_file(TuneCache& c, const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return 0;
    char line[512];
    int count = 0;
    while (std::fgets(line, sizeof(line), f)) {
        bmmc_options_t o;
        std::memset(&o, 0, sizeof(o));
        int n, w, method, cls, used;
        double ms;
        if (std::sscanf(line,
                        "{\"kind\": \"plain\", \"n\": %d, \"w\": %d, \"method\": %d, \"class\": %d, "
                        "\"used\": %d, \"threads\": %d, \"iters\": %d, \"t\": %d, \"run_in\": %d, "
                        "\"run_out\": %d, \"hints\": %d, \"tile_order\": %d, \"grid\": %d, \"swizzle\": %d, "
                        "\"ms\": %lf}",
                        &n, &w, &method, &cls, &used, &o.threads, &o.iters, &o.t, &o.run_in, &o.run_out,
                        &o.hints, &o.tile_order, &o.grid, &o.swizzle, &ms) == 15) {
            o.method = used;
            c.plain[{n, w, method, cls}] = {o, ms};
            count++;
            continue;
        }
        bmmc_batch_options_t b;
        std::memset(&b, 0, sizeof(b));
        uint64_t sig;
        if (std::sscanf(line,
                        "{\"kind\": \"batch\", \"sig\": \"%" SCNx64 "\", \"workgroups\": %d, \"chunk_tiles\": %d, "
                        "\"order\": %d, \"method\": %d, \"iters\": %d, \"tile_order\": %d, \"hints\": %d, "
                        "\"ms\": %lf}",
                        &sig, &b.workgroups, &b.chunk_tiles, &b.order, &b.method, &b.iters, &b.tile_order,
                        &b.hints, &ms) == 9 ||
            std::sscanf(line,
                        "{\"kind\": \"batch\", \"sig\": \"%" SCNx64 "\", \"workgroups\": %d, \"chunk_tiles\": %d, "
                        "\"order\": %d, \"method\": %d, \"iters\": %d, \"tile_order\": %d, \"ms\": %lf}",
                        &sig, &b.workgroups, &b.chunk_tiles, &b.order, &b.method, &b.iters, &b.tile_order,
                        &ms) == 8 ||
            std::sscanf(line,
                        "{\"kind\": \"batch\", \"sig\": \"%" SCNx64 "\", \"workgroups\": %d, \"chunk_tiles\": %d, "
                        "\"order\": %d, \"method\": %d, \"iters\": %d, \"ms\": %lf}",
                        &sig, &b.workgroups, &b.chunk_tiles, &b.order, &b.method, &b.iters, &ms) == 7) {
            c.batch[sig] = {b, ms};
            count++;
        }
    }
    std::fclose(f);
    return count;
}

// The tuning results shipped with the library: tuning/gfx950.jsonl beside
// libbmmc.so (found through the address of this function).
std::string packaged_tuning_file() {
    Dl_info info;
    if (!dladdr((void*)&packaged_tuning_file, &info) || !info.dli_fname) return std::string();
    std::string lib = info.dli_fname;
    const size_t slash = lib.find_last_of('/');
    const std::string dir = slash == std::string::npos ? std::string(".") : lib.substr(0, slash);
    return dir + "/tuning/gfx950.jsonl";
}

void ensure_loaded(TuneCache& c) {
    if (c.loaded) return;
    c.loaded = true;
    const char* path = std::getenv("BMMC_TUNE_CACHE");
    if (path) {
        if (*path) load_file(c, path);
        return;  // an empty value asks for no tuning results at all
    }
    const std::string own = packaged_tuning_file();
    if (!own.empty()) load_file(c, own.c_str());
}

int save_file(TuneCache& c, const char* path) {
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(BMMC_ERR_ARG, "cannot write %s", path);
    for (auto& kv : c.plain) {
        const bmmc_options_t& o = kv.second.first;
        std::fprintf(f,
                     "{\"kind\": \"plain\", \"n\": %d, \"w\": %d, \"method\": %d, \"class\": %d, "
                     "\"used\": %d, \"threads\": %d, \"iters\": %d, \"t\": %d, \"run_in\": %d, "
                     "\"run_out\": %d, \"hints\": %d, \"tile_order\": %d, \"grid\": %d, \"swizzle\": %d, "
                     "\"ms\": %.6f}\n",
                     std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                     o.method, o.threads, o.iters, o.t, o.run_in, o.run_out, o.hints, o.tile_order, o.grid,
                     o.swizzle, kv.second.second);
    }
    for (auto& kv : c.batch) {
        const bmmc_batch_options_t& b = kv.second.first;
        std::fprintf(f,
                     "{\"kind\": \"batch\", \"sig\": \"%016" PRIx64 "\", \"workgroups\": %d, \"chunk_tiles\": %d, "
                     "\"order\": %d, \"method\": %d, \"iters\": %d, \"tile_order\": %d, \"hints\": %d, "
                     "\"ms\": %.6f}\n",
                     kv.first, b.workgroups, b.chunk_tiles, b.order, b.method, b.iters, b.tile_order, b.hints,
                     kv.second.second);
    }
    std::fclose(f);
    return BMMC_OK;
}

void autosave(TuneCache& c) {
    const char* path = std::getenv("BMMC_TUNE_CACHE");
    if (path && *path) save_file(c, path);
}

uint64_t next_rand(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A random invertible matrix (rows drawn until independent) for timing.
void random_matrix(int n, uint64_t seed, uint64_t* rows, uint64_t* c) {
    Basis b;
    int k = 0;
    while (k < n) {
        uint64_t r = next_rand(&seed) & low_mask(n);
        if (b.insert(r)) rows[k++] = r;
    }
    *c = next_rand(&seed) & low_mask(n);
}

// A random bit permutation with complement (tiled at every t) for timing.
void random_bpc(int n, uint64_t seed, uint64_t* rows, uint64_t* c) {
    int perm[64];
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int i = n - 1; i > 0; i--) {
        const int j = (int)(next_rand(&seed) % (uint64_t)(i + 1));
        const int t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    for (int i = 0; i < n; i++) rows[i] = 1ull << perm[i];
    *c = next_rand(&seed) & low_mask(n);
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    // one pair per call of a flushed timing
    std::vector<hipEvent_t> as, bs;
    Timer() {
        hipEventCreate(&a);
        hipEventCreate(&b);
    }
    ~Timer() {
        hipEventDestroy(a);
        hipEventDestroy(b);
        for (hipEvent_t e : as) hipEventDestroy(e);
        for (hipEvent_t e : bs) hipEventDestroy(e);
    }
    bool reserve(size_t k) {
        while (as.size() < k) {
            hipEvent_t x = nullptr, y = nullptr;
            if (hipEventCreate(&x) != hipSuccess) return false;
            if (hipEventCreate(&y) != hipSuccess) {
                hipEventDestroy(x);
                return false;
            }
            as.push_back(x);
            bs.push_back(y);
        }
        return true;
    }
};

// The cache state calls are timed in from 64 MiB on: before each timed call,
// a copy of kFlushBytes between two other buffers (outside the timed
// interval) leaves the L2 caches and the 256 MB last-level cache holding
// another array's lines, many of them dirty, as when a call follows
// unrelated work.  Below 64 MiB calls are timed back to back (graph
// replays), the state of an array that stays in the caches between uses.
constexpr size_t kFlushBytes = (size_t)512 << 20;
constexpr size_t kFlushFrom = (size_t)64 << 20;

struct FlushBufs {
    void* a = nullptr;
    void* b = nullptr;
    ~FlushBufs() {
        if (a) hipFree(a);
        if (b) hipFree(b);
    }
    // false when the buffers cannot be allocated
    bool make(hipStream_t stream) {
        if (hipMalloc(&a, kFlushBytes) != hipSuccess || hipMalloc(&b, kFlushBytes) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return hipMemsetAsync(a, 0x3c, kFlushBytes, stream) == hipSuccess;
    }
    hipError_t flush(hipStream_t stream) const { return launch_copy(a, b, kFlushBytes, stream, 1, 0); }
};

}  // namespace

int matrix_class(const uint64_t* rows, int n) {
    if (n <= 0 || !rows) return 0;
    BitMat A;
    A.n = n;
    for (int i = 0; i < n; i++) A.r[i] = rows[i] & low_mask(n);
    const int t = n < 6 ? n : 6;
    return is_tiled(A, t) ? 1 : 0;
}

bool tuned_options(int n, int w, int method, int cls, bmmc_options_t* out) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    auto it = c.plain.find({n, w, method, cls});
    if (it == c.plain.end()) return false;
    *out = it->second.first;
    return true;
}

bool matrix_options(int n, int w, const uint64_t* rows, bmmc_options_t* out) {
    TuneCache& c = cache();
    if (c.nmatrix.load(std::memory_order_relaxed) == 0 || n <= 0 || !rows) return false;
    const std::vector<uint64_t> key = matrix_key(n, w, rows);
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.matrix.find(key);
    if (it == c.matrix.end()) return false;
    *out = it->second;
    return true;
}

bool tuned_batch_options(uint64_t signature, bmmc_batch_options_t* out) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    auto it = c.batch.find(signature);
    if (it == c.batch.end()) return false;
    *out = it->second.first;
    return true;
}

}  // namespace bmmc

using namespace bmmc;

extern "C" int bmmc_tune_lookup(int n, int elem_bytes, int method, const uint64_t* A_rows,
                                bmmc_options_t* opts_out) {
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    if (!opts_out || (n > 0 && !A_rows)) return set_error(BMMC_ERR_ARG, "NULL argument");
    if (method == BMMC_METHOD_AUTO && matrix_options(n, elem_bytes, A_rows, opts_out)) return 1;
    return tuned_options(n, elem_bytes, method, matrix_class(A_rows, n), opts_out) ? 1 : 0;
}

extern "C" int bmmc_tune_lookup_batched(const bmmc_desc_t* descs, int count, bmmc_batch_options_t* opts_out) {
    if (!opts_out || count < 0 || (count > 0 && !descs)) return set_error(BMMC_ERR_ARG, "NULL argument");
    return tuned_batch_options(batch_signature(descs, count), opts_out) ? 1 : 0;
}

extern "C" int bmmc_tune_save(const char* path) {
    if (!path) return set_error(BMMC_ERR_ARG, "path is NULL");
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    return save_file(c, path);
}

extern "C" int bmmc_tune_load(const char* path) {
    if (!path) return set_error(BMMC_ERR_ARG, "path is NULL");
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    c.loaded = true;
    return load_file(c, path);
}

namespace bmmc {
namespace {

struct TuneMatrix {
    uint64_t rows[64];
    uint64_t c;
};

// Mean time of one call with options o, summed over the matrices.  Arrays
// below 64 MiB run for a few microseconds, less than the host takes to
// issue a call: their `reps` calls are captured into a graph (on `cap`,
// where a first call outside the capture has made any scratch) and the
// graph's replay is timed, so that device time is what is compared.  From
// 64 MiB on, with `fl`, every call is timed on its own after a cache flush.
//
// The score is the mean of the per-matrix times and their maximum, times the
// number of matrices (so that dividing by the count gives a per-call time):
// a setting that is fast on average but slow for one matrix loses to one
// that is nearly as fast for every matrix.  (On 1 GiB arrays the shared
// setting of the plain sum ran seeds 0-7 of the benchmark's random matrices
// at 73-88 % of the copy, while settings within a point of its mean kept
// every matrix above 81 %.)
double time_options(int n, int elem_bytes, const std::vector<TuneMatrix>& mats, const bmmc_options_t& o,
                    const void* in, void* out, hipStream_t stream, hipStream_t cap, int reps, Timer& tm,
                    const FlushBufs* fl = nullptr) {
    double total = 0, worst = 0;
    auto add = [&](double t) {
        total += t;
        worst = std::max(worst, t);
    };
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    const bool graph = cap && bytes < kFlushFrom;
    for (const TuneMatrix& m : mats) {
        if (!graph && fl && fl->a && bytes >= kFlushFrom) {
            if (bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, stream) != BMMC_OK) return -1;
            if (!tm.reserve((size_t)reps)) return -1;
            for (int r = 0; r < reps; r++) {
                if (fl->flush(stream) != hipSuccess) return -1;
                hipEventRecord(tm.as[r], stream);
                bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, stream);
                hipEventRecord(tm.bs[r], stream);
            }
            if (hipEventSynchronize(tm.bs[reps - 1]) != hipSuccess) return -1;
            double sum = 0;
            for (int r = 0; r < reps; r++) {
                float ms = 0;
                hipEventElapsedTime(&ms, tm.as[r], tm.bs[r]);
                sum += ms;
            }
            add(sum / reps);
            continue;
        }
        if (!graph) {
            if (bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, stream) != BMMC_OK) return -1;
            hipEventRecord(tm.a, stream);
            for (int r = 0; r < reps; r++) bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, stream);
            hipEventRecord(tm.b, stream);
        } else {
            if (bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, cap) != BMMC_OK) return -1;
            if (hipStreamSynchronize(cap) != hipSuccess) return -1;
            if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return -1;
            int st = BMMC_OK;
            for (int r = 0; r < reps && st == BMMC_OK; r++)
                st = bmmc_permute_ex(in, out, n, m.rows, m.c, elem_bytes, &o, cap);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cap, &g);
            hipGraphExec_t x = nullptr;
            if (st != BMMC_OK || e != hipSuccess || hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
                if (g) hipGraphDestroy(g);
                (void)hipGetLastError();
                return -1;
            }
            hipGraphDestroy(g);
            hipGraphLaunch(x, stream);  // warm-up
            hipEventRecord(tm.a, stream);
            hipGraphLaunch(x, stream);
            hipEventRecord(tm.b, stream);
            hipEventSynchronize(tm.b);
            hipGraphExecDestroy(x);
        }
        hipEventSynchronize(tm.b);
        float ms = 0;
        hipEventElapsedTime(&ms, tm.a, tm.b);
        add(ms / reps);
    }
    return 0.5 * (total + worst * (double)mats.size());
}

// The capture stream of the graph timing (null if none could be made), and
// its release together with any scratch array the library made for it.
hipStream_t make_capture_stream() {
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        cap = nullptr;
        (void)hipGetLastError();
    }
    return cap;
}

void drop_capture_stream(DeviceState* ds, hipStream_t cap) {
    if (!cap) return;
    hipStreamSynchronize(cap);
    {
        std::lock_guard<std::mutex> lk(ds->mu);
        auto it = ds->scratch.find(cap);
        if (it != ds->scratch.end()) {
            if (it->second.ptr) hipFree(it->second.ptr);
            ds->scratch.erase(it);
        }
    }
    hipStreamDestroy(cap);
}

// Two stages, each candidate timed on the matrices (`reps` runs each): first
// tile shape, read/write runs, cache hints and method under two tile orders
// and both grid kinds; then, for the six fastest of those, every tile order
// and grid kind.  The library default for the size is always a candidate.
// Returns the fastest options and their time per matrix.
void tune_matrices(DeviceState* ds, int n, int elem_bytes, int method, bool with_tiled,
                   const std::vector<TuneMatrix>& mats, const void* in, void* out, hipStream_t stream, int reps,
                   const FlushBufs* fl, bmmc_options_t* bo, double* best) {
    static const int kShapes[][2] = {{256, 2}, {512, 2}, {256, 4}, {256, 8}, {512, 4}, {512, 8}, {1024, 4}, {256, 16}};
    // tile orders: plain, and neighbouring tiles writing neighbouring runs
    // for the 7 lowest tile-index bits (best for most large arrays)
    static const int kStage1Orders[] = {4, 4 + 16 * 7};
    static const int kOutAdj[] = {0, 2, 4, 5, 6, 7, 8, 9, 10, 12, 15};
    const size_t kBases = 6, kFinal = 8;
    std::vector<std::pair<double, bmmc_options_t>> timed;
    Timer tm;
    hipStream_t cap = make_capture_stream();
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    // cache hints (bit 0 non-temporal loads, bit 1 non-temporal stores, 4
    // none): up to 8 MiB none or stores, up to 64 MiB stores or both (these
    // sizes are timed warm, in graph replays); from 64 MiB on, where each
    // call is timed after a cache flush, all four
    const int hint_set[3][4] = {{4, 2, 0, 0}, {2, 3, 0, 0}, {1, 3, 2, 4}};
    const int hk = bytes >= kFlushFrom ? 2 : bytes > ((size_t)8 << 20) ? 1 : 0;
    const int* hints_of = hint_set[hk];
    const int nh = hk == 2 ? 4 : 2;
    auto persistent_grid = [&](const bmmc_options_t& o) {
        return ds->cu_count * tiled_occupancy(elem_bytes, o.threads, o.iters, 0) * 2;
    };
    // BMMC_TUNE_VERBOSE set: a line on stderr every 32 candidates, so that a
    // long tuning run (minutes for 1 GiB arrays) shows its progress
    static const bool verbose = std::getenv("BMMC_TUNE_VERBOSE") != nullptr;
    size_t ntimed = 0;
    auto run = [&](const bmmc_options_t& o) {
        const double t = time_options(n, elem_bytes, mats, o, in, out, stream, cap, reps, tm, fl);
        if (t > 0) timed.push_back({t, o});  // else: the shape does not fit this size
        if (verbose && ++ntimed % 32 == 0) {
            std::fprintf(stderr, "autotune n=%d w=%d method=%d: %zu settings timed\n", n, elem_bytes, method, ntimed);
            std::fflush(stderr);
        }
    };
    {
        bmmc_options_t o;
        std::memset(&o, 0, sizeof(o));
        o.method = method;
        run(effective_options(ds, n, elem_bytes, &o));
    }
    // runs of at least one 128-byte line on both sides
    int min_run = 7;
    for (int w = elem_bytes; w > 1; w >>= 1) min_run--;
    for (auto& sh : kShapes) {
        if (!tiled_kernel_available(elem_bytes, sh[0], sh[1], 0)) continue;
        KernelShape ks = default_shape(elem_bytes);
        ks.nt = sh[0];
        ks.iters = sh[1];
        const int D = ks.D();
        const int lo = min_run > ks.lv() ? min_run : ks.lv();
        // (read-run, write-run) bits filling the tile, or all but one bit of it
        for (int sum = D; sum >= D - 1; sum--) {
            for (int a = lo; sum - a >= lo; a++) {
                const int b = sum - a;
                for (int m = 0; m < (with_tiled ? 2 : 1); m++) {
                    const bool two = m == 1 || method == BMMC_METHOD_TILED;
                    // two-pass plans also with the scratch kept in the caches
                    for (int hi = 0; hi < (two ? 2 * nh : nh); hi++) {
                        for (int order : kStage1Orders) {
                            for (int g = 0; g < 2; g++) {
                                bmmc_options_t o;
                                std::memset(&o, 0, sizeof(o));
                                // auto also tries the paper's two-pass scheme
                                o.method = m == 0 ? method : BMMC_METHOD_TILED;
                                o.t = a < b ? a : b;
                                o.run_in = a;
                                o.run_out = b;
                                o.threads = ks.nt;
                                o.iters = ks.iters;
                                o.swizzle = 1;
                                o.hints = hints_of[hi % nh] | (hi >= nh ? 8 : 0);
                                o.tile_order = order;
                                o.grid = g == 0 ? -1 : persistent_grid(o);
                                run(o);
                            }
                        }
                    }
                }
            }
        }
    }
    auto by_time = [](const auto& x, const auto& y) { return x.first < y.first; };
    std::sort(timed.begin(), timed.end(), by_time);
    // stage 2: tile orders and grid kinds of the fastest distinct settings
    std::vector<bmmc_options_t> base;
    for (const auto& tv : timed) {
        bool seen = false;
        for (const auto& b : base)
            seen |= b.method == tv.second.method && b.threads == tv.second.threads && b.iters == tv.second.iters &&
                    b.run_in == tv.second.run_in && b.run_out == tv.second.run_out && b.hints == tv.second.hints;
        if (!seen) base.push_back(tv.second);
        if (base.size() == kBases) break;
    }
    for (const bmmc_options_t& b : base) {
        for (int k : kOutAdj) {
            for (int order : {4, 1, 2, 3}) {
                if (k && order >= 2) continue;  // XOR-mixed selection does not combine with k
                for (int g = 0; g < 2; g++) {
                    bmmc_options_t o = b;
                    o.tile_order = order + 16 * k;
                    o.grid = g == 0 ? -1 : persistent_grid(o);
                    run(o);
                }
            }
        }
    }
    *best = 1e30;
    std::memset(bo, 0, sizeof(*bo));
    std::sort(timed.begin(), timed.end(), by_time);
    // the fastest few again, in three interleaved rounds of at least 5 ms
    // of calls each (the best of each candidate's three), so that drift and
    // noise do not pick the winner among settings a percent apart
    const size_t keep = timed.size() < kFinal ? timed.size() : kFinal;
    std::vector<double> again(keep, 1e30);
    for (int round = 0; round < 3; round++)
        for (size_t i = 0; i < keep; i++) {
            const double per_call = timed[i].first / (double)mats.size();
            int r = (int)std::ceil(5.0 / (per_call > 1e-4 ? per_call : 1e-4));
            r = std::max(reps * 2, std::min(r, 200));
            const double t = time_options(n, elem_bytes, mats, timed[i].second, in, out, stream, cap, r, tm, fl);
            if (t > 0 && t < again[i]) again[i] = t;
        }
    for (size_t i = 0; i < keep; i++)
        if (again[i] < *best) {
            *best = again[i];
            *bo = timed[i].second;
        }
    if (*best < 1e30) *best /= (double)mats.size();
    drop_capture_stream(ds, cap);
}

}  // namespace
}  // namespace bmmc

// Time tile shapes, run widths, cache hints, tile order and grid size on a
// random permutation of 2^n elements (class 0) and on a random bit
// permutation (class 1); keep the fastest of each.  Returns class 0's.
extern "C" int bmmc_autotune(int n, int elem_bytes, int method, void* stream_, int reps,
                             bmmc_options_t* best_out, double* best_ms) {
    if (n < 1 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n out of range");
    if (!(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16))
        return set_error(BMMC_ERR_ARG, "bad elem_bytes");
    if (reps < 1) reps = 3;
    int st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    hipStream_t stream = (hipStream_t)stream_;
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    void *in = nullptr, *out = nullptr;
    if (hipMalloc(&in, bytes) != hipSuccess || hipMalloc(&out, bytes) != hipSuccess) {
        if (in) hipFree(in);
        (void)hipGetLastError();
        return set_error(BMMC_ERR_NOMEM, "autotune buffers of %zu bytes", bytes);
    }
    hipMemsetAsync(in, 0x5a, bytes, stream);
    FlushBufs fl;
    if (bytes >= kFlushFrom && !fl.make(stream)) {
        hipFree(in);
        hipFree(out);
        return set_error(BMMC_ERR_NOMEM, "autotune cache-flush buffers of 2 x %zu bytes", kFlushBytes);
    }
    bmmc_options_t bo[2];
    double best[2];
    for (int cls = 0; cls < 2; cls++) {
        // class 0: how a setting's accesses meet the memory system varies
        // from one random matrix to another, most beyond the last-level
        // cache (a spread of 10 % of the copy's rate at 1 GiB): three random
        // matrices, six from 256 MiB on.  Class 1: three bit permutations --
        // a random one, the bit reversal and the transpose of the half split
        // -- so that one setting serves the usual tiled matrices.
        // From 1 GiB on, sixteen: with the score's worst-matrix term, six
        // let settings through that ran one random matrix in eight at
        // 70-75 % of the copy (benchmark seeds 0-7 at 2^28 int32 and 2^27
        // int64) while balanced read and write runs keep all above 80 %.
        const int nrand = bytes >= ((size_t)1 << 30) ? 16 : bytes >= ((size_t)256 << 20) ? 6 : 3;
        std::vector<TuneMatrix> mats(cls == 0 ? nrand : 3);
        if (cls == 0) {
            for (int k = 0; k < nrand; k++)
                random_matrix(n, 0xA5A5A5A5ull + (uint64_t)n + ((uint64_t)k << 40), mats[k].rows, &mats[k].c);
        } else {
            random_bpc(n, 0x5A5A5A5Aull + (uint64_t)n, mats[0].rows, &mats[0].c);
            for (int i = 0; i < n; i++) {
                mats[1].rows[i] = 1ull << (n - 1 - i);
                const int h = n / 2;  // y = (x_low, x_high) swapped
                mats[2].rows[i] = 1ull << (i < n - h ? i + h : i - (n - h));
            }
            mats[1].c = mats[2].c = 0;
        }
        // a tiled matrix is one tiled pass by every method but the general tile
        tune_matrices(ds, n, elem_bytes, method, method == BMMC_METHOD_AUTO && cls == 0, mats, in, out, stream,
                      reps, &fl, &bo[cls], &best[cls]);
    }
    hipStreamSynchronize(stream);
    hipFree(in);
    hipFree(out);
    if (best[0] >= 1e30 || best[1] >= 1e30)
        return set_error(BMMC_ERR_RANGE, "no tile shape fits n = %d, w = %d", n, elem_bytes);
    {
        TuneCache& tc = cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        ensure_loaded(tc);
        for (int cls = 0; cls < 2; cls++) tc.plain[{n, elem_bytes, method, cls}] = {bo[cls], best[cls]};
        autosave(tc);
    }
    if (best_out) *best_out = bo[0];
    if (best_ms) *best_ms = best[0];
    return BMMC_OK;
}

// Time chunk size, queue order and persistent grid size on this batch; keep
// the fastest for batches with the same signature.
extern "C" int bmmc_autotune_batched(const bmmc_desc_t* descs, int count, void* stream_, int reps,
                                     bmmc_batch_options_t* best_out, double* best_ms) {
    int st = batch_validate(descs, count);
    if (st != BMMC_OK) return st;
    if (count == 0) return set_error(BMMC_ERR_ARG, "empty batch");
    if (reps < 1) reps = 3;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    hipStream_t stream = (hipStream_t)stream_;
    static const int kChunks[] = {1, 2, 4, 8, 16};
    double best = 1e30;
    bmmc_batch_options_t bo;
    std::memset(&bo, 0, sizeof(bo));
    Timer tm;
    // time graph replays of a resident batch: device time only
    auto time_batch = [&](const bmmc_batch_options_t& o, double* per) -> int {
        void* pb = nullptr;
        int s2 = bmmc_batch_create(descs, count, &o, &pb);
        if (s2 != BMMC_OK) return s2;
        bmmc_batch_launch(pb, stream);  // warm-up
        hipEventRecord(tm.a, stream);
        for (int r = 0; r < reps; r++) bmmc_batch_launch(pb, stream);
        hipEventRecord(tm.b, stream);
        hipEventSynchronize(tm.b);
        bmmc_batch_destroy(pb);
        float ms = 0;
        hipEventElapsedTime(&ms, tm.a, tm.b);
        *per = ms / reps;
        return BMMC_OK;
    };
    for (int method : {BMMC_METHOD_AUTO, BMMC_METHOD_TILED}) {
        for (int iters : {4, 8, 16, 32}) {
            const int occ = batched_occupancy(iters);
            for (int chunk : kChunks) {
                for (int order = 0; order < 2; order++) {
                    for (int g = 1; g <= 2; g++) {
                        bmmc_batch_options_t o;
                        std::memset(&o, 0, sizeof(o));
                        o.method = method;
                        o.iters = iters;
                        o.chunk_tiles = chunk;
                        o.order = order;
                        o.workgroups = ds->cu_count * occ * g / 2;
                        double per;
                        st = time_batch(o, &per);
                        if (st != BMMC_OK) return st;
                        if (per < best) {
                            best = per;
                            bo = o;
                        }
                    }
                }
            }
        }
    }
    // then the tile order of the best: XOR-mixed selection, or neighbouring
    // tiles writing neighbouring runs for k of the tile-index bits
    const bmmc_batch_options_t base = bo;
    for (int to : {2, 4 + 16 * 2, 4 + 16 * 4, 4 + 16 * 6, 4 + 16 * 7, 4 + 16 * 8, 4 + 16 * 15}) {
        bmmc_batch_options_t o = base;
        o.tile_order = to;
        double per;
        st = time_batch(o, &per);
        if (st != BMMC_OK) return st;
        if (per < best) {
            best = per;
            bo = o;
        }
    }
    // then the cache hints of the best (0 above: non-temporal loads and
    // stores once the batch outgrows the last-level cache)
    const bmmc_batch_options_t base2 = bo;
    for (int h : {1, 2, 3, 4}) {
        bmmc_batch_options_t o = base2;
        o.hints = h;
        double per;
        st = time_batch(o, &per);
        if (st != BMMC_OK) return st;
        if (per < best) {
            best = per;
            bo = o;
        }
    }
    {
        TuneCache& tc = cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        ensure_loaded(tc);
        tc.batch[batch_signature(descs, count)] = {bo, best};
        autosave(tc);
    }
    if (best_out) *best_out = bo;
    if (best_ms) *best_ms = best;
    return BMMC_OK;
}

// Time, on this matrix and these buffers, the options a call would use now
// (the tuned options of its class, else the size defaults) under every tile
// order, then a few other tile shapes under the tile orders that are usually
// best; the fastest few again in three interleaved rounds; keep the winner
// for later calls with this matrix.  Beyond the last-level cache the best
// setting differs from one random matrix to the next (which memory units a
// tile's runs and its neighbours' runs fall on depends on the matrix).
extern "C" int bmmc_autotune_matrix(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                                    int elem_bytes, void* stream_, int reps, bmmc_options_t* best_out,
                                    double* best_ms) {
    if (n < 1 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [1, %d]", n, BMMC_MAX_BITS);
    if (!(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16))
        return set_error(BMMC_ERR_ARG, "elem_bytes = %d not in {1,2,4,8,16}", elem_bytes);
    if (!A_rows) return set_error(BMMC_ERR_ARG, "A_rows is NULL");
    const size_t bytes = ((size_t)1 << n) * (size_t)elem_bytes;
    int st = validate_buffers(in, out, bytes);
    if (st != BMMC_OK) return st;
    if (reps < 1) reps = 3;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    hipStream_t stream = (hipStream_t)stream_;
    std::vector<TuneMatrix> mats(1);
    for (int i = 0; i < n; i++) mats[0].rows[i] = A_rows[i];
    mats[0].c = c;
    // a singular or malformed matrix fails here, before any timing
    st = bmmc_permute_ex(in, out, n, A_rows, c, elem_bytes, nullptr, stream);
    if (st != BMMC_OK) return st;

    bmmc_options_t base;
    std::memset(&base, 0, sizeof(base));
    tuned_options(n, elem_bytes, BMMC_METHOD_AUTO, matrix_class(A_rows, n), &base);
    base = effective_options(ds, n, elem_bytes, &base);
    static const int kOutAdj[] = {0, 2, 4, 5, 6, 7, 8, 9, 10, 12, 15};
    static const int kAltOutAdj[] = {4, 6, 7, 8, 10};
    // (threads, vectors per thread, read-run bits, write-run bits) of 4-byte
    // elements; 8-byte elements take one write-run bit less
    static const int kAltShapes[][4] = {{1024, 4, 6, 8}, {1024, 4, 5, 9}, {512, 8, 6, 8}, {256, 8, 5, 8}, {512, 4, 5, 8}};
    std::vector<bmmc_options_t> cands;
    for (int k : kOutAdj) {
        bmmc_options_t o = base;
        o.tile_order = ((base.tile_order & 7) == 1 ? 1 : 4) + 16 * k;
        cands.push_back(o);
    }
    {
        bmmc_options_t o = base;
        o.tile_order = 2;  // XOR-mixed tile selection
        cands.push_back(o);
    }
    if (bytes >= kFlushFrom) {
        // dealt output blocks (where the matrix allows them; else the plain
        // order), on the base shape and on a 16 KiB tile (512 threads x 2
        // vectors, one work-group per tile: the default's setting for
        // matrices that keep their block bits)
        bmmc_options_t o = base;
        o.tile_order = 256 + 4;
        cands.push_back(o);
        if ((elem_bytes == 4 || elem_bytes == 8) && base.method != BMMC_METHOD_TILED &&
            tiled_kernel_available(elem_bytes, 512, 2, 1)) {
            o.threads = 512;
            o.iters = 2;
            o.run_in = elem_bytes == 4 ? 5 : 4;
            o.run_out = 7;
            o.t = o.run_in;
            o.hints = 1;
            o.grid = -1;
            cands.push_back(o);
        }
    }
    if ((elem_bytes == 4 || elem_bytes == 8) && base.method != BMMC_METHOD_TILED) {
        // read runs longer than write runs, each XCD on its own range of
        // tiles whose neighbours write neighbouring runs (the bit reversal's
        // best beyond the last-level cache)
        static const int kReadHeavy[][4] = {{1024, 4, 8, 6}, {512, 8, 8, 6}, {256, 16, 8, 6}};
        for (const auto& sh : kReadHeavy) {
            const int b = sh[3] - (elem_bytes == 8 ? 1 : 0);
            if (!tiled_kernel_available(elem_bytes, sh[0], sh[1], 0)) continue;
            bmmc_options_t o = base;
            o.threads = sh[0];
            o.iters = sh[1];
            o.run_in = sh[2];
            o.run_out = b;
            o.t = b < sh[2] ? b : sh[2];
            o.tile_order = 1 + 16 * 7;
            if (base.grid > 0) o.grid = ds->cu_count * tiled_occupancy(elem_bytes, o.threads, o.iters, 0) * 2;
            cands.push_back(o);
        }
        for (const auto& sh : kAltShapes) {
            const int b = sh[3] - (elem_bytes == 8 ? 1 : 0);
            if (!tiled_kernel_available(elem_bytes, sh[0], sh[1], 0)) continue;
            if (sh[0] == base.threads && sh[1] == base.iters && sh[2] == base.run_in && b == base.run_out) continue;
            for (int k : kAltOutAdj) {
                bmmc_options_t o = base;
                o.threads = sh[0];
                o.iters = sh[1];
                o.run_in = sh[2];
                o.run_out = b;
                o.t = sh[2] < b ? sh[2] : b;
                o.tile_order = 4 + 16 * k;
                if (base.grid > 0) o.grid = ds->cu_count * tiled_occupancy(elem_bytes, o.threads, o.iters, 0) * 2;
                cands.push_back(o);
            }
        }
    }
    FlushBufs fl;
    if (bytes >= kFlushFrom && !fl.make(stream))
        return set_error(BMMC_ERR_NOMEM, "autotune cache-flush buffers of 2 x %zu bytes", kFlushBytes);
    Timer tm;
    hipStream_t cap = make_capture_stream();
    std::vector<std::pair<double, bmmc_options_t>> timed;
    for (const bmmc_options_t& o : cands) {
        const double t = time_options(n, elem_bytes, mats, o, in, out, stream, cap, reps, tm, &fl);
        if (t > 0) timed.push_back({t, o});  // else: the shape does not fit this size
    }
    std::sort(timed.begin(), timed.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    const size_t keep = timed.size() < 4 ? timed.size() : 4;
    std::vector<double> again(keep, 1e30);
    for (int round = 0; round < 3; round++)
        for (size_t i = 0; i < keep; i++) {
            const double per_call = timed[i].first;
            int r = (int)std::ceil(5.0 / (per_call > 1e-4 ? per_call : 1e-4));
            r = std::max(reps * 2, std::min(r, 200));
            const double t = time_options(n, elem_bytes, mats, timed[i].second, in, out, stream, cap, r, tm, &fl);
            if (t > 0 && t < again[i]) again[i] = t;
        }
    drop_capture_stream(ds, cap);
    double best = 1e30;
    bmmc_options_t bo;
    std::memset(&bo, 0, sizeof(bo));
    for (size_t i = 0; i < keep; i++)
        if (again[i] < best) {
            best = again[i];
            bo = timed[i].second;
        }
    if (best >= 1e30) return set_error(BMMC_ERR_RANGE, "no candidate setting ran for n = %d, w = %d", n, elem_bytes);
    {
        TuneCache& tc = cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        if (tc.matrix.size() >= kMaxMatrixEntries) tc.matrix.clear();
        tc.matrix[matrix_key(n, elem_bytes, A_rows)] = bo;
        tc.nmatrix.store(tc.matrix.size(), std::memory_order_relaxed);
    }
    // `out` holds the permutation of `in` again (every timed call wrote it)
    if (best_out) *best_out = bo;
    if (best_ms) *best_ms = best;
    return BMMC_OK;
}

// Forget every per-matrix setting.
extern "C" int bmmc_tune_clear_matrices(void) {
    TuneCache& tc = cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    tc.matrix.clear();
    tc.nmatrix.store(0, std::memory_order_relaxed);
    return BMMC_OK;
}
