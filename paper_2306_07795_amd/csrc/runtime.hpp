// Runtime shared by the C entry points: per-device state, plan cache,
// per-stream scratch, error reporting and launch profiling.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "bmmc.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace bmmc {

int set_error(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

struct PlanKey {
    int n, w, method, t, a, b, nt, iters, swizzle, tb_mix, iter_mix;
    uint64_t c;
    uint64_t rows[kMaxBits];
    bool operator==(const PlanKey& o) const;
};
struct PlanKeyHash {
    size_t operator()(const PlanKey& k) const;
};

struct ProfileEvent {
    std::string name;
    double bytes;
    hipEvent_t start, stop;
};

struct DeviceState {
    int device = 0;
    int cu_count = 0;
    int xcds = 8;  // work-groups are dealt round-robin to this many XCDs
    std::mutex mu;
    std::unordered_map<PlanKey, std::shared_ptr<const Plan>, PlanKeyHash> plans;
    struct Scratch {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    std::unordered_map<hipStream_t, Scratch> scratch;
    bool profiling = false;
    std::vector<ProfileEvent> events;
    std::vector<hipEvent_t> event_pool;
};

// State of the current device (created on first use).
DeviceState* device_state(int* status);

// Cached plan for (A, c, n, w, options).
int get_plan(DeviceState* ds, const uint64_t* rows, uint64_t c, int n, int w, const PlanOptions& o,
             std::shared_ptr<const Plan>* out);

// Scratch of at least `bytes` for `stream` (caller holds ds->mu).
int get_scratch(DeviceState* ds, hipStream_t stream, size_t bytes, void** out);

// Timing of one launch when profiling is on (caller holds ds->mu).  With
// one_kernel, the scope's events are bound to the one kernel launched in it
// (its execution, nothing else); otherwise (a graph or several kernels) they
// are recorded on the stream right before (constructor) and after
// (destructor) the work enqueued in the scope.  Streams under capture are not
// timed.
struct LaunchScope {
    DeviceState* ds;
    hipStream_t stream;
    hipEvent_t stop = nullptr;
    bool bound = false;
    LaunchScope(DeviceState* d, hipStream_t s, const char* name, double bytes, bool one_kernel = true);
    ~LaunchScope();
};

// Plan options from the public option struct.
PlanOptions plan_options(const bmmc_options_t* o, int w);
// The options a call runs with: o (NULL = all default) with the library's
// size-dependent defaults of the general one-pass tile filled in where o
// leaves them zero (the persistent grid only when ds is given).
bmmc_options_t effective_options(const DeviceState* ds, int n, int w, const bmmc_options_t* o);
// Launch-time choices from the public option struct (zero = default).
int resolve_hints(const bmmc_options_t* o, size_t bytes);
int resolve_order(const bmmc_options_t* o);

// Enqueue the passes of a plan (caller holds ds->mu).  Two-pass plans use
// `scratch` when given (2^n * w bytes), else the per-stream scratch.
int enqueue_plan(DeviceState* ds, const Plan& plan, const void* in, void* out, hipStream_t stream,
                 uint32_t grid, int hints = 0, int order = 0, void* scratch = nullptr);

int validate_buffers(const void* in, const void* out, size_t bytes);

// One array of a batched launch.
struct BatchArray {
    const void* in = nullptr;
    void* out = nullptr;
    void* scratch = nullptr;  // 2^n * w bytes for two-pass plans
    size_t bytes = 0;
    bool single = false;      // runs through the single-array kernels
    // launch settings of a single array (enqueue_plan's grid, hints, order)
    uint32_t grid = 0;
    int hints = 0, order = 0;
    std::shared_ptr<const Plan> plan;
};

int batch_validate(const bmmc_desc_t* descs, int count);
int plan_batch_array(DeviceState* ds, const bmmc_desc_t& d, int method, int iters, BatchArray* out,
                     int tile_order = 0);
// PlanOptions::tb_mix of a tile_order option (bits 1, 2 and 16*k; 0: -1, automatic)
int tile_order_mix(int tile_order);
// Do the three output bits above a 4 KiB block of w-byte elements depend
// only on the same three input bits (A's rows of those bits inside their
// columns)?  Then dealt output blocks keep each XCD's reads on its own
// eighth of the input blocks too.
bool keeps_block_bits(const uint64_t* rows, int n, int w);
// Arrays above this size (beyond the 256 MB last-level cache) whose matrix
// keeps its block bits get dealt output blocks by default (on 16 KiB tiles
// for 4- and 8-byte elements).
constexpr size_t kDealtFrom = (size_t)256 << 20;
// Those defaults applied to effective options *e (nothing for other arrays).
void dealt_default(bmmc_options_t* e, const uint64_t* rows, int n, int w);
// Plan one array as a single-array call without options would run it (the
// tuned options of its size and matrix class, else the size defaults, for
// `method`); marks it single, with those launch settings.
int plan_single_array(DeviceState* ds, const bmmc_desc_t& d, int method, BatchArray* out);
// Enqueue one batched launch (caller holds ds->mu).
int enqueue_batched(DeviceState* ds, std::vector<BatchArray>& arrays, const bmmc_batch_options_t& o,
                    hipStream_t stream);
// The same with the device table at `table` (cap bytes, owned by the
// caller) and plain launches: allocates no device memory; refuses arrays
// that take two passes and tables larger than cap (caller holds ds->mu).
int enqueue_batched_fixed(DeviceState* ds, std::vector<BatchArray>& arrays, const bmmc_batch_options_t& o,
                          hipStream_t stream, void* table, size_t cap);
// Options a batch takes when the caller gives none: the tuning cache's entry
// for its histogram of (n, width), else the untuned defaults.
void default_batch_options(const bmmc_desc_t* descs, int count, bmmc_batch_options_t* o);
uint64_t batch_signature(const bmmc_desc_t* descs, int count);
// Size the batch table and its pinned staging of `stream` for at least this
// many passes and work items now, so that later batched launches on it do
// not allocate (caller holds ds->mu or owns the stream).
int reserve_batch_state(hipStream_t stream, int device, size_t passes, size_t items);
// Free the batch table of `stream` (its work must have completed).
void release_batch_state(hipStream_t stream, int device);

// Tuning cache lookups (tune.cpp); false when nothing is cached.
// Matrix class of the tuning cache: 1 for a matrix tiled at the default run
// width (bit permutations among them), else 0.
int matrix_class(const uint64_t* rows, int n);
bool tuned_options(int n, int w, int method, int cls, bmmc_options_t* out);
// The options bmmc_autotune_matrix stored for this matrix, if any.
bool matrix_options(int n, int w, const uint64_t* rows, bmmc_options_t* out);
bool tuned_batch_options(uint64_t signature, bmmc_batch_options_t* out);

}  // namespace bmmc
