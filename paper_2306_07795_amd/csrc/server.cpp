// Serving loop: permutation requests arrive over time, are planned, admitted
// against an HBM budget and run with continuous batching.
//
//  * submit() queues a request with its arrival time (the caller's clock is
//    bmmc_server_now_ns; a future arrival time is honoured, so a client can
//    hand over a whole open-loop schedule at once);
//  * planner threads plan requests as they arrive;
//  * the dispatcher admits planned requests in arrival order while their
//    footprint (input + output + scratch) fits the budget, and whenever one
//    of its K streams is free it launches every admitted request on that
//    stream -- a few of them as their own tiled launches, more as one
//    batched persistent launch -- so launches overlap on the device and
//    requests that arrive while others run join the next launch;
//  * completions are seen by polling each stream's event; latency is
//    completion minus arrival.
// Outputs and scratch come from one device arena of `budget` bytes managed as
// a buddy allocator (all sizes are powers of two).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <queue>
#include <set>
#include <sys/prctl.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.hpp"

namespace bmmc {

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Buddy allocator over [0, 2^top) in blocks of 2^min_log bytes.
class Buddy {
   public:
    void init(int top_log, int min_log) {
        top_ = top_log;
        min_ = min_log;
        free_.assign(top_ + 1, {});
        free_[top_].insert(0);
    }
    // Offset of a block of at least `bytes`, or -1.
    int64_t alloc(size_t bytes) {
        int k = min_;
        while (((size_t)1 << k) < bytes) k++;
        if (k > top_) return -1;
        int j = k;
        while (j <= top_ && free_[j].empty()) j++;
        if (j > top_) return -1;
        int64_t off = *free_[j].begin();
        free_[j].erase(free_[j].begin());
        while (j > k) {
            j--;
            free_[j].insert(off + ((int64_t)1 << j));
        }
        size_[off] = k;
        return off;
    }
    void release(int64_t off) {
        auto it = size_.find(off);
        if (it == size_.end()) return;
        int k = it->second;
        size_.erase(it);
        while (k < top_) {
            const int64_t buddy = off ^ ((int64_t)1 << k);
            auto f = free_[k].find(buddy);
            if (f == free_[k].end()) break;
            free_[k].erase(f);
            off = std::min(off, buddy);
            k++;
        }
        free_[k].insert(off);
    }

   private:
    int top_ = 0, min_ = 12;
    std::vector<std::set<int64_t>> free_;
    std::unordered_map<int64_t, int> size_;
};

enum ReqState { kPending = 0, kPlanned, kAdmitted, kRunning, kDone, kFailed };

struct Request {
    int64_t ticket = 0;
    bmmc_desc_t desc{};
    uint64_t rows[64] = {};
    int64_t arrival_ns = 0;
    int64_t planned_ns = 0, launched_ns = 0;
    int64_t done_ns = 0;
    std::shared_ptr<const Plan> plan;
    bool solo = false;  // planned as a single-array call: always its own launch
    uint32_t grid = 0;  // launch settings of its own launch
    int hints = 0, order = 0;
    size_t bytes = 0;
    size_t footprint = 0;
    int64_t out_off = -1, scratch_off = -1;
    void* out = nullptr;
    void* scratch = nullptr;
    int state = kPending;
    int status = BMMC_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request*> reqs;
    bool busy = false;
};

struct ArrivalLater {
    bool operator()(const Request* a, const Request* b) const { return a->arrival_ns > b->arrival_ns; }
};

}  // namespace

struct Server {
    bmmc_server_options_t opt{};
    int device = 0;
    DeviceState* ds = nullptr;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    Buddy buddy;
    int64_t in_use = 0, peak = 0;
    size_t solo_bytes = 0;  // requests this large are planned as single-array calls (0: none)

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    // Bumped with every cv_work notification (new arrivals, planned
    // requests, freed memory, stop): threads that spin instead of sleeping
    // watch it without taking the lock.
    std::atomic<uint64_t> work_epoch{0};
    std::atomic<bool> stopping{false};
    void notify_work() {
        work_epoch.fetch_add(1, std::memory_order_release);
        cv_work.notify_all();
    }
    std::priority_queue<Request*, std::vector<Request*>, ArrivalLater> future;  // not arrived yet
    std::deque<Request*> to_plan, ready, admitted;
    std::unordered_map<int64_t, Request*> table;
    std::vector<Slot> slots;
    int64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> planners;
    std::thread dispatcher;

    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
    double bytes_moved = 0, batch_reqs = 0;
    int64_t first_arrival = -1, last_done = 0;
    std::vector<double> latencies_ms;
    double plan_ms = 0, wait_ms = 0, run_ms = 0;  // sums over completed requests

    void plan_loop();
    void dispatch_loop();
    // Plan r (no lock held), then record the outcome (lock held).
    int plan_request(Request* r, BatchArray* ba, bool* solo);
    void planned(Request* r, int st, const BatchArray& ba, bool solo);
    void finish_slot(Slot& s, int64_t t);
    bool try_admit(Request* r);
    void free_request_memory(Request* r, bool keep_out);
};

void Server::free_request_memory(Request* r, bool keep_out) {
    if (r->scratch_off >= 0) {
        buddy.release(r->scratch_off);
        r->scratch_off = -1;
        r->scratch = nullptr;
    }
    if (!keep_out && r->out_off >= 0) {
        buddy.release(r->out_off);
        r->out_off = -1;
    }
}

bool Server::try_admit(Request* r) {
    const bool two = !r->plan->naive && r->plan->npass == 2;
    r->footprint = r->bytes * (two ? 3 : 2);  // input + output (+ scratch)
    if (in_use + (int64_t)r->footprint > opt.budget_bytes) return false;
    if (opt.own_outputs) {
        r->out_off = buddy.alloc(r->bytes);
        if (r->out_off < 0) return false;
        r->out = (uint8_t*)arena + r->out_off;
        r->desc.out = r->out;
    }
    if (two) {
        r->scratch_off = buddy.alloc(r->bytes);
        if (r->scratch_off < 0) {
            if (r->out_off >= 0) buddy.release(r->out_off);
            r->out_off = -1;
            return false;
        }
        r->scratch = (uint8_t*)arena + r->scratch_off;
    }
    in_use += (int64_t)r->footprint;
    peak = std::max(peak, in_use);
    r->state = kAdmitted;
    return true;
}

int Server::plan_request(Request* r, BatchArray* ba, bool* solo) {
    const size_t bytes = ((size_t)1 << r->desc.n) * (size_t)r->desc.elem_bytes;
    *solo = solo_bytes > 0 && bytes >= solo_bytes && r->desc.elem_bytes >= 4;
    return *solo ? plan_single_array(ds, r->desc, opt.method, ba) : plan_batch_array(ds, r->desc, opt.method, 0, ba);
}

void Server::planned(Request* r, int st, const BatchArray& ba, bool solo) {
    if (st != BMMC_OK) {
        r->status = st;
        r->state = kFailed;
        r->done_ns = now_ns();
        rejected++;
        if (opt.own_outputs == 2) {  // nobody will poll: forget the request
            table.erase(r->ticket);
            delete r;
        }
        cv_done.notify_all();
        return;
    }
    r->plan = ba.plan;
    r->solo = solo;
    r->grid = ba.grid;
    r->hints = ba.hints;
    r->order = ba.order;
    r->state = kPlanned;
    r->planned_ns = now_ns();
    // planners finish out of order: keep `ready` in arrival order
    auto at = ready.end();
    while (at != ready.begin() && (*(at - 1))->arrival_ns > r->arrival_ns) --at;
    ready.insert(at, r);
    notify_work();
}

// Threads that would sleep first spin this long on work_epoch: waking a
// sleeping thread costs tens of microseconds, about the time the whole path
// of a small request takes.
constexpr int64_t kSpinNs = 200000;

void Server::plan_loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (!stop && to_plan.empty()) {
            const uint64_t seen = work_epoch.load(std::memory_order_acquire);
            lk.unlock();
            const int64_t until = now_ns() + kSpinNs;
            while (work_epoch.load(std::memory_order_acquire) == seen && !stopping.load(std::memory_order_relaxed) &&
                   now_ns() < until)
                __builtin_ia32_pause();
            lk.lock();
        }
        cv_work.wait(lk, [&] { return stop || !to_plan.empty(); });
        if (stop) return;
        Request* r = to_plan.front();
        to_plan.pop_front();
        lk.unlock();
        BatchArray ba;
        bool solo = false;
        const int st = plan_request(r, &ba, &solo);
        lk.lock();
        planned(r, st, ba, solo);
    }
}

void Server::finish_slot(Slot& s, int64_t t) {
    for (Request* r : s.reqs) {
        r->done_ns = t;
        r->state = kDone;
        const double lat = (double)(t - r->arrival_ns) * 1e-6;
        latencies_ms.push_back(lat);
        plan_ms += (double)(r->planned_ns - r->arrival_ns) * 1e-6;
        wait_ms += (double)(r->launched_ns - r->planned_ns) * 1e-6;
        run_ms += (double)(t - r->launched_ns) * 1e-6;
        completed++;
        bytes_moved += 2.0 * (double)r->bytes;
        last_done = std::max(last_done, t);
        // The input stops counting once read; the output stays until the
        // client releases it (own_outputs == 1) or is dropped now (== 2).
        const bool keep_out = opt.own_outputs == 1;
        free_request_memory(r, keep_out);
        in_use -= (int64_t)(r->footprint - (keep_out ? r->bytes : 0));
        r->footprint = keep_out ? r->bytes : 0;
        if (opt.own_outputs == 2) {  // nobody will poll: forget the request
            table.erase(r->ticket);
            delete r;
        }
    }
    s.reqs.clear();
    s.busy = false;
}

// Queues up to this many admitted requests count as short (see below).
constexpr size_t kShortQueue = 16;

void Server::dispatch_loop() {
    hipSetDevice(device);
    // Timed waits of this thread end on time: Linux lets a sleeping thread
    // wake up to 50 us late by default, which would sit in every latency.
    prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        bool progress = false;
        const int64_t t = now_ns();
        // arrivals go to the planners (planning in this thread measured
        // worse: an arrival's planning, now and then a plan-cache eviction,
        // held up every other request -- p99 at 20k requests/s 1.55 ms
        // against 0.66 ms)
        while (!future.empty() && future.top()->arrival_ns <= t) {
            to_plan.push_back(future.top());
            future.pop();
            notify_work();
        }
        // completions
        for (Slot& s : slots) {
            if (s.busy && hipEventQuery(s.done) == hipSuccess) {
                finish_slot(s, now_ns());
                progress = true;
                cv_done.notify_all();
            }
        }
        // admission in arrival order
        while (!ready.empty() && try_admit(ready.front())) {
            admitted.push_back(ready.front());
            ready.pop_front();
            progress = true;
        }
        // launch what is admitted on the free streams, in arrival order.
        // While the queue is short (or another stream is free): the leading
        // run of requests planned into a shared launch (small ones)
        // together, or a request planned as its own launch (a large one)
        // alone, the rest to the next free stream, so that small requests do
        // not share a launch, and its completion, with a large one.  When the
        // queue is long (the load exceeds what the streams carry), everything
        // queued in one launch: batching is then what keeps up.
        if (!admitted.empty()) {
            for (size_t si = 0; si < slots.size(); si++) {
                Slot& s = slots[si];
                if (s.busy) continue;
                size_t take = admitted.size();
                if (opt.max_batch > 0) take = std::min(take, (size_t)opt.max_batch);
                bool other_free = false;
                for (size_t sj = si + 1; sj < slots.size(); sj++) other_free |= !slots[sj].busy;
                if (other_free || admitted.size() <= kShortQueue) {
                    size_t k = 0;
                    while (k < take && !admitted[k]->solo) k++;
                    take = k == 0 ? 1 : k;
                }
                std::vector<BatchArray> arrays(take);
                for (size_t i = 0; i < take; i++) {
                    Request* r = admitted[i];
                    BatchArray& ba = arrays[i];
                    ba.in = r->desc.in;
                    ba.out = r->desc.out;
                    ba.scratch = r->scratch;
                    ba.bytes = r->bytes;
                    ba.plan = r->plan;
                    ba.single = r->solo || r->plan->npass == 0 || r->plan->naive || r->desc.elem_bytes < 4;
                    ba.grid = r->grid;
                    ba.hints = r->hints;
                    ba.order = r->order;
                    r->state = kRunning;
                    r->launched_ns = now_ns();
                    s.reqs.push_back(r);
                }
                admitted.erase(admitted.begin(), admitted.begin() + take);
                bmmc_batch_options_t bo;
                std::memset(&bo, 0, sizeof(bo));
                bo.method = opt.method;
                bo.use_graph = opt.use_graph > 0 ? 1 : -1;
                int st = BMMC_OK;
                {
                    std::lock_guard<std::mutex> dl(ds->mu);
                    const int direct_max = opt.direct_max == 0 ? 4 : opt.direct_max;
                    if ((int64_t)take <= (int64_t)direct_max) {
                        // a few arrays: their own tiled launches (tables in the
                        // kernel arguments, no table upload, no persistent grid)
                        for (size_t i = 0; i < take && st == BMMC_OK; i++) {
                            const BatchArray& ba = arrays[i];
                            st = enqueue_plan(ds, *ba.plan, ba.in, ba.out, s.stream, ba.grid, ba.hints,
                                              ba.order, ba.scratch);
                        }
                    } else {
                        st = enqueue_batched(ds, arrays, bo, s.stream);
                    }
                }
                if (st == BMMC_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = BMMC_ERR_HIP;
                if (st != BMMC_OK) {
                    // launches enqueued before the failure may still use the
                    // requests' memory: let them end before it is freed
                    (void)hipStreamSynchronize(s.stream);
                    for (Request* r : s.reqs) {
                        r->status = st;
                        r->state = kFailed;
                        r->done_ns = now_ns();
                        free_request_memory(r, false);
                        in_use -= (int64_t)r->footprint;
                        r->footprint = 0;
                        rejected++;
                        if (opt.own_outputs == 2) {
                            table.erase(r->ticket);
                            delete r;
                        }
                    }
                    s.reqs.clear();
                    cv_done.notify_all();
                } else {
                    s.busy = true;
                    batches++;
                    batch_reqs += (double)take;
                }
                progress = true;
                if (admitted.empty()) break;
            }
        }
        if (!progress) {
            // While a stream is busy or an arrival is near, spin: until new
            // work is queued, the next arrival is due or a busy stream
            // completes (the streams' events are this thread's own).
            bool busy_now = false;
            for (Slot& s : slots) busy_now |= s.busy;
            const int64_t next_arrival = future.empty() ? INT64_MAX : future.top()->arrival_ns;
            const int64_t t0 = now_ns();
            if (busy_now || next_arrival - t0 < kSpinNs) {
                const uint64_t seen = work_epoch.load(std::memory_order_acquire);
                lk.unlock();
                const int64_t until = std::min(t0 + kSpinNs, next_arrival);
                for (;;) {
                    if (work_epoch.load(std::memory_order_acquire) != seen || stopping.load(std::memory_order_relaxed))
                        break;
                    if (now_ns() >= until) break;
                    bool done = false;
                    for (Slot& s : slots) done |= s.busy && hipEventQuery(s.done) == hipSuccess;
                    if (done) break;
                    __builtin_ia32_pause();
                }
                lk.lock();
                continue;
            }
            // Otherwise sleep until new work arrives or briefly, to poll the
            // streams every 5 us.
            int64_t wait_ns = 5000;
            if (!future.empty()) wait_ns = std::min<int64_t>(wait_ns, std::max<int64_t>(0, future.top()->arrival_ns - now_ns()));
            bool any_busy = false;
            for (Slot& s : slots) any_busy |= s.busy;
            if (!any_busy && future.empty() && ready.empty() && to_plan.empty())
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else if (wait_ns > 0)
                cv_work.wait_for(lk, std::chrono::nanoseconds(wait_ns));
        }
    }
}

}  // namespace bmmc

using namespace bmmc;

extern "C" int64_t bmmc_server_now_ns(void) { return now_ns(); }

namespace bmmc {
namespace {

// Latency percentiles and means of completed requests into *out.
void fill_latency_stats(std::vector<double> v, bmmc_server_stats_t* out) {
    if (v.empty()) return;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        size_t k = (size_t)(p * (double)(v.size() - 1) + 0.5);
        return v[std::min(k, v.size() - 1)];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / (double)v.size();
    out->max_ms = v.back();
}

// One stream of the unbatched baseline: an issuing thread that calls
// bmmc_permute for each of its requests at the request's arrival time and
// records an event after it, and a waiting thread that stamps each request's
// completion when its event has passed.
struct DirectLane {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ring;  // event slots, reused in issue order
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::pair<int, size_t>> issued;  // (request, event slot)
    size_t n_issued = 0, n_done = 0;
    bool finished = false;
};

}  // namespace
}  // namespace bmmc

extern "C" int bmmc_serve_direct(const bmmc_desc_t* descs, const int64_t* arrival_ns, int count, int streams,
                                 bmmc_server_stats_t* stats_out) {
    if (!stats_out || count < 0 || (count > 0 && (!descs || !arrival_ns)))
        return set_error(BMMC_ERR_ARG, "NULL argument");
    if (streams <= 0) streams = 4;
    if (streams > 16) return set_error(BMMC_ERR_ARG, "streams = %d above 16", streams);
    // each request on its own (requests of one stream run in order, so they
    // may share an output buffer)
    for (int k = 0; k < count; k++) {
        const bmmc_desc_t& d = descs[k];
        if (d.n < 0 || d.n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "request %d: n = %d", k, d.n);
        const int w = d.elem_bytes;
        if (!(w == 1 || w == 2 || w == 4 || w == 8 || w == 16))
            return set_error(BMMC_ERR_ARG, "request %d: elem_bytes = %d", k, w);
        if (d.n > 0 && !d.A_rows) return set_error(BMMC_ERR_ARG, "request %d: A_rows is NULL", k);
        const int s0 = validate_buffers(d.in, d.out, ((size_t)1 << d.n) * (size_t)w);
        if (s0 != BMMC_OK) return set_error(s0, "request %d: %s", k, bmmc_last_error());
    }
    int st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    const int device = ds->device;
    constexpr size_t kRing = 1024;
    std::vector<DirectLane> lanes(streams);
    for (DirectLane& L : lanes) {
        hipError_t e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        for (size_t i = 0; e == hipSuccess && i < kRing; i++) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) L.ring.push_back(ev);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (DirectLane& M : lanes) {
                for (hipEvent_t ev : M.ring) hipEventDestroy(ev);
                if (M.stream) hipStreamDestroy(M.stream);
            }
            return set_error(BMMC_ERR_HIP, "baseline stream or event: %s", hipGetErrorString(e));
        }
    }
    std::vector<int64_t> issued_ns(count, 0), done_ns(count, 0);
    std::vector<int> status(count, BMMC_OK);
    std::vector<std::thread> threads;
    for (int li = 0; li < streams; li++) {
        DirectLane* L = &lanes[li];
        threads.emplace_back([&, L, li] {
            hipSetDevice(device);
            prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
            for (int k = li; k < count; k += streams) {
                // wait for the arrival: sleep while it is far, then spin
                for (;;) {
                    const int64_t left = arrival_ns[k] - now_ns();
                    if (left <= 0) break;
                    if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
                }
                size_t slot;
                {
                    std::unique_lock<std::mutex> lk(L->mu);
                    L->cv.wait(lk, [&] { return L->n_issued - L->n_done < kRing; });
                    slot = L->n_issued % kRing;
                }
                const bmmc_desc_t& d = descs[k];
                int s2 = bmmc_permute(d.in, d.out, d.n, d.A_rows, d.c, d.elem_bytes, L->stream);
                if (s2 == BMMC_OK && hipEventRecord(L->ring[slot], L->stream) != hipSuccess) s2 = BMMC_ERR_HIP;
                issued_ns[k] = now_ns();
                status[k] = s2;
                std::lock_guard<std::mutex> lk(L->mu);
                if (s2 == BMMC_OK) {
                    L->issued.push_back({k, slot});
                    L->n_issued++;
                }
                L->cv.notify_all();
            }
            std::lock_guard<std::mutex> lk(L->mu);
            L->finished = true;
            L->cv.notify_all();
        });
        threads.emplace_back([&, L] {
            hipSetDevice(device);
            for (;;) {
                std::pair<int, size_t> job;
                {
                    std::unique_lock<std::mutex> lk(L->mu);
                    L->cv.wait(lk, [&] { return !L->issued.empty() || L->finished; });
                    if (L->issued.empty()) return;
                    job = L->issued.front();
                    L->issued.pop_front();
                }
                const hipError_t e = hipEventSynchronize(L->ring[job.second]);
                done_ns[job.first] = now_ns();
                if (e != hipSuccess) status[job.first] = BMMC_ERR_HIP;
                std::lock_guard<std::mutex> lk(L->mu);
                L->n_done++;
                L->cv.notify_all();
            }
        });
    }
    for (auto& t : threads) t.join();
    for (DirectLane& L : lanes) {
        hipStreamSynchronize(L.stream);
        for (hipEvent_t ev : L.ring) hipEventDestroy(ev);
        hipStreamDestroy(L.stream);
    }
    bmmc_server_stats_t& out = *stats_out;
    std::memset(&out, 0, sizeof(out));
    out.submitted = count;
    std::vector<double> lat;
    int64_t first = -1, last = 0;
    double plan = 0, run = 0;
    for (int k = 0; k < count; k++) {
        if (status[k] != BMMC_OK) {
            out.rejected++;
            continue;
        }
        out.completed++;
        out.bytes_moved += 2.0 * (double)((size_t)1 << descs[k].n) * (double)descs[k].elem_bytes;
        lat.push_back((double)(done_ns[k] - arrival_ns[k]) * 1e-6);
        plan += (double)(issued_ns[k] - arrival_ns[k]) * 1e-6;
        run += (double)(done_ns[k] - issued_ns[k]) * 1e-6;
        if (first < 0 || arrival_ns[k] < first) first = arrival_ns[k];
        last = std::max(last, done_ns[k]);
    }
    out.batches = out.completed;
    out.mean_batch = out.completed ? 1.0 : 0.0;
    out.busy_s = first >= 0 ? (double)(last - first) * 1e-9 : 0.0;
    if (out.completed) {
        out.mean_plan_ms = plan / (double)out.completed;
        out.mean_run_ms = run / (double)out.completed;
    }
    fill_latency_stats(lat, &out);
    for (int k = 0; k < count; k++)
        if (status[k] != BMMC_OK) return set_error(status[k], "request %d failed: %s", k, bmmc_strerror(status[k]));
    return BMMC_OK;
}

extern "C" int bmmc_server_create(const bmmc_server_options_t* opts, void** handle_out) {
    if (!opts || !handle_out) return set_error(BMMC_ERR_ARG, "opts/handle_out is NULL");
    if (opts->budget_bytes < (1 << 20)) return set_error(BMMC_ERR_ARG, "budget below 1 MiB");
    if (opts->solo_log2 > 40) return set_error(BMMC_ERR_ARG, "solo_log2 = %d above 40", opts->solo_log2);
    int st;
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    auto* s = new Server();
    s->opt = *opts;
    if (s->opt.streams <= 0) s->opt.streams = 4;
    if (s->opt.streams > 16) s->opt.streams = 16;
    s->solo_bytes = s->opt.solo_log2 < 0 ? 0 : (size_t)1 << (s->opt.solo_log2 == 0 ? 24 : s->opt.solo_log2);
    s->ds = ds;
    s->device = ds->device;
    // Arena: the largest power of two not above the budget, for outputs and scratch.
    int top = 20;
    while (((int64_t)1 << (top + 1)) <= s->opt.budget_bytes && top < 46) top++;
    s->arena_bytes = (size_t)1 << top;
    hipError_t e = hipMalloc(&s->arena, s->arena_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return set_error(BMMC_ERR_NOMEM, "server arena of %zu bytes: %s", (size_t)1 << top, hipGetErrorString(e));
    }
    s->buddy.init(top, 12);
    s->slots.resize(s->opt.streams);
    for (Slot& sl : s->slots) {
        hipError_t e2 = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e2 != hipSuccess) {
            (void)hipGetLastError();
            bmmc_server_destroy(s);
            return set_error(BMMC_ERR_HIP, "server stream or event: %s", hipGetErrorString(e2));
        }
        // the batch table of each stream made now: allocating it (device
        // memory, pinned staging) while serving would stall every stream
        const int st2 = reserve_batch_state(sl.stream, ds->device, 128, 8192);
        if (st2 != BMMC_OK) {
            bmmc_server_destroy(s);
            return st2;
        }
    }
    // Planning a random BMMC costs tens of microseconds; at tens of
    // thousands of requests per second several planners keep up.
    for (int k = 0; k < 4; k++) s->planners.emplace_back([s] { s->plan_loop(); });
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    *handle_out = s;
    return BMMC_OK;
}

extern "C" int bmmc_server_submit(void* handle, const bmmc_desc_t* desc, int64_t arrival_ns, int64_t* ticket_out) {
    Server* s = (Server*)handle;
    if (!s || !desc || !ticket_out) return set_error(BMMC_ERR_ARG, "NULL argument");
    const bmmc_desc_t& d = *desc;
    if (d.n < 0 || d.n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n out of range");
    if (!(d.elem_bytes == 1 || d.elem_bytes == 2 || d.elem_bytes == 4 || d.elem_bytes == 8 || d.elem_bytes == 16))
        return set_error(BMMC_ERR_ARG, "bad elem_bytes");
    if (d.n > 0 && !d.A_rows) return set_error(BMMC_ERR_ARG, "A_rows is NULL");
    const size_t bytes = ((size_t)1 << d.n) * (size_t)d.elem_bytes;
    if (!d.in || ((uintptr_t)d.in & 15u)) return set_error(BMMC_ERR_ARG, "in must be 16-byte aligned device memory");
    if (!s->opt.own_outputs) {
        int st = validate_buffers(d.in, d.out, bytes);
        if (st != BMMC_OK) return st;
    }
    if ((int64_t)(3 * bytes) > s->opt.budget_bytes || bytes > s->arena_bytes / 2)
        return set_error(BMMC_ERR_NOMEM, "request of %zu bytes can never fit the budget", bytes);
    auto* r = new Request();
    r->desc = d;
    for (int i = 0; i < d.n; i++) r->rows[i] = d.A_rows[i];
    r->desc.A_rows = r->rows;
    r->arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
    r->bytes = bytes;
    r->footprint = 0;  // set at admission
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->table[r->ticket] = r;
    s->submitted++;
    if (s->first_arrival < 0 || r->arrival_ns < s->first_arrival) s->first_arrival = r->arrival_ns;
    s->future.push(r);
    s->notify_work();
    *ticket_out = r->ticket;
    return BMMC_OK;
}

extern "C" int bmmc_server_poll(void* handle, int64_t ticket, int wait, int64_t* done_ns, void** out_ptr) {
    Server* s = (Server*)handle;
    if (!s) return set_error(BMMC_ERR_ARG, "NULL handle");
    // Requests of own_outputs == 2 are freed when they finish: waiting on one
    // could outlive it, so such tickets can only be polled without waiting
    // (BMMC_ERR_BUSY while pending, BMMC_ERR_NOTFOUND once finished).
    if (wait && s->opt.own_outputs == 2)
        return set_error(BMMC_ERR_ARG, "tickets of a server with own_outputs == 2 cannot be waited on");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return set_error(BMMC_ERR_NOTFOUND, "unknown ticket %lld", (long long)ticket);
    Request* r = it->second;
    if (wait) s->cv_done.wait(lk, [&] { return r->state == kDone || r->state == kFailed; });
    if (r->state == kFailed) return set_error(r->status, "request failed: %s", bmmc_strerror(r->status));
    if (r->state != kDone) return BMMC_ERR_BUSY;
    if (done_ns) *done_ns = r->done_ns;
    if (out_ptr) *out_ptr = r->desc.out;
    return BMMC_OK;
}

extern "C" int bmmc_server_release(void* handle, int64_t ticket) {
    Server* s = (Server*)handle;
    if (!s) return set_error(BMMC_ERR_ARG, "NULL handle");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return set_error(BMMC_ERR_NOTFOUND, "unknown ticket %lld", (long long)ticket);
    Request* r = it->second;
    if (r->state != kDone && r->state != kFailed) return set_error(BMMC_ERR_BUSY, "request still running");
    if (r->out_off >= 0) {
        s->buddy.release(r->out_off);
        r->out_off = -1;
    }
    s->in_use -= (int64_t)r->footprint;
    r->footprint = 0;
    s->table.erase(it);
    delete r;
    s->notify_work();
    return BMMC_OK;
}

extern "C" int bmmc_server_drain(void* handle) {
    Server* s = (Server*)handle;
    if (!s) return set_error(BMMC_ERR_ARG, "NULL handle");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        for (auto& kv : s->table)
            if (kv.second->state != kDone && kv.second->state != kFailed) return false;
        return true;
    });
    return BMMC_OK;
}

extern "C" int bmmc_server_stats(void* handle, bmmc_server_stats_t* out) {
    Server* s = (Server*)handle;
    if (!s || !out) return set_error(BMMC_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->batches = s->batches;
    out->bytes_moved = s->bytes_moved;
    out->busy_s = s->first_arrival >= 0 ? (double)(s->last_done - s->first_arrival) * 1e-9 : 0.0;
    out->in_use_bytes = s->in_use;
    out->peak_bytes = s->peak;
    out->mean_batch = s->batches ? s->batch_reqs / (double)s->batches : 0.0;
    if (s->completed) {
        out->mean_plan_ms = s->plan_ms / (double)s->completed;
        out->mean_wait_ms = s->wait_ms / (double)s->completed;
        out->mean_run_ms = s->run_ms / (double)s->completed;
    }
    fill_latency_stats(s->latencies_ms, out);
    return BMMC_OK;
}

extern "C" int bmmc_server_reset_stats(void* handle) {
    Server* s = (Server*)handle;
    if (!s) return set_error(BMMC_ERR_ARG, "NULL handle");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->rejected = s->batches = 0;
    s->bytes_moved = s->batch_reqs = 0;
    s->first_arrival = -1;
    s->last_done = 0;
    s->latencies_ms.clear();
    s->plan_ms = s->wait_ms = s->run_ms = 0;
    s->peak = s->in_use;
    return BMMC_OK;
}

extern "C" int bmmc_server_destroy(void* handle) {
    Server* s = (Server*)handle;
    if (!s) return set_error(BMMC_ERR_ARG, "NULL handle");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->stopping.store(true);
        s->notify_work();
    }
    for (auto& t : s->planners) t.join();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    for (Slot& sl : s->slots) {
        if (!sl.stream) continue;
        hipStreamSynchronize(sl.stream);
        release_batch_state(sl.stream, s->device);
        hipStreamDestroy(sl.stream);
        if (sl.done) hipEventDestroy(sl.done);
    }
    hipFree(s->arena);
    for (auto& kv : s->table) delete kv.second;
    while (!s->future.empty()) s->future.pop();
    delete s;
    return BMMC_OK;
}
