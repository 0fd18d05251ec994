// Batched permutations without device allocation: the batch's descriptor
// table, work items and queue heads live in one fixed device array of this
// file instead of memory the library allocates per stream.
//
// `scratch` is a device-side array.  In host code its name is only a host
// stand-in for the symbol, so the host never passes it to a kernel or a copy:
// on each device, the first call (with that device current) resolves the
// array's device address with hipGetSymbolAddress, and every later use goes
// through that per-device address.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "runtime.hpp"

namespace bmmc {
namespace {

constexpr size_t kFixedTableBytes = (size_t)4 << 20;
static __device__ __align__(256) uint8_t scratch[kFixedTableBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, resolved once.
int fixed_table(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return set_error(BMMC_ERR_HIP, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return BMMC_OK;
}

}  // namespace
}  // namespace bmmc

using namespace bmmc;

extern "C" size_t bmmc_noalloc_table_bytes(void) { return kFixedTableBytes; }

extern "C" int bmmc_permute_batched_noalloc(const bmmc_desc_t* descs, int count, const bmmc_batch_options_t* opts,
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
    if (o.method == BMMC_METHOD_TILED)
        return set_error(BMMC_ERR_ARG, "BMMC_METHOD_TILED needs scratch arrays; the allocation-free call "
                                       "runs one pass per array");
    DeviceState* ds = device_state(&st);
    if (!ds) return st;
    void* table = nullptr;
    st = fixed_table(ds->device, &table);
    if (st != BMMC_OK) return st;
    std::vector<BatchArray> arrays(count);
    for (int i = 0; i < count; i++) {
        st = plan_batch_array(ds, descs[i], o.method, o.iters, &arrays[i], o.tile_order);
        if (st != BMMC_OK) return set_error(st, "array %d: %s", i, bmmc_last_error());
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    return enqueue_batched_fixed(ds, arrays, o, (hipStream_t)stream_, table, kFixedTableBytes);
}
