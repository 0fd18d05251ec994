// Launchers for the gfx950 kernels (definitions in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pass.hpp"

namespace bmmc {

// Column masks of A for the naive kernel: col[j] = A.e_j (0 for j >= n).
struct NaiveArgs {
    uint32_t n;
    uint32_t c;
    uint32_t col[kMaxTbBits];
};

// True when a tiled kernel exists for (w, nt, iters, hints); hints bit 0
// selects non-temporal loads, bit 1 non-temporal stores.
bool tiled_kernel_available(int w, int nt, int iters, int hints = 0);

// One LDS-staged pass over `ntiles` tiles with `grid` work-groups
// (grid-stride over tiles).  in/out are 16-byte aligned device pointers.
// xcds > 0: give each of the xcds XCDs (which receive work-groups
// round-robin) a contiguous range of tiles.
hipError_t launch_tiled(int w, int nt, int iters, int hints, const void* in, void* out,
                        const PassTables& tab, uint32_t ntiles, uint32_t grid, uint32_t xcds,
                        hipStream_t stream);

// Tiled pass of 4-byte keys that runs the sorting-network columns `cols` on
// each staged tile in LDS before writing it (op 1: int32 order, 2: uint32).
// Shapes (nt, iters) = (256, 8) and (256, 4).
bool tiled_net_available(int nt, int iters);
hipError_t launch_tiled_net(int nt, int iters, int op, bool regs, const void* in, void* out, const PassTables& tab,
                            const NetColumns& cols, uint32_t ntiles, uint32_t grid, hipStream_t stream);

// One sorting-network column in place at the keys' own positions: the pair k
// sits at Q.(2k) and Q.(2k) XOR Q.e_0, col[j] = Q.e_j (0 for j >= n), n >= 1.
struct DirectArgs {
    uint32_t n;
    uint32_t col[kMaxTbBits];
};
hipError_t launch_cmp_direct(void* data, const DirectArgs& args, int op, hipStream_t stream);

// Naive kernel: 2^n elements, one 16-byte vector (or one element when
// 2^n * w < 16 * 256) per lane, scattered element stores.
hipError_t launch_naive(int w, int n, const void* in, void* out, const NaiveArgs& args,
                        hipStream_t stream);

// 16-byte vector copy of `bytes` bytes (tail handled bytewise), vpt vectors
// per lane (1, 2, 4, 8).
hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t stream, int vpt = 4,
                       int hints = 0);

// Batched persistent kernel: runs items range[phase] .. range[phase + 1]
// (device pointers; *head must be zero at launch) with tiles of 256 threads x
// `iters` (4 or 8) 16-byte vectors.
hipError_t launch_batched(const BatchPass* passes, const BatchItem* items, const uint32_t* range,
                          uint32_t phase, uint32_t* head, uint32_t grid, int hints, int size, hipStream_t stream);
// Resident work-groups per CU of the batched kernel / of a tiled kernel.
int batched_occupancy(int size);
int tiled_occupancy(int w, int nt, int iters, int hints = 0);
// Shape of the batched kernel's tile by its size, the tile's 16-byte vectors
// over 256 (the batch option `iters`): 4 (default) -> 256 threads x 4
// vectors, 8 -> 256 x 8, 16 -> 512 x 8, 32 -> 1024 x 8.
inline int batched_size(int asked) { return asked == 8 || asked == 16 || asked == 32 ? asked : 4; }
inline int batched_threads(int size) { return size == 32 ? 1024 : size == 16 ? 512 : 256; }
inline int batched_vectors(int size) { return size >= 16 ? 8 : size; }

// Timing events bound to the next kernel launched by this thread through the
// launchers above (hipExtLaunchKernel): their interval is that kernel's
// execution.  A pair serves one launch; kernel_events_pending() tells whether
// it is still unused.  Null events: plain launches.
void set_kernel_events(hipEvent_t start, hipEvent_t stop);
bool kernel_events_pending();

// Clears `count` 32-bit words with a kernel (no memset nodes in graphs).
hipError_t launch_zero(uint32_t* p, uint32_t count, hipStream_t stream);

}  // namespace bmmc
