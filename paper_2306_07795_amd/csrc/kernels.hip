// gfx950 kernels for BMMC permutations: the LDS-staged tiled pass, the naive
// direct-index kernel, the vector copy and the batched persistent kernel.
//
// Every index computation is XOR-linear (see pass.hpp): a lane's input and
// output addresses are a per-tile scalar part XOR a per-thread part computed
// once XOR a compile-time-selected per-iteration part, so the per-element cost
// is one XOR and one shift whatever the matrix.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <type_traits>

#include "kernels.hpp"

namespace bmmc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// The same vector in the global address space: accesses through these
// pointers are global (not flat) loads and stores, which count only against
// the vector-memory counter and so never hold up waits on LDS or scalar loads.
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

template <int W> struct ElemT;
template <> struct ElemT<1> { using T = uint8_t; };
template <> struct ElemT<2> { using T = uint16_t; };
template <> struct ElemT<4> { using T = uint32_t; };
template <> struct ElemT<8> { using T = uint64_t; };
template <> struct ElemT<16> { using T = u32x4; };

// 16 bytes seen either as one vector or as 16/W elements.
template <int W>
union Vec16 {
    u32x4 v;
    typename ElemT<W>::T e[16 / W];
};

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Timing events for the next kernel this thread launches (profiling): the
// runtime binds them to the kernel's own dispatch, so their interval is the
// kernel's execution, with no marker commands between kernels.  A pair is
// used by one launch only.
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

void set_kernel_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

bool kernel_events_pending() { return t_ev_start != nullptr; }

template <typename F, typename... Args>
static void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (t_ev_start) {
        hipEvent_t a = t_ev_start, b = t_ev_stop;
        t_ev_start = t_ev_stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

// 16-byte global accesses; HINT bit 0 marks loads and bit 1 stores as
// non-temporal (streamed, not kept in the caches).
template <int HINT>
__device__ __forceinline__ u32x4 ld16(const g_u32x4* p) {
    if constexpr (HINT & 1) return __builtin_nontemporal_load(p);
    else return *p;
}
template <int HINT>
__device__ __forceinline__ void st16(g_u32x4* p, u32x4 v) {
    if constexpr (HINT & 2) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// XOR of tab[BASE + k] over the set bits k of a compile-time value.
template <int BASE, int NBITS>
__device__ __forceinline__ uint32_t lin_const(const uint32_t* tab, uint32_t v) {
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < NBITS; k++)
        if ((v >> k) & 1u) r ^= tab[BASE + k];
    return r;
}

// ---------------------------------------------------------------------------
// One tile of a pass (paper, Section 4.1 kernel with the tiled-BMMC output
// address of Section 5.1 and the iterations of Section 4.3):
//   read phase : each thread loads ITERS 16-byte vectors, each lying in one
//                contiguous run of the input, and scatters their elements to
//                LDS slots F(v);
//   barrier;
//   write phase: each thread gathers the elements of ITERS output vectors from
//                LDS slots G(u) and stores them to contiguous output runs.
// The slot of a thread's element e of vector `it` is
//   s = it * NT * VEC + tid * VEC + e.
// Slots at or above 2^d do not exist when the array is smaller than the tile.
// ---------------------------------------------------------------------------
template <int W, int NT, int ITERS, int HINT = 0>
struct TileCtx {
    using E = typename ElemT<W>::T;
    static constexpr int VEC = 16 / W;
    static constexpr int LV = ilog2(VEC);
    static constexpr int LT = ilog2(NT);
    static constexpr int LI = ilog2(ITERS);
    static constexpr int D = LV + LT + LI;

    uint32_t xt, ft, yt, gt;  // per-thread parts
    uint32_t vlim;            // valid vector slots

    __device__ __forceinline__ void init(const PassTables& P, uint32_t tid) {
        xt = ft = yt = gt = 0;
#pragma unroll
        for (int k = 0; k < LT; k++) {
            const uint32_t m = 0u - ((tid >> k) & 1u);
            xt ^= P.X[LV + k] & m;
            ft ^= P.F[LV + k] & m;
            yt ^= P.Y[LV + k] & m;
            gt ^= P.G[LV + k] & m;
        }
        vlim = 1u << (P.d - LV);
    }

    // Per-tile parts: coset representative r (input), output base yb and LDS
    // offset gx, each the XOR of the tile-selecting vectors of the tile
    // index's set bits.  Uniform over the work-group: a short scalar loop
    // over the set bits only, one 16-byte scalar load per bit.
    struct Parts {
        uint32_t r, yb, gx;
    };
    __device__ __forceinline__ Parts parts(const PassTables& P, uint32_t tile) const {
        Parts p{0u, P.c_hi, P.c_lds};
        for (uint32_t m = tile; m; m &= m - 1) {
            const uint32_t j = __builtin_ctz(m);
            p.r ^= P.tb[j][0];
            p.yb ^= P.tb[j][1];
            p.gx ^= P.tb[j][2];
        }
        return p;
    }

    // Read phase, global part: ITERS 16-byte loads, each inside one input run.
    __device__ __forceinline__ void load(const PassTables& P, const g_u32x4* __restrict__ in, uint32_t r,
                                         uint32_t tid, Vec16<W>* buf) const {
#pragma unroll
        for (int it = 0; it < ITERS; it++) {
            if ((uint32_t)(it * NT) + tid < vlim) {
                const uint32_t x = r ^ xt ^ lin_const<LV + LT, LI>(P.X, it);
                buf[it].v = ld16<HINT>(in + (x >> LV));
            }
        }
    }

    // Read phase, LDS part: each element to its swizzled slot F(v).  With
    // RECOMPUTE the slots are recomputed for every tile (a few XORs) rather
    // than kept in registers across tiles, which frees registers for a
    // register-hungry mid step; the empty asm hides that ftl equals ft.
    template <bool RECOMPUTE>
    __device__ __forceinline__ void to_lds(const PassTables& P, E* lds, uint32_t tid, const Vec16<W>* buf) const {
        uint32_t ftl = ft;
        if constexpr (RECOMPUTE) asm volatile("" : "+v"(ftl));
#pragma unroll
        for (int it = 0; it < ITERS; it++) {
            if ((uint32_t)(it * NT) + tid < vlim) {
                const uint32_t f = ftl ^ lin_const<LV + LT, LI>(P.F, it);
#pragma unroll
                for (int e = 0; e < VEC; e++) lds[f ^ lin_const<0, LV>(P.F, e)] = buf[it].e[e];
            }
        }
    }

    // Write phase: gather each output vector from slots G(u), store it to
    // one output run at T.r XOR c XOR Y(u).
    __device__ __forceinline__ void store(const PassTables& P, g_u32x4* __restrict__ out, const E* lds,
                                          const Parts& pt, uint32_t tid) const {
#pragma unroll
        for (int it = 0; it < ITERS; it++) {
            if ((uint32_t)(it * NT) + tid < vlim) {
                const uint32_t g = gt ^ pt.gx ^ lin_const<LV + LT, LI>(P.G, it);
                Vec16<W> o;
#pragma unroll
                for (int e = 0; e < VEC; e++) o.e[e] = lds[g ^ lin_const<0, LV>(P.G, e)];
                const uint32_t y = pt.yb ^ yt ^ lin_const<LV + LT, LI>(P.Y, it);
                st16<HINT>(out + (y >> LV), o.v);
            }
        }
    }

    // Tiles first, first + step, ... below last.  The loads of the next tile
    // are issued right after the barrier that ends the current tile's LDS
    // writes, so they are in flight while the current tile is written out.
    // mid(parts) runs on the staged tile before it is written out (its own
    // barriers included).
    struct NoMid {
        __device__ __forceinline__ void operator()(const Parts&) const {}
    };
    template <typename Mid = NoMid>
    __device__ __forceinline__ void run_tiles(const PassTables& P, const g_u32x4* __restrict__ in,
                                              g_u32x4* __restrict__ out, E* lds, uint32_t first,
                                              uint32_t last, uint32_t step, uint32_t tid,
                                              const Mid& mid = Mid()) const {
        if (first >= last) return;
        Vec16<W> buf[ITERS];
        uint32_t tile = first;
        Parts cur = parts(P, tile);
        load(P, in, cur.r, tid, buf);
        for (;;) {
            to_lds<!std::is_same<Mid, NoMid>::value>(P, lds, tid, buf);
            __syncthreads();
            const uint32_t next = tile + step;
            const bool more = next < last;
            Parts nxt = cur;
            if (more) {
                nxt = parts(P, next);
                load(P, in, nxt.r, tid, buf);
            }
            mid(cur);
            store(P, out, lds, cur, tid);
            __syncthreads();
            if (!more) break;
            tile = next;
            cur = nxt;
        }
    }
};

// Work-groups are dealt to the XCDs round-robin (block b runs on XCD
// b mod xcds).  With xcds > 0, renumber them so that each XCD owns one
// contiguous range of logical blocks, hence of tiles: the work-groups sharing
// an XCD's L2 then cover every value of the low tile bits.
__device__ __forceinline__ uint32_t logical_block(uint32_t xcds) {
    const uint32_t b = blockIdx.x;
    if (xcds <= 1) return b;
    const uint32_t g = gridDim.x, per = g / xcds, rem = g % xcds;
    const uint32_t x = b % xcds, k = b / xcds;
    return x * per + (x < rem ? x : rem) + k;
}

template <int W, int NT, int ITERS, int HINT>
__global__ void __launch_bounds__(NT)
k_tiled(const u32x4* __restrict__ in, u32x4* __restrict__ out, const PassTables P, uint32_t ntiles,
        uint32_t xcds) {
    using C = TileCtx<W, NT, ITERS, HINT>;
    __shared__ typename C::E lds[1 << C::D];
    C ctx;
    ctx.init(P, threadIdx.x);
    ctx.run_tiles(P, (const g_u32x4*)in, (g_u32x4*)out, lds, logical_block(xcds), ntiles, gridDim.x,
                  threadIdx.x);
}

struct TiledEntry {
    int w, nt, iters, hints;
    void (*fn)(const u32x4*, u32x4*, const PassTables, uint32_t, uint32_t);
};

#define BMMC_TILED(W, NT, IT) {W, NT, IT, 0, k_tiled<W, NT, IT, 0>}
#define BMMC_TILED_H(W, NT, IT)                                                      \
    {W, NT, IT, 0, k_tiled<W, NT, IT, 0>}, {W, NT, IT, 1, k_tiled<W, NT, IT, 1>},    \
        {W, NT, IT, 2, k_tiled<W, NT, IT, 2>}, {W, NT, IT, 3, k_tiled<W, NT, IT, 3>}
static const TiledEntry kTiled[] = {
    BMMC_TILED_H(4, 256, 4),  BMMC_TILED_H(4, 512, 4),  BMMC_TILED_H(4, 256, 8), BMMC_TILED_H(4, 512, 2),
    BMMC_TILED_H(4, 256, 2),  BMMC_TILED_H(4, 1024, 2), BMMC_TILED_H(4, 1024, 4), BMMC_TILED_H(4, 256, 16),
    BMMC_TILED_H(4, 512, 8),
    BMMC_TILED_H(8, 256, 4),  BMMC_TILED_H(8, 512, 4),  BMMC_TILED_H(8, 256, 8), BMMC_TILED_H(8, 512, 8),
    BMMC_TILED_H(8, 1024, 4), BMMC_TILED_H(8, 256, 16), BMMC_TILED_H(8, 256, 2), BMMC_TILED_H(8, 512, 2),
    BMMC_TILED_H(16, 256, 4), BMMC_TILED_H(16, 256, 8), BMMC_TILED_H(16, 512, 4), BMMC_TILED_H(16, 256, 2),
    BMMC_TILED_H(2, 256, 2),  BMMC_TILED_H(2, 256, 4),
    BMMC_TILED_H(1, 256, 1),  BMMC_TILED_H(1, 256, 4),
};
#undef BMMC_TILED
#undef BMMC_TILED_H

static const TiledEntry* find_tiled(int w, int nt, int iters, int hints) {
    for (const auto& e : kTiled)
        if (e.w == w && e.nt == nt && e.iters == iters && e.hints == hints) return &e;
    return nullptr;
}

bool tiled_kernel_available(int w, int nt, int iters, int hints) {
    return find_tiled(w, nt, iters, hints) != nullptr;
}

hipError_t launch_tiled(int w, int nt, int iters, int hints, const void* in, void* out,
                        const PassTables& tab, uint32_t ntiles, uint32_t grid, uint32_t xcds,
                        hipStream_t stream) {
    const TiledEntry* e = find_tiled(w, nt, iters, hints);
    if (!e) return hipErrorInvalidValue;
    if (grid == 0 || grid > ntiles) grid = ntiles;
    launch_k(e->fn, dim3(grid), dim3(nt), stream, (const u32x4*)in, (u32x4*)out, tab, ntiles, xcds);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Several columns of the sorting network per pass: between the read and the
// write phase each column compare-exchanges, in LDS, the pairs of slots
// (s, s XOR f) of the staged tile; a barrier separates the columns.  Pair k
// of a column is the slot s0 that has bit p = lowest set bit of f cleared,
// the other bits those of k, and its partner s0 XOR f.
// ---------------------------------------------------------------------------
template <int OP>
struct NetMid {
    const NetColumns& C;
    uint32_t* lds;
    uint32_t npairs;  // 2^(d-1)
    uint32_t tid, nt;
    template <typename PartsT>
    __device__ __forceinline__ void operator()(const PartsT& pt) const {
        for (uint32_t i = 0; i < C.count; i++) {
            const NetCol c = C.col[i];
            const uint32_t p = __builtin_ctz(c.f);
            const uint32_t lo = (1u << p) - 1u;
            const uint32_t alpha = __builtin_popcount(c.g & pt.r) & 1u;
            for (uint32_t k = tid; k < npairs; k += nt) {
                const uint32_t s0 = ((k & ~lo) << 1) | (k & lo);
                const uint32_t s1 = s0 ^ c.f;
                const uint32_t a = lds[s0], b = lds[s1];
                // bit 0 of s0's index in the column's space: 0 keeps the smaller
                const uint32_t hi0 = alpha ^ (__builtin_popcount(c.beta & s0) & 1u);
                const bool gt = OP == 1 ? (int32_t)a > (int32_t)b : a > b;
                if (gt != (hi0 != 0)) {
                    lds[s0] = b;
                    lds[s1] = a;
                }
            }
            __syncthreads();
        }
    }
};

// The columns of a register group (see NetGroup): thread registers j and
// j | 1 << K hold a pair; j keeps the smaller key when d0 XOR parity(q & j)
// is 0.  Register indices are compile-time constants.
template <int K, int OP>
__device__ __forceinline__ void net_cx(uint32_t (&reg)[32], uint32_t q, uint32_t d0) {
#pragma unroll
    for (int jl = 0; jl < 32; jl++) {
        if (jl & (1 << K)) continue;
        const int jh = jl | (1 << K);
        const uint32_t x = reg[jl], y = reg[jh];
        const uint32_t mn = OP == 1 ? (uint32_t)min((int32_t)x, (int32_t)y) : min(x, y);
        const uint32_t mx = OP == 1 ? (uint32_t)max((int32_t)x, (int32_t)y) : max(x, y);
        const bool dir = ((d0 ^ (uint32_t)__builtin_popcount(q & (uint32_t)jl)) & 1u) != 0;
        reg[jl] = dir ? mx : mn;
        reg[jh] = dir ? mn : mx;
    }
}

// Columns in register groups (2^13-slot tiles, 256 threads): per group, each
// thread loads its 32 slots, runs the group's columns in registers and
// stores them back; one barrier per group.
template <int OP>
struct NetMidRegs {
    const NetColumns& C;
    uint32_t* lds;
    uint32_t tid;
    template <typename PartsT>
    __device__ __forceinline__ void operator()(const PartsT& pt) const {
        for (uint32_t gi = 0; gi < C.ngroups; gi++) {
            const NetGroup& G = C.grp[gi];
            uint32_t base = 0;
#pragma unroll
            for (int b = 0; b < 8; b++) base |= ((tid >> b) & 1u) << ((G.cpos >> (4 * b)) & 15u);
            // slots in Gray-code order: one XOR per step, one address live
            uint32_t reg[32];
            {
                uint32_t sl = base;
                reg[0] = lds[sl];
#pragma unroll
                for (int i = 1; i < 32; i++) {
                    sl ^= G.S[__builtin_ctz(i)];
                    reg[i ^ (i >> 1)] = lds[sl];
                }
            }
            for (uint32_t i = G.first; i < G.last; i++) {
                const NetCol c = C.col[i];
                const uint32_t d0 =
                    ((uint32_t)__builtin_popcount(c.g & pt.r) ^ (uint32_t)__builtin_popcount(c.beta & base)) & 1u;
                const uint32_t q = c.rg >> 3;
                switch (c.rg & 7u) {
                    case 0: net_cx<0, OP>(reg, q, d0); break;
                    case 1: net_cx<1, OP>(reg, q, d0); break;
                    case 2: net_cx<2, OP>(reg, q, d0); break;
                    case 3: net_cx<3, OP>(reg, q, d0); break;
                    default: net_cx<4, OP>(reg, q, d0); break;
                }
            }
            {
                uint32_t sl = base;
                lds[sl] = reg[0];
#pragma unroll
                for (int i = 1; i < 32; i++) {
                    sl ^= G.S[__builtin_ctz(i)];
                    lds[sl] = reg[i ^ (i >> 1)];
                }
            }
            __syncthreads();
        }
    }
};

// REGS: the columns in register groups (the host plans them only for the
// full 2^13-slot tile of 256 threads); else each column through LDS.  Two
// kernels, because the register groups need many more VGPRs, and so fewer
// resident work-groups, than passes with few columns can afford.
template <int NT, int ITERS, int OP, bool REGS>
__global__ void __launch_bounds__(NT)
k_tiled_net(const u32x4* __restrict__ in, u32x4* __restrict__ out, const PassTables P, const NetColumns C,
            uint32_t ntiles, uint32_t xcds) {
    using Ctx = TileCtx<4, NT, ITERS, 0>;
    __shared__ typename Ctx::E lds[1 << Ctx::D];
    Ctx ctx;
    ctx.init(P, threadIdx.x);
    if constexpr (REGS) {
        static_assert(NT == 256 && Ctx::D == 13, "register groups are planned for 256 threads x 2^13 slots");
        const NetMidRegs<OP> mid{C, lds, threadIdx.x};
        ctx.run_tiles(P, (const g_u32x4*)in, (g_u32x4*)out, lds, logical_block(xcds), ntiles, gridDim.x,
                      threadIdx.x, mid);
    } else {
        const NetMid<OP> mid{C, lds, 1u << (P.d - 1), threadIdx.x, NT};
        ctx.run_tiles(P, (const g_u32x4*)in, (g_u32x4*)out, lds, logical_block(xcds), ntiles, gridDim.x,
                      threadIdx.x, mid);
    }
}

struct TiledNetEntry {
    int nt, iters, op;
    bool regs;
    void (*fn)(const u32x4*, u32x4*, const PassTables, const NetColumns, uint32_t, uint32_t);
};
static const TiledNetEntry kTiledNet[] = {
    {256, 8, 1, false, k_tiled_net<256, 8, 1, false>}, {256, 8, 2, false, k_tiled_net<256, 8, 2, false>},
    {256, 8, 1, true, k_tiled_net<256, 8, 1, true>},   {256, 8, 2, true, k_tiled_net<256, 8, 2, true>},
    {256, 4, 1, false, k_tiled_net<256, 4, 1, false>}, {256, 4, 2, false, k_tiled_net<256, 4, 2, false>},
};

bool tiled_net_available(int nt, int iters) {
    for (const auto& e : kTiledNet)
        if (e.nt == nt && e.iters == iters) return true;
    return false;
}

hipError_t launch_tiled_net(int nt, int iters, int op, bool regs, const void* in, void* out, const PassTables& tab,
                            const NetColumns& cols, uint32_t ntiles, uint32_t grid, hipStream_t stream) {
    if (tab.d < 1) return hipErrorInvalidValue;
    if (regs && (cols.ngroups == 0 || tab.d != 13)) return hipErrorInvalidValue;
    for (const auto& e : kTiledNet) {
        if (e.nt != nt || e.iters != iters || e.op != op || e.regs != regs) continue;
        if (grid == 0 || grid > ntiles) grid = ntiles;
        launch_k(e.fn, dim3(grid), dim3(nt), stream, (const u32x4*)in, (u32x4*)out, tab, cols, ntiles, 0u);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// One column of the sorting network at the keys' own positions, in place:
// lane k takes the pair whose positions in the column's index space are 2k
// and 2k + 1, i.e. Q.(2k) and Q.(2k) XOR Q.e_0 in the array (Q linear), and
// leaves the smaller key at the first.  The accesses follow Q, so in general
// they are not coalesced: this is the uncompiled form of the network.
// ---------------------------------------------------------------------------
template <int OP>
__global__ void __launch_bounds__(256)
k_cmp_direct(uint32_t* __restrict__ data, const DirectArgs P) {
    const uint32_t tid = threadIdx.x;
    const uint64_t k = (uint64_t)blockIdx.x * 256 + tid;
    if ((k >> (P.n - 1)) != 0) return;
    // bit j of k is bit j + 1 of the pair's first position 2k
    uint32_t p0 = 0;
#pragma unroll
    for (int j = 0; j < 8; j++)
        if ((tid >> j) & 1u) p0 ^= P.col[j + 1];
    const uint32_t b = blockIdx.x;
    for (int j = 0; j + 9 < kMaxTbBits; j++)
        if ((b >> j) & 1u) p0 ^= P.col[j + 9];
    const uint32_t p1 = p0 ^ P.col[0];
    const uint32_t a = data[p0], c = data[p1];
    const bool swap = OP == 1 ? (int32_t)a > (int32_t)c : a > c;
    data[p0] = swap ? c : a;
    data[p1] = swap ? a : c;
}

hipError_t launch_cmp_direct(void* data, const DirectArgs& args, int op, hipStream_t stream) {
    if (args.n < 1 || args.n > kMaxTbBits) return hipErrorInvalidValue;
    const uint64_t pairs = 1ull << (args.n - 1);
    const uint32_t grid = (uint32_t)((pairs + 255) / 256);
    if (op == 1)
        launch_k(k_cmp_direct<1>, dim3(grid), dim3(256), stream, (uint32_t*)data, args);
    else if (op == 2)
        launch_k(k_cmp_direct<2>, dim3(grid), dim3(256), stream, (uint32_t*)data, args);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Naive kernel (the paper's naive bit-reverse kernel in the Appendix,
// generalised to any A): each lane reads VEC consecutive elements with one
// load and writes each to A.x XOR c.  The output index is the XOR of a
// block-uniform part and a per-thread part (linearity of A).
// ---------------------------------------------------------------------------
template <int W, int VEC>
__global__ void __launch_bounds__(256)
k_naive(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, const NaiveArgs P) {
    using E = typename ElemT<W>::T;
    constexpr int LV = ilog2(VEC);
    const uint32_t tid = threadIdx.x;
    const uint64_t x0 = ((uint64_t)blockIdx.x * 256 + tid) << LV;
    if ((x0 >> P.n) != 0) return;
    const uint64_t base = (uint64_t)blockIdx.x << (LV + 8);
    uint32_t yb = P.c;
#pragma unroll
    for (int j = LV + 8; j < kMaxTbBits; j++)
        if ((base >> j) & 1u) yb ^= P.col[j];
    uint32_t yt = 0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if ((tid >> k) & 1u) yt ^= P.col[LV + k];
    E* o = reinterpret_cast<E*>(out);
    if constexpr (VEC * W == 16) {
        Vec16<W> v;
        v.v = reinterpret_cast<const u32x4*>(in)[x0 >> LV];
#pragma unroll
        for (int e = 0; e < VEC; e++) o[yb ^ yt ^ lin_const<0, LV>(P.col, e)] = v.e[e];
    } else {
        o[yb ^ yt] = reinterpret_cast<const E*>(in)[x0];
    }
}

hipError_t launch_naive(int w, int n, const void* in, void* out, const NaiveArgs& args,
                        hipStream_t stream) {
    const uint64_t size = 1ull << n;
    const int vec = 16 / w;
    const bool vector = size >= (uint64_t)vec * 256;
    const uint64_t lanes = vector ? size / vec : size;
    const uint32_t grid = (uint32_t)((lanes + 255) / 256);
    const uint8_t* i8 = (const uint8_t*)in;
    uint8_t* o8 = (uint8_t*)out;
#define BMMC_NAIVE(WW)                                                                            \
    case WW:                                                                                      \
        if (vector)                                                                               \
            launch_k(k_naive<WW, 16 / WW>, dim3(grid), dim3(256), stream, i8, o8, args);            \
        else                                                                                      \
            launch_k(k_naive<WW, 1>, dim3(grid), dim3(256), stream, i8, o8, args);                  \
        break;
    switch (w) {
        BMMC_NAIVE(1)
        BMMC_NAIVE(2)
        BMMC_NAIVE(4)
        BMMC_NAIVE(8)
        BMMC_NAIVE(16)
        default:
            return hipErrorInvalidValue;
    }
#undef BMMC_NAIVE
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Copy: VPT independent 16-byte vectors per lane (Section 2.3 "copy" bound).
// ---------------------------------------------------------------------------
template <int VPT, int HINT>
__global__ void __launch_bounds__(256)
k_copy(const u32x4* __restrict__ in, u32x4* __restrict__ out, uint64_t nvec) {
    const uint64_t first = (uint64_t)blockIdx.x * (256 * VPT);
    const uint64_t base = first + threadIdx.x;
    u32x4 v[VPT];
    if (first + 256 * VPT <= nvec) {
        // a whole chunk (every work-group but the last): no per-vector tests,
        // so the loads go out back to back instead of one at a time
#pragma unroll
        for (int k = 0; k < VPT; k++) v[k] = ld16<HINT>((const g_u32x4*)in + base + k * 256);
#pragma unroll
        for (int k = 0; k < VPT; k++) st16<HINT>((g_u32x4*)out + base + k * 256, v[k]);
        return;
    }
#pragma unroll
    for (int k = 0; k < VPT; k++)
        if (base + k * 256 < nvec) v[k] = ld16<HINT>((const g_u32x4*)in + base + k * 256);
#pragma unroll
    for (int k = 0; k < VPT; k++)
        if (base + k * 256 < nvec) st16<HINT>((g_u32x4*)out + base + k * 256, v[k]);
}

__global__ void k_copy_tail(const uint8_t* in, uint8_t* out, uint32_t count) {
    const uint32_t i = threadIdx.x;
    if (i < count) out[i] = in[i];
}

hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t stream, int vpt, int hints) {
    const uint64_t nvec = bytes / 16;
    const uint32_t tail = (uint32_t)(bytes % 16);
    if (nvec) {
        const uint64_t per = 256ull * (uint64_t)vpt;
        const dim3 grid((uint32_t)((nvec + per - 1) / per));
        const u32x4* i4 = (const u32x4*)in;
        u32x4* o4 = (u32x4*)out;
#define BMMC_COPY_H(V, H) launch_k(k_copy<V, H>, grid, dim3(256), stream, i4, o4, nvec)
#define BMMC_COPY(V)                            \
    case V:                                     \
        switch (hints) {                        \
            case 0: BMMC_COPY_H(V, 0); break;   \
            case 1: BMMC_COPY_H(V, 1); break;   \
            case 2: BMMC_COPY_H(V, 2); break;   \
            default: BMMC_COPY_H(V, 3); break;  \
        }                                       \
        break;
        switch (vpt) {
            BMMC_COPY(1)
            BMMC_COPY(2)
            BMMC_COPY(8)
            default:
            BMMC_COPY(4)
        }
#undef BMMC_COPY
#undef BMMC_COPY_H
    }
    if (tail)
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(16), 0, stream, (const uint8_t*)in + nvec * 16,
                           (uint8_t*)out + nvec * 16, tail);
    return hipGetLastError();
}

__global__ void k_zero(uint32_t* p, uint32_t count) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = 0;
}

hipError_t launch_zero(uint32_t* p, uint32_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((count + 255) / 256), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched persistent kernel.  Work items are ranges of tiles of one pass of
// one array, taken in queue order through an atomic head.  One launch runs
// one phase: the first passes of two-pass arrays together with the one-pass
// arrays, then a second launch (stream-ordered, in the same graph) runs the
// second passes, so every second pass reads a scratch array whose first pass
// has completed, without any wait or device-wide fence inside a kernel.
// Every width (4, 8 or 16 bytes; the host sends narrower elements through
// the single-array kernels) uses the same tile buffer of NT threads x ITERS
// vectors x 16 bytes (256 x 4, 256 x 8, 512 x 8 or 1024 x 8: 16, 32, 64 or
// 128 KiB).
// Thread 0 fetches the next item's index as soon as the current item
// starts, so the atomic's latency overlaps the current item's tiles.
// ---------------------------------------------------------------------------
template <int W, int HINT, int NT, int ITERS>
__device__ __forceinline__ void batch_tiles(const BatchPass& bp, uint32_t t0, uint32_t t1,
                                            uint8_t* lds_bytes, uint32_t tid) {
    using C = TileCtx<W, NT, ITERS, HINT>;
    C ctx;
    ctx.init(bp.tab, tid);
    ctx.run_tiles(bp.tab, (const g_u32x4*)bp.in, (g_u32x4*)bp.out, (typename C::E*)lds_bytes, t0, t1, 1, tid);
}

// range[phase] .. range[phase + 1] are this launch's items.
template <int HINT, int NT, int ITERS>
__global__ void __launch_bounds__(NT)
k_batched(const BatchPass* __restrict__ passes, const BatchItem* __restrict__ items,
          const uint32_t* __restrict__ range, uint32_t phase, uint32_t* head) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[NT * ITERS * 16];
    __shared__ uint32_t s_next;
    const uint32_t tid = threadIdx.x;
    const uint32_t first = range[phase], last = range[phase + 1];
    if (tid == 0) s_next = first + __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (;;) {
        const uint32_t idx = s_next;
        __syncthreads();  // every thread has read s_next before it is rewritten
        if (idx >= last) break;
        if (tid == 0) s_next = first + __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const BatchItem item = items[idx];
        const BatchPass& bp = passes[item.pass];
        switch (bp.w) {
            case 4: batch_tiles<4, HINT, NT, ITERS>(bp, item.tile_begin, item.tile_end, lds, tid); break;
            case 8: batch_tiles<8, HINT, NT, ITERS>(bp, item.tile_begin, item.tile_end, lds, tid); break;
            default: batch_tiles<16, HINT, NT, ITERS>(bp, item.tile_begin, item.tile_end, lds, tid); break;
        }
        __syncthreads();  // s_next written by thread 0 is visible to all
    }
}

hipError_t launch_batched(const BatchPass* passes, const BatchItem* items, const uint32_t* range,
                          uint32_t phase, uint32_t* head, uint32_t grid, int hints, int size, hipStream_t stream) {
#define BMMC_BATCHED(H, NT, I) \
    launch_k(k_batched<H, NT, I>, dim3(grid), dim3(NT), stream, passes, items, range, phase, head)
#define BMMC_BATCHED_H(NT, I)                  \
    switch (hints & 3) {                        \
        case 0: BMMC_BATCHED(0, NT, I); break; \
        case 1: BMMC_BATCHED(1, NT, I); break; \
        case 2: BMMC_BATCHED(2, NT, I); break; \
        default: BMMC_BATCHED(3, NT, I); break; \
    }
    if (size == 32) {
        BMMC_BATCHED_H(1024, 8)
    } else if (size == 16) {
        BMMC_BATCHED_H(512, 8)
    } else if (size == 8) {
        BMMC_BATCHED_H(256, 8)
    } else if (size == 4) {
        BMMC_BATCHED_H(256, 4)
    } else {
        return hipErrorInvalidValue;
    }
#undef BMMC_BATCHED_H
#undef BMMC_BATCHED
    return hipGetLastError();
}

int batched_occupancy(int size) {
    int blocks = 0;
    hipError_t e;
    if (size == 32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<0, 1024, 8>, 1024, 0);
    else if (size == 16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<0, 512, 8>, 512, 0);
    else if (size == 8)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<0, 256, 8>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<0, 256, 4>, 256, 0);
    if (e != hipSuccess) blocks = 4;
    return blocks > 0 ? blocks : 1;
}

int tiled_occupancy(int w, int nt, int iters, int hints) {
    const TiledEntry* e = find_tiled(w, nt, iters, hints);
    if (!e) return 1;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, e->fn, nt, 0) != hipSuccess) return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace bmmc
