// Host planner for BMMC permutations.
//
//  * tiled test (paper, Section 5.1);
//  * factorization A = (U.R)(R.L.P) into two tiled factors (Section 5.2),
//    applied as (R.L.P, 0) first and (U.R, c) second;
//  * per-pass tile geometry (Section 4.1 bit partition, Section 4.3 iteration
//    bits) expressed as XOR-linear address tables (see pass.hpp);
//  * the LDS layout: an XOR swizzle chosen so that each wave's LDS accesses hit
//    distinct banks on both sides of the tile (the aim of Section 4.2's row
//    shift, reached with a different layout for 64-lane waves).
#include "plan.hpp"

#include <cstring>
#include <initializer_list>

#include "bmmc.h"

namespace bmmc {

namespace {

inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Rank of a few vectors over F_2.
int small_rank(const uint64_t* v, int count) {
    uint64_t basis[64];
    uint64_t leads = 0;
    int r = 0;
    for (int i = 0; i < count; i++) {
        uint64_t x = v[i];
        for (uint64_t m = x & leads; m; m = x & leads) x ^= basis[63 - __builtin_clzll(m)];
        if (x) {
            const int top = 63 - __builtin_clzll(x);
            basis[top] = x;
            leads |= 1ull << top;
            r++;
        }
    }
    return r;
}

// Rank deficit of the lanes of one wave against one bank model.
// `vecs[i]` is the LDS slot offset driven by lane bit i.  With nb banks of
// 4 bytes and w-byte elements, nb*4/w lanes are serviced together, and they
// are conflict-free when their slot indices differ in the low
// log2(nb*4/w) bits.
int lane_deficit(const uint32_t* vecs, int active, int w, int nb) {
    if (w < 4) return 0;
    int gl = nb * 4 / w;
    if (gl > 64) gl = 64;
    int lb = __builtin_ctz(gl);
    if (active < lb) lb = active < 0 ? 0 : active;
    uint64_t v[8];
    for (int i = 0; i < lb; i++) v[i] = vecs[i] & low_mask(lb);
    return lb - small_rank(v, lb);
}

int side_deficit(const uint32_t* map, int d, int lv, int w, int nb) {
    uint32_t v[8] = {};
    for (int i = 0; i < 6 && lv + i < d; i++) v[i] = map[lv + i];
    return lane_deficit(v, d - lv, w, nb);
}

}  // namespace

int lds_conflict_score(const PassTables& tab, const KernelShape& ks) {
    int s = 0;
    const int d = (int)tab.d;
    for (int nb : {32, 64}) {
        s += side_deficit(tab.F, d, ks.lv(), ks.w, nb);
        s += side_deficit(tab.G, d, ks.lv(), ks.w, nb);
    }
    return s;
}

uint64_t tiled_row_mask(const BitMat& A, int t) {
    // bit j of `below` is set when some entry a_ij with i >= t is 1
    uint64_t below = 0;
    for (int i = t; i < A.n; i++) below |= A.r[i];
    return ~below & low_mask(A.n);
}

bool factorize_ulp(const BitMat& A, BitMat* U, BitMat* L, BitMat* P, BitMat* T1, BitMat* T2) {
    const int n = A.n;
    // Upward elimination, bottom row first: pick in row i a column q_i not
    // used yet (the highest such column), then clear that column in every
    // row above.  E records the row operations, which only add a row into a
    // row above it, so E is upper unitriangular and M = E.A.
    BitMat M = A, E = BitMat::identity(n);
    uint64_t used = 0;
    int q[kMaxBits];
    for (int i = n - 1; i >= 0; i--) {
        uint64_t cand = M.r[i] & ~used & low_mask(n);
        if (!cand) return false;  // singular
        int qi = 63 - __builtin_clzll(cand);
        q[i] = qi;
        used |= 1ull << qi;
        for (int k = 0; k < i; k++)
            if ((M.r[k] >> qi) & 1ull) {
                M.r[k] ^= M.r[i];
                E.r[k] ^= E.r[i];
            }
    }
    // Column q_i of M is 1 at row i and 0 above it.  With P.e_{q_i} = e_i and
    // L.e_i = M.e_{q_i}, L is lower unitriangular and M = L.P.
    BitMat Pm, Lm;
    Pm.n = Lm.n = n;
    for (int i = 0; i < n; i++) Pm.r[i] = 1ull << q[i];
    for (int row = 0; row < n; row++) {
        uint64_t v = 0;
        for (int i = 0; i < n; i++) v |= ((M.r[row] >> q[i]) & 1ull) << i;
        Lm.r[row] = v;
    }
    BitMat Um;
    if (!inverse(E, &Um)) return false;
    const BitMat R = BitMat::reversal(n);
    BitMat t1 = mul(Um, R);
    BitMat t2 = mul(R, mul(Lm, Pm));
    if (!(mul(t1, t2) == A)) return false;
    if (U) *U = Um;
    if (L) *L = Lm;
    if (P) *P = Pm;
    if (T1) *T1 = t1;
    if (T2) *T2 = t2;
    return true;
}

KernelShape default_shape(int w) {
    KernelShape k;
    k.w = w;
    k.nt = 256;
    k.vec = 16 / w;
    switch (w) {
        case 1: k.iters = 4; break;   // D = 14: runs of 2^7 bytes
        case 2: k.iters = 2; break;   // D = 12
        case 4: k.iters = 4; break;   // D = 12, 16 KiB tile
        case 8: k.iters = 8; break;   // D = 12, 32 KiB tile
        default: k.iters = 8; break;  // w = 16: D = 11, 32 KiB tile
    }
    return k;
}

int default_t(const KernelShape& ks) { return ks.D() / 2; }

KernelShape general_shape(int w) {
    KernelShape k = default_shape(w);
    if (w == 4) k.iters = 8;  // D = 13
    return k;
}

void general_runs(const KernelShape& ks, int* a, int* b) {
    const int D = ks.D();
    // measured on 2^26..2^28-element random matrices: the longer run on the
    // write side for 4-byte elements, on the read side for 8-byte elements
    if (ks.w == 8 && D == 12) {
        *a = 7;
        *b = 5;
        return;
    }
    *b = (D + 1) / 2;
    *a = D - *b;
}

int build_pass(const BitMat& T, uint64_t c, int a, int b, const KernelShape& ks, int swizzle,
               uint64_t seed, PassPlan* p, int tb_mix, int iter_mix, const uint64_t* extra, int nextra) {
    const int n = T.n;
    const int D = ks.D();
    BitMat Ti;
    if (!inverse(T, &Ti)) return BMMC_ERR_SINGULAR;
    *p = PassPlan();
    p->T = T;
    p->c = c;

    uint64_t X[kMaxBits] = {}, Y[kMaxBits] = {}, G0[kMaxBits] = {};
    int d = 0;
    // The three index bits above a 4 KiB block of elements.
    int blk = 12;
    for (int wb = ks.w; wb > 1; wb >>= 1) blk--;
    const uint64_t block_bits = 7ull << blk;
    bool dealt = ((tb_mix >> 8) & 1) && n > D && blk + 3 <= n;
    Basis vb;  // read-coordinate basis, inserted in coordinate order
    if (n <= D) {
        // Whole array in one tile: any matrix, read and write fully contiguous.
        a = b = n;
        for (int k = 0; k < n; k++) {
            X[d++] = 1ull << k;
            vb.insert(1ull << k);
        }
        p->coordinate = true;
        p->dim_v0 = n;
    } else {
        if (a > n) a = n;
        if (b > n) b = n;
        for (int k = 0; k < a; k++) {
            X[d++] = 1ull << k;
            vb.insert(1ull << k);
        }
        // Inputs whose images are the low b outputs: T^-1 e_k, k < b, taken
        // modulo the low a bits already in the tile.
        Basis hb;
        uint64_t hs[kMaxBits];
        int nh = 0;
        uint64_t J = 0;
        for (int k = 0; k < b; k++) {
            uint64_t h = Ti.col(k) & ~low_mask(a);
            J |= h;
            if (hb.insert(h)) hs[nh++] = h;
        }
        if (popcount64(J) == hb.count) {
            // Coordinate tile (a tiled BMMC): the extra tile bits are the
            // tile row bits outside the column bits, in ascending order.
            p->coordinate = true;
            for (int j = 0; j < n; j++)
                if ((J >> j) & 1ull) {
                    X[d++] = 1ull << j;
                    vb.insert(1ull << j);
                }
        } else {
            p->coordinate = false;
            for (int i = 0; i < nh; i++) {
                X[d++] = hs[i];
                vb.insert(hs[i]);
            }
        }
        // Vectors the caller needs inside every tile, taken modulo the low a
        // input bits (already in the tile): a coordinate's input offset must
        // keep the element bits of a 16-byte vector clear.
        for (int i = 0; i < nextra; i++) {
            const uint64_t v = extra[i] & low_mask(n) & ~low_mask(a);
            if (!v || !vb.insert(v)) continue;
            X[d++] = v;
            if (popcount64(v) != 1) p->coordinate = false;
        }
        p->dim_v0 = d;
        if (d > D) return BMMC_ERR_RANGE;
        // Dealt output blocks (see the tile-selecting vectors below) need a
        // tile none of whose vectors moves the output's block bits.
        for (int k = 0; k < d && dealt; k++) dealt = (T.apply(X[k]) & block_bits) == 0;
        // Iteration bits: the lowest remaining index bits fill the tile.
        // With iter_mix each is XOR-ed with a random choice of the remaining
        // higher index bits, so one tile's rows spread over the address space.
        // With dealt output blocks, only bits whose images keep the block.
        uint64_t s = seed ^ 0x17E7ull;
        for (int j = a; j < n && d < D; j++) {
            if (dealt && (T.apply(1ull << j) & block_bits)) continue;
            if (!vb.contains(1ull << j)) {
                uint64_t v = 1ull << j;
                if (iter_mix && !dealt) {
                    s = mix64(s);
                    for (int k = j + 1; k < n; k++)
                        if (((s >> (k & 63)) & 1ull) && !vb.contains(1ull << k)) v ^= 1ull << k;
                }
                if (!vb.insert(v)) continue;
                X[d++] = v;
                p->iter_mask |= v;
            }
        }
    }
    p->a = a;
    p->b = b;
    p->d = d;
    p->col_mask = low_mask(a);
    p->row_mask = tiled_row_mask(T, b);
    p->n_over = popcount64(p->row_mask & p->col_mask);

    // Tile-selecting bits: positions that are not leading bits of the tile
    // basis; with them the tile basis completes to a basis of the index space.
    uint32_t tbpos[kMaxBits];
    int ntb = 0;
    for (int j = 0; j < n; j++)
        if (!((vb.leads >> j) & 1ull)) tbpos[ntb++] = j;
    if (ntb != n - d) return BMMC_ERR_INTERNAL;
    for (int i = 0; i < ntb; i++) p->tb_mask |= 1ull << tbpos[i];

    // Write coordinates: the low b output bits, then images of the read
    // coordinates taken modulo the low b output bits.
    Basis yb;
    int m = 0;
    for (int k = 0; k < b; k++) {
        Y[m++] = 1ull << k;
        yb.insert(1ull << k);
    }
    for (int k = 0; k < d && m < d; k++) {
        uint64_t q = T.apply(X[k]) & ~low_mask(b);
        if (q && yb.insert(q)) Y[m++] = q;
    }
    if (m != d) return BMMC_ERR_INTERNAL;
    // G0[k]: read coordinates of the element with write coordinate e_k.
    for (int k = 0; k < d; k++) {
        uint64_t cc = vb.coords(Ti.apply(Y[k]));
        if (cc == ~0ull) return BMMC_ERR_INTERNAL;
        G0[k] = cc;
    }

    // The kernels move 16-byte vectors: beyond the vector's own element
    // bits, no read or write coordinate may touch them.
    for (int k = ks.lv(); k < d; k++)
        if ((X[k] | Y[k]) & low_mask(ks.lv())) return BMMC_ERR_INTERNAL;

    PassTables& tab = p->tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.n = (uint32_t)n;
    tab.d = (uint32_t)d;
    tab.ntb = (uint32_t)ntb;
    for (int k = 0; k < d; k++) {
        tab.X[k] = (uint32_t)X[k];
        tab.Y[k] = (uint32_t)Y[k];
    }

    // LDS layout F: unitriangular XOR map on slot indices (F(e_k) = e_k plus
    // lower bits), so it is always invertible.  Start from the plain layout
    // and search deterministic random candidates until the lanes of every
    // wave access hit distinct banks in both bank models, keeping the best
    // seen.  Only the columns that a wave's lane bits reach are varied:
    // slot bits lv..lv+5 on the read side and the read coordinates of write
    // slot bits lv..lv+5 on the write side.
    const int lv = ks.lv();
    const int nl = (d - lv) < 6 ? (d - lv) : 6;  // lane bits that reach the tile
    uint32_t Fbest[kMaxTileBits], Fc[kMaxTileBits];
    for (int k = 0; k < d; k++) Fbest[k] = 1u << k;
    uint64_t relevant = 0;
    for (int i = 0; i < nl; i++) relevant |= (1ull << (lv + i)) | G0[lv + i];
    auto score_of = [&](const uint32_t* Fm) {
        uint32_t rv[6] = {}, wv[6] = {};
        for (int i = 0; i < nl; i++) {
            rv[i] = Fm[lv + i];
            uint32_t g = 0;
            for (uint64_t m = G0[lv + i]; m; m &= m - 1) g ^= Fm[__builtin_ctzll(m)];
            wv[i] = g;
        }
        int sc = 0;
        for (int nb : {32, 64}) sc += lane_deficit(rv, nl, ks.w, nb) + lane_deficit(wv, nl, ks.w, nb);
        return sc;
    };
    int best = score_of(Fbest);
    if (swizzle && best > 0) {
        uint64_t s = seed ^ 0x5EEDull;
        std::memcpy(Fc, Fbest, sizeof(uint32_t) * d);
        for (int attempt = 0; attempt < 2048 && best > 0; attempt++) {
            for (uint64_t m = relevant; m; m &= m - 1) {
                const int k = __builtin_ctzll(m);
                s = mix64(s);
                const int lo = k < 6 ? k : 6;
                Fc[k] = (1u << k) ^ (uint32_t)(s & low_mask(lo));
            }
            const int sc = score_of(Fc);
            if (sc < best) {
                best = sc;
                std::memcpy(Fbest, Fc, sizeof(uint32_t) * d);
            }
        }
    }
    for (int k = 0; k < d; k++) {
        tab.F[k] = Fbest[k];
        uint32_t g = 0;
        for (uint64_t m = G0[k]; m; m &= m - 1) g ^= Fbest[__builtin_ctzll(m)];
        tab.G[k] = g;
    }
    p->lds_score = lds_conflict_score(tab, ks);

    auto gmap = [&](uint64_t lowbits) {
        uint32_t g = 0;
        for (int k = 0; k < b; k++)
            if ((lowbits >> k) & 1ull) g ^= tab.G[k];
        return g;
    };
    // Tile-selecting vectors: the complement's index bits, or (tb_mix) each
    // XOR-ed with a random choice of the higher ones -- an invertible change
    // of basis of the same complement, which changes which tiles run
    // together but not what any tile holds.
    // With out_adj = k > 0 (tb_mix >> 4), the first k tile-selecting vectors
    // are instead the inputs T^-1 e_j of output bits j = b, b+1, ... reduced
    // modulo the tile, so tiles of neighbouring index write neighbouring runs
    // of the output (k = 15: as many as there are).
    // With bit 8 of tb_mix (dealt output blocks), when the tile allows it,
    // the first three tile-selecting vectors are the inputs T^-1 e_j of the
    // output block bits j (the three above a 4 KiB block) and every other one
    // is made to keep those bits, so tile t writes only the blocks whose
    // index is t mod 8 (XOR a constant from c).  Work-groups are dealt to the
    // eight XCDs in turn, so in the plain tile order each XCD then writes one
    // eighth of the output's 4 KiB blocks.  Beyond the last-level cache that
    // is faster for some matrices and slower for others (whose reads then
    // follow the XCDs through coarse address bits), so it is an option that
    // the per-matrix tuner tries, not a default.
    const int out_adj = (tb_mix >> 4) & 15;
    uint64_t tbv[kMaxBits];
    for (int i = 0; i < ntb; i++) tbv[i] = 1ull << tbpos[i];
    if (dealt && ntb >= 3) {
        Basis cb = vb;
        uint64_t u[3];
        int nt = 0;
        for (int i = 0; i < 3; i++) {
            u[i] = vb.reduce(Ti.col(blk + i));
            if (!u[i] || !cb.insert(u[i])) return BMMC_ERR_INTERNAL;
            tbv[nt++] = u[i];
        }
        for (int k = 0; k < ntb && nt < ntb; k++) {
            uint64_t v = 1ull << tbpos[k];
            const uint64_t sig = (T.apply(v) >> blk) & 7ull;
            for (int i = 0; i < 3; i++)
                if ((sig >> i) & 1ull) v ^= u[i];
            v = vb.reduce(v);
            if (v && cb.insert(v)) tbv[nt++] = v;
        }
        if (nt != ntb) return BMMC_ERR_INTERNAL;
    } else if (out_adj) {
        Basis cb = vb;
        int nt = 0;
        const int want = out_adj == 15 ? ntb : (out_adj < ntb ? out_adj : ntb);
        for (int j = b; j < n && nt < want; j++) {
            const uint64_t u = vb.reduce(Ti.col(j));
            if (u && cb.insert(u)) tbv[nt++] = u;
        }
        for (int i = 0; i < ntb && nt < ntb; i++)
            if (cb.insert(1ull << tbpos[i])) tbv[nt++] = 1ull << tbpos[i];
        if (nt != ntb) return BMMC_ERR_INTERNAL;
    } else if (tb_mix & 1) {
        uint64_t s = seed ^ 0x7B1Dull;
        for (int i = 0; i < ntb; i++) {
            s = mix64(s);
            for (int j = i + 1; j < ntb; j++)
                if ((s >> (j & 63)) & 1ull) tbv[i] ^= 1ull << tbpos[j];
        }
    }
    for (int i = 0; i < ntb; i++) {
        uint64_t col = T.apply(tbv[i]);
        tab.tb[i][0] = (uint32_t)tbv[i];
        tab.tb[i][1] = (uint32_t)(col & ~low_mask(b));
        tab.tb[i][2] = gmap(col & low_mask(b));
    }
    tab.c_hi = (uint32_t)(c & ~low_mask(b));
    tab.c_lds = gmap(c & low_mask(b));
    return BMMC_OK;
}

int make_plan(const uint64_t* rows, uint64_t c, int n, int w, const PlanOptions& opt, Plan* p) {
    if (n < 0 || n > BMMC_MAX_BITS) return BMMC_ERR_RANGE;
    if (!(w == 1 || w == 2 || w == 4 || w == 8 || w == 16)) return BMMC_ERR_ARG;
    if (n > 0 && rows == nullptr) return BMMC_ERR_ARG;
    if (c & ~low_mask(n)) return BMMC_ERR_ARG;
    BitMat A;
    A.n = n;
    for (int i = 0; i < n; i++) {
        if (rows[i] & ~low_mask(n)) return BMMC_ERR_ARG;
        A.r[i] = rows[i];
    }
    if (rank(A) != n) return BMMC_ERR_SINGULAR;

    *p = Plan();
    p->n = n;
    p->w = w;
    p->A = A;
    p->c = c;
    p->method = opt.method;
    p->shape = opt.shape_given ? opt.shape : default_shape(w);
    if (p->shape.w != w) return BMMC_ERR_ARG;
    const KernelShape& ks = p->shape;
    if (n == 0) return BMMC_OK;  // one element: plain copy
    if (opt.method == kMethodNaive || n < ks.lv()) {
        p->naive = true;
        p->npass = 1;
        return BMMC_OK;
    }
    const int D = ks.D();
    int t = opt.t > 0 ? opt.t : default_t(ks);
    const int a = opt.a > 0 ? opt.a : t;  // read runs of 2^a elements
    const int b = opt.b > 0 ? opt.b : t;  // write runs of 2^b elements
    if (a < ks.lv() || b < ks.lv() || a > D || b > D) return BMMC_ERR_RANGE;
    p->t = t;
    uint64_t seed = 0x243F6A8885A308D3ull ^ ((uint64_t)n << 32) ^ (uint64_t)w;
    int st;
    if (opt.method != kMethodOnePass && (n <= D || is_tiled(A, b))) {
        // One tiled pass: the whole array fits a tile, or A is tiled (its
        // inputs that reach the low b output bits are index bits).  Tiles of
        // a tiled matrix larger than a tile have their rows at power-of-two
        // strides; by default, mixing which tiles run together spreads the
        // concurrent accesses.
        const int mix = opt.tb_mix >= 0 ? opt.tb_mix : (n > D ? 1 : 0);
        st = build_pass(A, c, a, b, ks, opt.swizzle, seed, &p->pass[0], mix, opt.iter_mix);
        if (st != BMMC_OK) return st;
        p->npass = 1;
        return BMMC_OK;
    }
    if (opt.method == kMethodOnePass || opt.method == kMethodAuto) {
        // One pass with a general tile: the span of the low a input bits and
        // of the inputs that reach the low b output bits.  With a + b <= D it
        // fits one tile for every A.
        if (!opt.shape_given) p->shape = general_shape(w);
        const KernelShape& gs = p->shape;
        int ga = a, gb = b;
        if (opt.t <= 0 && opt.a <= 0 && opt.b <= 0) general_runs(gs, &ga, &gb);
        if (ga < gs.lv() || gb < gs.lv() || ga > gs.D() || gb > gs.D()) return BMMC_ERR_RANGE;
        st = build_pass(A, c, ga, gb, gs, opt.swizzle, seed, &p->pass[0], opt.tb_mix > 0 ? opt.tb_mix : 0,
                        opt.iter_mix);
        if (st != BMMC_OK) return st;
        p->npass = 1;
        return BMMC_OK;
    }
    BitMat T1, T2;
    if (!factorize_ulp(A, nullptr, nullptr, nullptr, &T1, &T2)) return BMMC_ERR_SINGULAR;
    st = build_pass(T2, 0, a, b, ks, opt.swizzle, seed, &p->pass[0], opt.tb_mix > 0 ? opt.tb_mix : 0, opt.iter_mix);
    if (st != BMMC_OK) return st;
    st = build_pass(T1, c, a, b, ks, opt.swizzle, seed + 1, &p->pass[1], opt.tb_mix > 0 ? opt.tb_mix : 0, opt.iter_mix);
    if (st != BMMC_OK) return st;
    p->npass = 2;
    return BMMC_OK;
}

}  // namespace bmmc
