// The sorting network of Section 7.1 (even/odd merge sort with a balanced
// periodic merger of V-shaped columns, all written with parm), compiled with
// the parm identity of Section 7.2: parm m f = bmmc(A^-1) . parm 2^(n-1) f .
// bmmc(A), A the parm matrix of m.
//
// Unfolding the recursion gives a sequence of BMMCs and compare-exchange
// columns.  A column always acts, in the index space it sees, on the adjacent
// pairs (2k, 2k + 1) (vcolumn 1 on two elements, lifted through parm
// 2^(n-1), which keeps the low index bits), smaller key first.  Adjacent BMMCs
// fuse by composition (Section 3), so the network is
//     M_0, C, M_1, C, ..., C, M_S      (S = n(n+1)/2 columns)
// and M_S ... M_0 = I.  On the device consecutive stages are grouped into
// tiled passes: a pass applies T = M_e ... M_s and runs the columns C_s .. C_e
// on each staged tile in LDS, which works as long as every column's pairs lie
// inside the tile -- the pass's tile subspace then contains the pair vectors
// P^-1.e_0 of all its columns (P the product of the pass's matrices up to the
// column) besides the low input bits and T^-1 of the low output bits that
// keep the reads and writes coalesced.  Stages are added to a pass greedily
// while that subspace fits the tile.  The direct form runs the columns in
// place at the keys' own positions (pair k of column s at Q.(2k),
// Q.(2k + 1) with Q = (M_s ... M_0)^-1), without the permutations.
#include <algorithm>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

namespace bmmc {

BitMat parm_matrix(uint64_t mask, int n);  // algebra.cpp

namespace {

struct NetOp {
    bool cmp;  // a compare-exchange column, else the BMMC M
    BitMat M;
};

// f applied to both halves (parm 2^(n-1) f): a BMMC of the n-1 low bits keeps
// the top bit; a column of adjacent pairs stays one.
NetOp lift(const NetOp& op, int n) {
    if (op.cmp) return op;
    NetOp r{false, BitMat::identity(n)};
    for (int i = 0; i < n - 1; i++) r.M.r[i] = op.M.r[i];
    return r;
}

void parm(uint64_t mask, int n, const std::vector<NetOp>& inner, std::vector<NetOp>* out) {
    const BitMat A = parm_matrix(mask, n);
    BitMat Ai;
    inverse(A, &Ai);
    out->push_back({false, A});
    for (const NetOp& op : inner) out->push_back(lift(op, n));
    out->push_back({false, Ai});
}

std::vector<NetOp> vcolumn(int n) {
    std::vector<NetOp> ops;
    if (n == 1) ops.push_back({true, BitMat::identity(1)});
    if (n >= 2) parm(3, n, vcolumn(n - 1), &ops);
    return ops;
}

std::vector<NetOp> merge(int n) {
    if (n == 0) return {};
    std::vector<NetOp> ops = vcolumn(n);
    parm(1ull << (n - 1), n, merge(n - 1), &ops);
    return ops;
}

std::vector<NetOp> sortnet(int n) {
    if (n == 0) return {};
    std::vector<NetOp> ops;
    parm(1, n, sortnet(n - 1), &ops);
    const std::vector<NetOp> m = merge(n);
    ops.insert(ops.end(), m.begin(), m.end());
    return ops;
}

// M_0 .. M_S, fused; empty on an internal inconsistency.
std::vector<BitMat> compile(int n) {
    std::vector<BitMat> stages;
    BitMat cur = BitMat::identity(n), total = BitMat::identity(n);
    for (const NetOp& op : sortnet(n)) {
        if (op.cmp) {
            stages.push_back(cur);
            cur = BitMat::identity(n);
        } else {
            cur = mul(op.M, cur);
            total = mul(op.M, total);
        }
    }
    stages.push_back(cur);
    for (int i = 0; i < n; i++)
        if (total.r[i] != (1ull << i)) return {};
    if ((int)stages.size() != n * (n + 1) / 2 + 1) return {};
    return stages;
}

std::mutex g_net_mu;
std::map<int, std::vector<BitMat>> g_nets;

const std::vector<BitMat>* stages_for(int n) {
    std::lock_guard<std::mutex> lk(g_net_mu);
    auto it = g_nets.find(n);
    if (it == g_nets.end()) {
        std::vector<BitMat> s = compile(n);
        if (s.empty()) return nullptr;
        it = g_nets.emplace(n, std::move(s)).first;
    }
    return &it->second;
}

int run_direct(DeviceState* ds, const std::vector<BitMat>& st, const void* in, void* out, int n, int op,
               hipStream_t stream) {
    const size_t bytes = (size_t)4 << n;
    std::lock_guard<std::mutex> lk(ds->mu);
    {
        LaunchScope ls(ds, stream, "k_copy<4,0>", 2.0 * bytes);
        hipError_t e = launch_copy(in, out, bytes, stream);
        if (e != hipSuccess) return hip_fail(e, "copy launch");
    }
    BitMat P = BitMat::identity(n);
    for (size_t s = 0; s + 1 < st.size(); s++) {
        P = mul(st[s], P);
        BitMat Q;
        if (!inverse(P, &Q)) return set_error(BMMC_ERR_INTERNAL, "network stage %zu singular", s);
        DirectArgs da;
        std::memset(&da, 0, sizeof(da));
        da.n = (uint32_t)n;
        for (int j = 0; j < n; j++) da.col[j] = (uint32_t)Q.col(j);
        LaunchScope ls(ds, stream, op == 1 ? "k_cmp_direct<1>" : "k_cmp_direct<2>", 2.0 * bytes);
        hipError_t e = launch_cmp_direct(out, da, op, stream);
        if (e != hipSuccess) return hip_fail(e, "direct column launch");
    }
    return BMMC_OK;
}

// Tile shape and run bits of the network's passes: 2^13-key tiles with
// reads and writes in runs of 2^6 keys (256 bytes), so that every pass holds
// at least one column (6 + 6 + 1 <= 13).
constexpr int kNetThreads = 256, kNetIters = 8, kNetRunIn = 6, kNetRunOut = 6;
// Fewest columns of a pass that runs them in register groups (measured on
// 2^16..2^26 keys): the register kernel holds fewer work-groups per CU, which
// costs a memory-bound pass more than it saves unless the pass has many
// columns; while the keys fit the caches, a few columns suffice.
uint32_t net_reg_min_cols(size_t bytes) { return bytes <= ((size_t)16 << 20) ? 4 : 16; }

struct NetPass {
    PassPlan plan;
    NetColumns cols;
};

KernelShape net_shape() {
    KernelShape ks = default_shape(4);
    ks.nt = kNetThreads;
    ks.iters = kNetIters;
    return ks;
}

// Does the tile subspace of a pass T holding the pair vectors `us` fit?
bool fits(const BitMat& T, const std::vector<uint64_t>& us, int D) {
    const int n = T.n;
    if (n <= D) return (int)us.size() <= kMaxNetCols;
    if ((int)us.size() > kMaxNetCols) return false;
    BitMat Ti;
    if (!inverse(T, &Ti)) return false;
    Basis b;
    for (int k = 0; k < kNetRunIn && k < n; k++) b.insert(1ull << k);
    for (int k = 0; k < kNetRunOut && k < n; k++) b.insert(Ti.col(k));
    for (uint64_t u : us) b.insert(u);
    return b.count <= D;
}

// Column i of a pass, in the slot space of its tile: f = F(coordinates of the
// pair vector u), beta = the direction functional g read through X and F^-1.
int column_tables(const PassTables& tab, uint64_t u, uint64_t g, NetCol* out) {
    Basis xb;
    for (uint32_t k = 0; k < tab.d; k++) xb.insert(tab.X[k]);
    const uint64_t cu = xb.coords(u);
    if (cu == ~0ull) return BMMC_ERR_INTERNAL;
    uint32_t f = 0;
    for (uint64_t m = cu; m; m &= m - 1) f ^= tab.F[__builtin_ctzll(m)];
    uint32_t beta = 0;
    for (uint32_t k = 0; k < tab.d; k++) {
        // coordinates v with F(v) = e_k (F has its top bit of column j at j)
        uint32_t t = 1u << k, v = 0;
        for (int j = (int)tab.d - 1; j >= 0; j--)
            if ((t >> j) & 1u) {
                v |= 1u << j;
                t ^= tab.F[j];
            }
        uint32_t x = 0;
        for (uint32_t m = v; m; m &= m - 1) x ^= tab.X[__builtin_ctz(m)];
        beta |= (uint32_t)(__builtin_popcountll(g & x) & 1) << k;
    }
    // the two slots of a pair sit on opposite sides of the column
    if (f == 0 || (__builtin_popcount(beta & f) & 1) != 1) return BMMC_ERR_INTERNAL;
    out->f = f;
    out->beta = beta;
    out->g = (uint32_t)g;
    return BMMC_OK;
}

// Register groups of a pass whose tile is a full 2^13 slots for 256 threads
// (32 slots a thread): consecutive columns whose pair vectors f are among at
// most kNetRegBits independent slot vectors form one group; its basis is
// completed with unit vectors (lowest bits first) to kNetRegBits, then to a
// basis of the slot space by 8 unit vectors for the thread bits.  Leaves
// ngroups = 0 (the LDS path) for smaller tiles or more than kMaxNetGroups.
void register_groups(uint32_t d, NetColumns* C) {
    C->ngroups = 0;
    if (d != 13 || C->count == 0) return;
    const int kThreadBits = 8;
    uint32_t ng = 0;
    for (uint32_t i = 0; i < C->count;) {
        if (ng == (uint32_t)kMaxNetGroups) {
            C->ngroups = 0;
            return;
        }
        NetGroup& G = C->grp[ng];
        Basis sb;
        int ns = 0;
        uint32_t j = i;
        for (; j < C->count; j++) {
            const uint32_t f = C->col[j].f;
            int k = 0;
            while (k < ns && G.S[k] != f) k++;
            if (k < ns) continue;  // already a basis vector
            if (ns == kNetRegBits || !sb.insert(f)) break;
            G.S[ns++] = f;
        }
        for (uint32_t b = 0; b < d && ns < kNetRegBits; b++)
            if (sb.insert(1u << b)) G.S[ns++] = 1u << b;
        G.cpos = 0;
        int nc = 0;
        for (uint32_t b = 0; b < d && nc < kThreadBits; b++)
            if (sb.insert(1u << b)) G.cpos |= b << (4 * nc++);
        if (ns != kNetRegBits || nc != kThreadBits) {  // cannot happen for d = 13
            C->ngroups = 0;
            return;
        }
        G.first = i;
        G.last = j;
        for (uint32_t c = i; c < j; c++) {
            NetCol& col = C->col[c];
            uint32_t idx = 0;
            while (G.S[idx] != col.f) idx++;
            uint32_t q = 0;
            for (int k = 0; k < kNetRegBits; k++) q |= (uint32_t)(__builtin_popcount(col.beta & G.S[k]) & 1) << k;
            col.rg = idx | (q << 3);
        }
        ng++;
        i = j;
    }
    C->ngroups = ng;
}

int build_net_pass(const BitMat& T, const std::vector<uint64_t>& us, const std::vector<uint64_t>& gs,
                   uint64_t seed, NetPass* np) {
    const KernelShape ks = net_shape();
    int st = build_pass(T, 0, kNetRunIn, kNetRunOut, ks, 1, seed, &np->plan, 0, 0, us.data(), (int)us.size());
    if (st != BMMC_OK) return st;
    std::memset(&np->cols, 0, sizeof(np->cols));
    np->cols.count = (uint32_t)us.size();
    for (size_t i = 0; i < us.size(); i++) {
        st = column_tables(np->plan.tab, us[i], gs[i], &np->cols.col[i]);
        if (st != BMMC_OK) return st;
    }
    register_groups(np->plan.tab.d, &np->cols);
    return BMMC_OK;
}

// Greedy grouping of M_0, C_0, ..., C_(S-1), M_S into passes.
int group_passes(const std::vector<BitMat>& st, int n, std::vector<NetPass>* out) {
    const int D = net_shape().D();
    const size_t S = st.size() - 1;
    size_t s = 0;
    uint64_t seed = 0x6E65747Full ^ (uint64_t)n;
    while (s < S) {
        BitMat T = st[s];
        BitMat Ti;
        inverse(T, &Ti);
        std::vector<uint64_t> us{Ti.col(0)}, gs{T.r[0]};
        size_t e = s;
        while (e + 1 < S) {  // the next matrix with its column
            const BitMat T2 = mul(st[e + 1], T);
            BitMat T2i;
            inverse(T2, &T2i);
            us.push_back(T2i.col(0));
            if (!fits(T2, us, D)) {
                us.pop_back();
                break;
            }
            gs.push_back(T2.r[0]);
            T = T2;
            e++;
        }
        if (e + 1 == S) {  // the final matrix, if it fits too
            const BitMat T2 = mul(st[S], T);
            if (fits(T2, us, D)) {
                T = T2;
                e = S;
            }
        }
        NetPass np;
        int rc = build_net_pass(T, us, gs, seed++, &np);
        if (rc != BMMC_OK) return rc;
        out->push_back(np);
        s = e + 1;
    }
    if (s == S) {  // the final matrix alone
        NetPass np;
        int rc = build_net_pass(st[S], {}, {}, seed++, &np);
        if (rc != BMMC_OK) return rc;
        out->push_back(np);
    }
    return BMMC_OK;
}

std::mutex g_pass_mu;
std::map<int, std::vector<NetPass>> g_passes;

int passes_for(int n, const std::vector<BitMat>& st, const std::vector<NetPass>** out) {
    std::lock_guard<std::mutex> lk(g_pass_mu);
    auto it = g_passes.find(n);
    if (it == g_passes.end()) {
        std::vector<NetPass> v;
        int rc = group_passes(st, n, &v);
        if (rc != BMMC_OK) return set_error(rc, "grouping the network of n = %d into passes failed", n);
        it = g_passes.emplace(n, std::move(v)).first;
    }
    *out = &it->second;
    return BMMC_OK;
}

int run_passes(DeviceState* ds, const std::vector<BitMat>& st, const void* in, void* out, int n, int op,
               hipStream_t stream) {
    const size_t bytes = (size_t)4 << n;
    const std::vector<NetPass>* passes = nullptr;
    int rc = passes_for(n, st, &passes);
    if (rc != BMMC_OK) return rc;
    std::lock_guard<std::mutex> lk(ds->mu);
    void* mid = nullptr;
    if (passes->size() > 1) {
        rc = get_scratch(ds, stream, bytes, &mid);
        if (rc != BMMC_OK) return rc;
    }
    // the last pass writes `out`; the ones before alternate with scratch
    const size_t last = passes->size() - 1;
    const void* src = in;
    char name[64];
    for (size_t k = 0; k <= last; k++) {
        void* dst = ((last - k) % 2 == 0) ? out : mid;
        const NetPass& np = (*passes)[k];
        const PassTables& tab = np.plan.tab;
        // register groups for passes with many columns; passes with few
        // keep the LDS kernel, whose lower register use leaves more
        // work-groups resident to hide the memory latency
        const bool regs = np.cols.ngroups > 0 && np.cols.count >= net_reg_min_cols(bytes);
        snprintf(name, sizeof(name), "k_tiled_net<%d,%d,%d,%d>", kNetThreads, kNetIters, op, regs ? 1 : 0);
        LaunchScope ls(ds, stream, name, 2.0 * bytes);
        hipError_t e =
            launch_tiled_net(kNetThreads, kNetIters, op, regs, src, dst, tab, np.cols, 1u << tab.ntb, 0, stream);
        if (e != hipSuccess) return hip_fail(e, "sorting-network pass launch");
        src = dst;
    }
    return BMMC_OK;
}

// Host emulation of one k_tiled_net pass with the same tables: tile by tile,
// the read phase by X and F, the columns by f, beta and g, the write phase by
// Y and G, each 16-byte vector addressed as the kernel addresses it (the
// vector index from the coordinates above the element bits).
int emulate_net_pass(const NetPass& np, int op, const uint32_t* src, uint32_t* dst) {
    const PassTables& P = np.plan.tab;
    const uint32_t d = P.d, slots = 1u << d;
    const uint32_t lv = d < 2 ? d : 2, em = (1u << lv) - 1u;  // 4-byte keys: 4 per vector
    std::vector<uint32_t> lds(slots);
    auto lin = [](const uint32_t* tab, uint32_t v) {
        uint32_t r = 0;
        for (; v; v &= v - 1) r ^= tab[__builtin_ctz(v)];
        return r;
    };
    for (uint32_t tile = 0; tile < (1u << P.ntb); tile++) {
        uint32_t r = 0, yb = P.c_hi, gx = P.c_lds;
        for (uint32_t j = 0; j < P.ntb; j++)
            if ((tile >> j) & 1u) {
                r ^= P.tb[j][0];
                yb ^= P.tb[j][1];
                gx ^= P.tb[j][2];
            }
        for (uint32_t v = 0; v < slots; v++) {
            const uint32_t x = r ^ lin(P.X, v & ~em);
            lds[lin(P.F, v)] = src[(x & ~em) | (v & em)];
        }
        if (np.cols.ngroups == 0) {
            for (uint32_t i = 0; i < np.cols.count; i++) {
                const NetCol& c = np.cols.col[i];
                const uint32_t p = __builtin_ctz(c.f), lo = (1u << p) - 1u;
                const uint32_t alpha = __builtin_popcount(c.g & r) & 1u;
                for (uint32_t k = 0; k < slots / 2; k++) {
                    const uint32_t s0 = ((k & ~lo) << 1) | (k & lo), s1 = s0 ^ c.f;
                    const uint32_t a = lds[s0], b = lds[s1];
                    const uint32_t hi0 = alpha ^ (__builtin_popcount(c.beta & s0) & 1u);
                    const bool gt = op == 1 ? (int32_t)a > (int32_t)b : a > b;
                    if (gt != (hi0 != 0)) {
                        lds[s0] = b;
                        lds[s1] = a;
                    }
                }
            }
        } else {
            // the register groups as the kernel runs them: each of the 256
            // threads loads its 32 slots, runs the group's columns on them,
            // stores them back
            for (uint32_t gi = 0; gi < np.cols.ngroups; gi++) {
                const NetGroup& G = np.cols.grp[gi];
                std::vector<uint32_t> next(lds);
                std::vector<int> seen(slots, 0);
                for (uint32_t t = 0; t < 256; t++) {
                    uint32_t base = 0;
                    for (int b = 0; b < 8; b++)
                        if ((t >> b) & 1u) base |= 1u << ((G.cpos >> (4 * b)) & 15u);
                    uint32_t slot[32], reg[32];
                    for (uint32_t j = 0; j < 32; j++) {
                        slot[j] = base;
                        for (int k = 0; k < kNetRegBits; k++)
                            if ((j >> k) & 1u) slot[j] ^= G.S[k];
                        reg[j] = lds[slot[j]];
                        seen[slot[j]]++;
                    }
                    for (uint32_t i = G.first; i < G.last; i++) {
                        const NetCol& c = np.cols.col[i];
                        const uint32_t idx = c.rg & 7u, q = c.rg >> 3;
                        const uint32_t d0 = (__builtin_popcount(c.g & r) ^ __builtin_popcount(c.beta & base)) & 1u;
                        for (uint32_t jl = 0; jl < 32; jl++) {
                            if ((jl >> idx) & 1u) continue;
                            const uint32_t jh = jl | (1u << idx);
                            const uint32_t x = reg[jl], y = reg[jh];
                            const bool lt = op == 1 ? (int32_t)x < (int32_t)y : x < y;
                            const uint32_t mn = lt ? x : y, mx = lt ? y : x;
                            const bool dir = (d0 ^ (__builtin_popcount(q & jl) & 1u)) != 0;
                            reg[jl] = dir ? mx : mn;
                            reg[jh] = dir ? mn : mx;
                        }
                    }
                    for (uint32_t j = 0; j < 32; j++) next[slot[j]] = reg[j];
                }
                for (uint32_t v = 0; v < slots; v++)
                    if (seen[v] != 1) return BMMC_ERR_INTERNAL;  // every slot in exactly one thread's registers
                lds.swap(next);
            }
        }
        for (uint32_t u = 0; u < slots; u++) {
            const uint32_t y = yb ^ lin(P.Y, u & ~em);
            dst[(y & ~em) | (u & em)] = lds[gx ^ lin(P.G, u)];
        }
    }
    return BMMC_OK;
}

}  // namespace
}  // namespace bmmc

using namespace bmmc;

extern "C" int bmmc_sortnet_passes(int n, int* passes_out, int* columns_out) {
    if (n < 2 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [2, %d]", n, BMMC_MAX_BITS);
    const std::vector<BitMat>* st = stages_for(n);
    if (!st) return set_error(BMMC_ERR_INTERNAL, "network compilation failed for n = %d", n);
    const std::vector<NetPass>* passes = nullptr;
    int rc = passes_for(n, *st, &passes);
    if (rc != BMMC_OK) return rc;
    if (passes_out) *passes_out = (int)passes->size();
    if (columns_out) {
        int most = 0;
        for (const NetPass& np : *passes) most = std::max(most, (int)np.cols.count);
        *columns_out = most;
    }
    return BMMC_OK;
}

extern "C" int bmmc_sortnet_emulate(const void* in, void* out, int n, int key_type, int* passes_out) {
    if (n < 2 || n > 24) return set_error(BMMC_ERR_RANGE, "emulation supports 2 <= n <= 24");
    if (!in || !out) return set_error(BMMC_ERR_ARG, "in/out must not be NULL");
    if (key_type != BMMC_KEY_I32 && key_type != BMMC_KEY_U32)
        return set_error(BMMC_ERR_ARG, "key_type = %d is not a bmmc_key_type", key_type);
    const std::vector<BitMat>* st = stages_for(n);
    if (!st) return set_error(BMMC_ERR_INTERNAL, "network compilation failed for n = %d", n);
    const std::vector<NetPass>* passes = nullptr;
    int rc = passes_for(n, *st, &passes);
    if (rc != BMMC_OK) return rc;
    const size_t count = (size_t)1 << n;
    std::vector<uint32_t> a((const uint32_t*)in, (const uint32_t*)in + count), b(count);
    for (const NetPass& np : *passes) {
        rc = emulate_net_pass(np, key_type == BMMC_KEY_I32 ? 1 : 2, a.data(), b.data());
        if (rc != BMMC_OK) return set_error(rc, "register groups of a pass do not cover its tile");
        a.swap(b);
    }
    std::memcpy(out, a.data(), count * 4);
    if (passes_out) *passes_out = (int)passes->size();
    return BMMC_OK;
}

extern "C" int bmmc_sortnet_stages(int n, uint64_t* rows_out, int max_matrices, int* count_out) {
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    const std::vector<BitMat>* st = stages_for(n);
    if (!st) return set_error(BMMC_ERR_INTERNAL, "network compilation failed for n = %d", n);
    if (count_out) *count_out = (int)st->size();
    if (!rows_out) return BMMC_OK;
    if (max_matrices < (int)st->size())
        return set_error(BMMC_ERR_RANGE, "%zu matrices do not fit %d", st->size(), max_matrices);
    for (size_t s = 0; s < st->size(); s++)
        for (int i = 0; i < n; i++) rows_out[s * n + i] = (*st)[s].r[i];
    return BMMC_OK;
}

extern "C" int bmmc_sortnet(const void* in, void* out, int n, int key_type, int method, void* stream) {
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    if (key_type != BMMC_KEY_I32 && key_type != BMMC_KEY_U32)
        return set_error(BMMC_ERR_ARG, "key_type = %d is not a bmmc_key_type", key_type);
    if (method != BMMC_SORTNET_PASSES && method != BMMC_SORTNET_DIRECT)
        return set_error(BMMC_ERR_ARG, "method = %d is not a bmmc_sortnet_method", method);
    const size_t bytes = (size_t)4 << n;
    int rc = validate_buffers(in, out, bytes);
    if (rc != BMMC_OK) return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    const std::vector<BitMat>* st = stages_for(n);
    if (!st) return set_error(BMMC_ERR_INTERNAL, "network compilation failed for n = %d", n);
    const int op = key_type == BMMC_KEY_I32 ? 1 : 2;
    hipStream_t s = (hipStream_t)stream;
    // fewer than one 16-byte vector of keys: the direct form
    if (method == BMMC_SORTNET_DIRECT || n < 2) {
        if (n == 0) {
            std::lock_guard<std::mutex> lk(ds->mu);
            hipError_t e = launch_copy(in, out, bytes, s);
            return e == hipSuccess ? BMMC_OK : hip_fail(e, "copy launch");
        }
        return run_direct(ds, *st, in, out, n, op, s);
    }
    return run_passes(ds, *st, in, out, n, op, s);
}
