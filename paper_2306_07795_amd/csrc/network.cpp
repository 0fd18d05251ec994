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
// and M_S ... M_0 = I.  On the device each M_s with its column is one tiled
// pass whose store compare-exchanges the pairs of every 16-byte vector; M_S is
// a plain pass.  The direct form runs the columns in place at the keys' own
// positions (pair k of column s at P_s^-1.(2k), P_s^-1.(2k + 1) with
// P_s = M_s ... M_0), without the permutations.
#include <cstring>
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
        LaunchScope ls(ds, stream, "k_copy", 2.0 * bytes);
        hipError_t e = launch_copy(in, out, bytes, stream, 4, 0, ls.events());
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
        hipError_t e = launch_cmp_direct(out, da, op, stream, ls.events());
        if (e != hipSuccess) return hip_fail(e, "direct column launch");
    }
    return BMMC_OK;
}

int run_passes(DeviceState* ds, const std::vector<BitMat>& st, const void* in, void* out, int n, int op,
               hipStream_t stream) {
    const size_t bytes = (size_t)4 << n;
    // one plan per stage (cached by matrix), before taking the device lock
    std::vector<std::shared_ptr<const Plan>> plans(st.size());
    PlanOptions po;
    po.method = kMethodAuto;
    for (size_t s = 0; s < st.size(); s++) {
        int rc = get_plan(ds, st[s].r, 0, n, 4, po, &plans[s]);
        if (rc != BMMC_OK) return rc;
        const Plan& p = *plans[s];
        if (p.naive || p.npass != 1) return set_error(BMMC_ERR_INTERNAL, "network stage %zu is not one pass", s);
        if (s + 1 < st.size() && !tiled_cmp_available(p.shape.nt, p.shape.iters))
            return set_error(BMMC_ERR_INTERNAL, "no compare-exchange pass for threads=%d iters=%d", p.shape.nt,
                             p.shape.iters);
    }
    std::lock_guard<std::mutex> lk(ds->mu);
    void* mid = nullptr;
    int rc = get_scratch(ds, stream, bytes, &mid);
    if (rc != BMMC_OK) return rc;
    // the last pass writes `out`; the ones before alternate with scratch
    const size_t last = st.size() - 1;
    const void* src = in;
    char name[64];
    for (size_t s = 0; s <= last; s++) {
        void* dst = ((last - s) % 2 == 0) ? out : mid;
        const Plan& p = *plans[s];
        if (s == last) {
            rc = enqueue_plan(ds, p, src, dst, stream, 0);
            if (rc != BMMC_OK) return rc;
        } else {
            const PassTables& tab = p.pass[0].tab;
            snprintf(name, sizeof(name), "k_tiled_cmp<%d,%d,%d>", p.shape.nt, p.shape.iters, op);
            LaunchScope ls(ds, stream, name, 2.0 * bytes);
            hipError_t e = launch_tiled_cmp(p.shape.nt, p.shape.iters, op, src, dst, tab, 1u << tab.ntb, 0, 0,
                                            stream, ls.events());
            if (e != hipSuccess) return hip_fail(e, "compare-exchange pass launch");
        }
        src = dst;
    }
    return BMMC_OK;
}

}  // namespace
}  // namespace bmmc

using namespace bmmc;

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
