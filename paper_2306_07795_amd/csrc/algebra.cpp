// Host BMMC algebra: composition and inverse (the fusion rule of Section
// 3), the parm matrices of Section 7.2, and fused sequences.
#include <cstring>

#include "runtime.hpp"

namespace bmmc {

namespace {

int load_matrix(const uint64_t* rows, int n, BitMat* out, const char* what) {
    if (n < 1 || n > 64) return set_error(BMMC_ERR_RANGE, "n = %d outside [1, 64]", n);
    if (!rows) return set_error(BMMC_ERR_ARG, "%s is NULL", what);
    out->n = n;
    for (int i = 0; i < n; i++) {
        if (rows[i] & ~low_mask(n)) return set_error(BMMC_ERR_ARG, "%s row %d has bits at positions >= n", what, i);
        out->r[i] = rows[i];
    }
    return BMMC_OK;
}

}  // namespace

// bmmc(A, c) after bmmc(B, d): x -> A.(B.x + d) + c = (AB).x + (A.d + c).
void compose(const BitMat& A, uint64_t c, const BitMat& B, uint64_t d, BitMat* out, uint64_t* out_c) {
    const uint64_t e = A.apply(d) ^ c;
    *out = mul(A, B);
    *out_c = e;
}

// Section 7.2: the element at x goes to y with the bit at lsb(mask) removed
// from x as the low n-1 bits, and the sub-array x.mask as the top bit.
BitMat parm_matrix(uint64_t mask, int n) {
    const int l = __builtin_ctzll(mask);
    BitMat A;
    A.n = n;
    for (int i = 0; i < n - 1; i++) A.r[i] = 1ull << (i < l ? i : i + 1);
    A.r[n - 1] = mask;
    return A;
}

}  // namespace bmmc

using namespace bmmc;

extern "C" int bmmc_compose(const uint64_t* A_rows, uint64_t c, const uint64_t* B_rows, uint64_t d, int n,
                            uint64_t* out_rows, uint64_t* out_c) {
    BitMat A, B;
    int st = load_matrix(A_rows, n, &A, "A_rows");
    if (st != BMMC_OK) return st;
    st = load_matrix(B_rows, n, &B, "B_rows");
    if (st != BMMC_OK) return st;
    if (!out_rows || !out_c) return set_error(BMMC_ERR_ARG, "outputs are NULL");
    if ((c | d) & ~low_mask(n)) return set_error(BMMC_ERR_ARG, "complement bits at positions >= n");
    BitMat M;
    uint64_t e;
    compose(A, c, B, d, &M, &e);
    for (int i = 0; i < n; i++) out_rows[i] = M.r[i];
    *out_c = e;
    return BMMC_OK;
}

extern "C" int bmmc_invert(const uint64_t* A_rows, uint64_t c, int n, uint64_t* out_rows, uint64_t* out_c) {
    BitMat A, Ai;
    int st = load_matrix(A_rows, n, &A, "A_rows");
    if (st != BMMC_OK) return st;
    if (!out_rows || !out_c) return set_error(BMMC_ERR_ARG, "outputs are NULL");
    if (c & ~low_mask(n)) return set_error(BMMC_ERR_ARG, "complement bits at positions >= n");
    if (!inverse(A, &Ai)) return set_error(BMMC_ERR_SINGULAR, "A is singular over F_2");
    const uint64_t ci = Ai.apply(c);
    for (int i = 0; i < n; i++) out_rows[i] = Ai.r[i];
    *out_c = ci;
    return BMMC_OK;
}

extern "C" int bmmc_parm_matrix(uint64_t mask, int n, uint64_t* rows_out, uint64_t* inv_rows_out) {
    if (n < 1 || n > 64) return set_error(BMMC_ERR_RANGE, "n = %d outside [1, 64]", n);
    if (mask == 0 || (mask & ~low_mask(n))) return set_error(BMMC_ERR_ARG, "mask must be nonzero and below 2^n");
    const BitMat A = parm_matrix(mask, n);
    BitMat Ai;
    if (!inverse(A, &Ai)) return set_error(BMMC_ERR_INTERNAL, "parm matrix not invertible");
    for (int i = 0; i < n; i++) {
        if (rows_out) rows_out[i] = A.r[i];
        if (inv_rows_out) inv_rows_out[i] = Ai.r[i];
    }
    return BMMC_OK;
}

extern "C" int bmmc_permute_seq(const void* in, void* out, int n, int count, const uint64_t* A_rows_seq,
                                const uint64_t* c_seq, int elem_bytes, void* stream) {
    if (count < 1 || !A_rows_seq || !c_seq) return set_error(BMMC_ERR_ARG, "empty or NULL sequence");
    if (n < 0 || n > BMMC_MAX_BITS) return set_error(BMMC_ERR_RANGE, "n = %d outside [0, %d]", n, BMMC_MAX_BITS);
    BitMat M = BitMat::identity(n);
    uint64_t e = 0;
    for (int k = 0; k < count; k++) {
        BitMat A;
        if (n > 0) {
            int st = load_matrix(A_rows_seq + (size_t)k * n, n, &A, "A_rows_seq");
            if (st != BMMC_OK) return st;
        } else {
            A.n = 0;
        }
        if (c_seq[k] & ~low_mask(n)) return set_error(BMMC_ERR_ARG, "complement %d has bits at positions >= n", k);
        BitMat next;
        uint64_t ne;
        compose(A, c_seq[k], M, e, &next, &ne);  // A_k after everything so far
        M = next;
        e = ne;
    }
    return bmmc_permute(in, out, n, M.r, e, elem_bytes, stream);
}
