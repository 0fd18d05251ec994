// Bit-packed linear algebra over F_2 for the host planner.
//
// An index x in [0, 2^n) is the vector of its bits, bit 0 least significant
// (paper, Section 3).  A matrix is stored as packed rows: r[i] holds row i,
// bit j of r[i] being the entry a_ij, so that output bit i of A.x is the parity
// of (r[i] AND x).
#pragma once
#include <cstdint>

namespace bmmc {

constexpr int kMaxBits = 64;

inline int parity64(uint64_t v) { return __builtin_parityll(v); }
inline int popcount64(uint64_t v) { return __builtin_popcountll(v); }
inline uint64_t low_mask(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1); }

struct BitMat {
    int n = 0;
    uint64_t r[kMaxBits] = {};

    static BitMat identity(int n) {
        BitMat m;
        m.n = n;
        for (int i = 0; i < n; i++) m.r[i] = 1ull << i;
        return m;
    }
    // Bit reversal: entry (i, j) is 1 exactly when i + j = n - 1 (Section 5.2).
    static BitMat reversal(int n) {
        BitMat m;
        m.n = n;
        for (int i = 0; i < n; i++) m.r[i] = 1ull << (n - 1 - i);
        return m;
    }
    // y = A.x (no complement).
    uint64_t apply(uint64_t x) const {
        uint64_t y = 0;
        for (int i = 0; i < n; i++) y |= (uint64_t)parity64(r[i] & x) << i;
        return y;
    }
    // Column j = A.e_j as a packed vector.
    uint64_t col(int j) const {
        uint64_t v = 0;
        for (int i = 0; i < n; i++) v |= ((r[i] >> j) & 1ull) << i;
        return v;
    }
    bool get(int i, int j) const { return (r[i] >> j) & 1ull; }
    void set(int i, int j, bool b) {
        if (b) r[i] |= 1ull << j; else r[i] &= ~(1ull << j);
    }
    bool operator==(const BitMat& o) const {
        if (n != o.n) return false;
        for (int i = 0; i < n; i++) if (r[i] != o.r[i]) return false;
        return true;
    }
};

// (A.B)_ij = sum_k a_ik b_kj: row i of AB is the XOR of the rows k of B with a_ik = 1.
inline BitMat mul(const BitMat& a, const BitMat& b) {
    BitMat m;
    m.n = a.n;
    for (int i = 0; i < a.n; i++) {
        uint64_t acc = 0, bits = a.r[i];
        while (bits) {
            int k = __builtin_ctzll(bits);
            bits &= bits - 1;
            acc ^= b.r[k];
        }
        m.r[i] = acc;
    }
    return m;
}

inline BitMat transpose(const BitMat& a) {
    BitMat t;
    t.n = a.n;
    for (int j = 0; j < a.n; j++) t.r[j] = a.col(j);
    return t;
}

// Rank by elimination on the packed rows.
inline int rank(const BitMat& a) {
    uint64_t rows[kMaxBits];
    for (int i = 0; i < a.n; i++) rows[i] = a.r[i];
    int rk = 0;
    for (int bit = 0; bit < a.n && rk < a.n; bit++) {
        int piv = -1;
        for (int i = rk; i < a.n; i++)
            if ((rows[i] >> bit) & 1ull) { piv = i; break; }
        if (piv < 0) continue;
        uint64_t p = rows[piv];
        rows[piv] = rows[rk];
        rows[rk] = p;
        for (int i = 0; i < a.n; i++)
            if (i != rk && ((rows[i] >> bit) & 1ull)) rows[i] ^= p;
        rk++;
    }
    return rk;
}

// Gauss-Jordan inverse; returns false when a is singular.
inline bool inverse(const BitMat& a, BitMat* out) {
    const int n = a.n;
    uint64_t m[kMaxBits], inv[kMaxBits];
    for (int i = 0; i < n; i++) { m[i] = a.r[i]; inv[i] = 1ull << i; }
    for (int c = 0; c < n; c++) {
        int piv = -1;
        for (int i = c; i < n; i++)
            if ((m[i] >> c) & 1ull) { piv = i; break; }
        if (piv < 0) return false;
        uint64_t t = m[piv]; m[piv] = m[c]; m[c] = t;
        t = inv[piv]; inv[piv] = inv[c]; inv[c] = t;
        for (int i = 0; i < n; i++)
            if (i != c && ((m[i] >> c) & 1ull)) { m[i] ^= m[c]; inv[i] ^= inv[c]; }
    }
    out->n = n;
    for (int i = 0; i < n; i++) out->r[i] = inv[i];
    return true;
}

// A set of independent vectors kept in echelon form keyed by leading (highest)
// bit, remembering for each stored vector which inserted vectors it combines.
// Used to test independence, to complete bases and to express a vector in
// the coordinates of a chosen basis.
struct Basis {
    int count = 0;                 // number of vectors inserted successfully
    uint64_t vec[kMaxBits] = {};   // vec[lead] = reduced vector with leading bit lead
    uint64_t comb[kMaxBits] = {};  // comb[lead] = bit k set if inserted vector k contributes
    uint64_t leads = 0;            // mask of leading bits in use

    // Reduce v against the stored vectors; returns the residue and, in *c,
    // the combination of inserted vectors that was subtracted.
    uint64_t reduce(uint64_t v, uint64_t* c = nullptr) const {
        // vec[b] has leading bit b, so clearing the highest shared leading
        // bit never re-sets a higher one: at most one step per leading bit.
        uint64_t cc = 0;
        for (uint64_t m = v & leads; m; m = v & leads) {
            const int top = 63 - __builtin_clzll(m);
            v ^= vec[top];
            cc ^= comb[top];
        }
        if (c) *c = cc;
        return v;
    }
    // Insert v as inserted vector number `count`; false if dependent.
    bool insert(uint64_t v) {
        uint64_t c;
        uint64_t res = reduce(v, &c);
        if (!res) return false;
        int top = 63 - __builtin_clzll(res);
        vec[top] = res;
        comb[top] = c ^ (1ull << count);
        leads |= 1ull << top;
        count++;
        return true;
    }
    bool contains(uint64_t v) const { return reduce(v) == 0; }
    // Coordinates of v (which must lie in the span) over the inserted vectors.
    uint64_t coords(uint64_t v) const {
        uint64_t c;
        uint64_t res = reduce(v, &c);
        return res ? ~0ull : c;
    }
};

}  // namespace bmmc
