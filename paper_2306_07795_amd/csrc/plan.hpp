// Host planner: tiled test, factorization into tiled factors, per-pass tile
// geometry and the LDS layout.  Pure host code (no HIP calls).
#pragma once
#include <cstdint>

#include "f2.hpp"
#include "pass.hpp"

namespace bmmc {

enum Method : int {
    kMethodAuto = 0,     // one tiled pass if A is tiled, else one pass with a general tile
    kMethodTiled = 1,    // the paper's scheme: one tiled pass if A is tiled, else two
    kMethodOnePass = 2,  // one pass with a general (non-coordinate) tile
    kMethodNaive = 3,    // one element per lane, scattered writes
};

// Compile-time shape of a tiled-pass kernel instance: work-group size NT,
// elements per 16-byte vector VEC, vectors per thread ITERS.  The tile holds
// NT*VEC*ITERS = 2^D elements.
struct KernelShape {
    int w = 4;
    int nt = 256;
    int vec = 4;
    int iters = 4;
    int lt() const { return __builtin_ctz(nt); }
    int lv() const { return __builtin_ctz(vec); }
    int li() const { return __builtin_ctz(iters); }
    int D() const { return lt() + lv() + li(); }
};

struct PassPlan {
    BitMat T;
    uint64_t c = 0;
    int a = 0, b = 0;       // read-run and write-run bits
    int d = 0;              // tile bits actually used
    int dim_v0 = 0;         // dimension of the tile before iteration bits
    bool coordinate = false;// tile spanned by unit vectors (paper's tiles)
    uint64_t col_mask = 0;  // low a input bits
    uint64_t row_mask = 0;  // tile row bits S (coordinate tiles)
    uint64_t iter_mask = 0; // iteration bits added to fill the tile
    uint64_t tb_mask = 0;   // tile-selecting bits (coordinate complement)
    int n_over = 0;         // |col bits AND row bits|
    int lds_score = 0;      // bank-conflict residue of the chosen LDS layout
    PassTables tab{};
};

struct PlanOptions {
    int method = kMethodAuto;
    int t = 0;        // run bits; 0 = default for the shape
    int a = 0;        // read-run bits; 0 = t
    int b = 0;        // write-run bits; 0 = t
    int swizzle = 1;  // 0: plain layout, 1: conflict-avoiding XOR layout
    // bit 0: tile-selecting vectors are XOR combinations of index bits;
    // bits 4-7: how many of them step the output (neighbouring tiles write
    // neighbouring runs; 15 = all); bit 8: the first three step the output's
    // 4 KiB-block bits and no other tile vector moves them, where the tile
    // allows it (dealt output blocks); -1: auto
    int tb_mix = -1;
    int iter_mix = 0; // 1: iteration vectors are XOR combinations of index bits
    bool shape_given = false;  // false: the default shape for the width and kind of tile
    KernelShape shape;         // used when shape_given
};

struct Plan {
    int n = 0, w = 0, method = 0, t = 0;
    int npass = 0;  // 0 (n == 0 copy), 1 or 2
    bool naive = false;
    PassPlan pass[2];
    KernelShape shape;
    BitMat A;
    uint64_t c = 0;
};

// Tile row bits S = {j : column j of A is zero below row t}.  For invertible A,
// A is tiled at t (Section 5.1 condition) exactly when |S| = t.
uint64_t tiled_row_mask(const BitMat& A, int t);
inline bool is_tiled(const BitMat& A, int t) { return popcount64(tiled_row_mask(A, t)) == t; }

// A = U.L.P with U upper unitriangular, L lower unitriangular, P a permutation
// (Section 5.2), then T1 = U.R and T2 = R.L.P so that A = T1.T2 with both
// factors tiled at any t.  Returns false if A is singular.
bool factorize_ulp(const BitMat& A, BitMat* U, BitMat* L, BitMat* P, BitMat* T1, BitMat* T2);

// Geometry and tables of one pass out[T.x XOR c] = in[x] with read runs of
// 2^a and write runs of 2^b elements, for the given kernel shape; the tile
// subspace also contains the `nextra` input-space vectors `extra`.
// Returns 0 or a negative bmmc_status (BMMC_ERR_RANGE: the tile would not fit).
int build_pass(const BitMat& T, uint64_t c, int a, int b, const KernelShape& ks, int swizzle,
               uint64_t seed, PassPlan* out, int tb_mix = 0, int iter_mix = 0,
               const uint64_t* extra = nullptr, int nextra = 0);

// Full plan for out[A.x XOR c] = in[x].
int make_plan(const uint64_t* rows, uint64_t c, int n, int w, const PlanOptions& opt, Plan* out);

// Default kernel shape and run bits for an element width.
KernelShape default_shape(int w);
int default_t(const KernelShape& ks);
// Defaults of the general one-pass tile: its shape, and the read-run and
// write-run bits (a, b) with a + b <= D, so that any A fits one tile.
KernelShape general_shape(int w);
void general_runs(const KernelShape& ks, int* a, int* b);

// Bank-conflict residue of an LDS layout for the lanes of one wave
// (sum over read side / write side and 32 / 64 bank models of the rank
// deficit).  0 means every access is conflict-free in both models.
int lds_conflict_score(const PassTables& tab, const KernelShape& ks);

}  // namespace bmmc
