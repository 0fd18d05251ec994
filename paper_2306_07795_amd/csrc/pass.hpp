// Tables that drive one LDS-staged pass.  Shared by the host planner and the
// device kernels; plain data only.
//
// A pass moves out[T.x XOR c] = in[x] one tile at a time.  A tile is a coset
// r XOR V of a d-dimensional subspace V of the index space (paper, Section 4.1
// tiles and Section 5.1 tiled BMMCs; the iteration bits of Section 4.3 are
// extra dimensions of V).  Inside a tile an element has
//   * read coordinates v in [0, 2^d): input index  x = r XOR X(v),
//   * write coordinates u in [0, 2^d): output index y = T.r XOR c XOR Y(u),
// where X and Y are linear maps given by their values on the unit vectors.
// X keeps the low `a` input bits as its first coordinates and Y the low `b`
// output bits, so every run of 2^a read slots is a contiguous aligned run of
// the input and every run of 2^b write slots a contiguous aligned run of the
// output.  The element with read coordinates v sits in LDS at slot F(v); the
// element with write coordinates u at slot G(u) = F(M^-1 u).  All maps are
// XOR-linear, so each address is a XOR of a per-tile part, a per-thread part
// and a per-iteration part (the amortization of Section 4.3, extended to any
// tiled BMMC by linearity).
#pragma once
#include <cstdint>

namespace bmmc {

constexpr int kMaxTileBits = 16;  // largest tile: 2^16 elements
constexpr int kMaxTbBits = 32;    // index math is 32-bit: n <= 32

struct PassTables {
    uint32_t n;      // index bits of the array
    uint32_t d;      // tile bits used (d = min(n, D))
    uint32_t ntb;    // tile-selecting bits, n - d
    uint32_t c_hi;   // complement with its low b bits cleared
    uint32_t c_lds;  // LDS slot offset that absorbs the low b bits of c
    uint32_t pad_[3];
    uint32_t X[kMaxTileBits];    // input offset of read-coordinate bit k
    uint32_t F[kMaxTileBits];    // LDS slot of read-coordinate bit k
    uint32_t Y[kMaxTileBits];    // output offset of write-coordinate bit k
    uint32_t G[kMaxTileBits];    // LDS slot of write-coordinate bit k
    // Per tile-index bit j: tb[j][0] input offset, tb[j][1] output offset
    // (low b bits cleared), tb[j][2] LDS offset absorbing the low b bits of
    // T.tb[j][0]; tb[j][3] unused.  Interleaved so that one 16-byte scalar
    // load fetches all three.
    uint32_t tb[kMaxTbBits][4];
};

// One work item of the batched persistent kernel: a range of tiles of one
// pass of one array.
struct BatchItem {
    uint32_t pass;        // index into the pass table
    uint32_t tile_begin;  // first tile
    uint32_t tile_end;    // one past the last tile
    uint32_t pad_;
};

// Columns of the sorting network done inside each tile, in LDS, between the
// read and the write phase of a pass.  Column i pairs the slots s and
// s XOR f; bit 0 of the index, in column i's own index space, of the element
// at slot s is parity(beta & s) XOR parity(g & r), r the tile's coset
// representative; of each pair, the element whose bit is 0 keeps the smaller
// key.
constexpr int kMaxNetCols = 96;
struct NetCol {
    uint32_t f, beta, g;
    uint32_t rg;  // register groups: index of f in its group's basis (bits 0-2), q (bits 3-7)
};
// Register groups (full 2^13-slot tiles of 256 threads): a run of columns
// whose pair vectors are among kNetRegBits independent slot vectors S[0..4]
// is done in registers.  Thread t holds the 32 slots base(t) XOR S(j),
// j in [0, 32), where base(t) sets slot bit cpos[i] for each set bit i of t
// (the unit vectors cpos complete S to a basis of the slot space).  For a
// column with f = S[idx], the pair (j, j | 1 << idx) keeps the smaller key at
// j exactly when parity(g & r) XOR parity(beta & base(t)) XOR parity(q & j)
// is 0, q_k = parity(beta & S[k]).  One LDS round trip and one barrier per
// group instead of one barrier per column.
constexpr int kNetRegBits = 5;
constexpr int kMaxNetGroups = 32;
struct NetGroup {
    uint32_t S[kNetRegBits];
    uint32_t cpos;            // 8 slot-bit positions, 4 bits each, for thread bits 0..7
    uint32_t first, last;     // columns [first, last)
};
struct NetColumns {
    uint32_t count;
    uint32_t ngroups;  // 0: every column through LDS, one barrier each
    uint32_t pad_[2];
    NetCol col[kMaxNetCols];
    NetGroup grp[kMaxNetGroups];
};

// Per-pass device descriptor for the batched kernel.
struct BatchPass {
    const void* in;
    void* out;
    uint32_t w;      // element bytes
    uint32_t pad_[3];
    PassTables tab;
};

}  // namespace bmmc
