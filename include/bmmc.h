/*
 * bmmc.h -- C interface of the MI355X BMMC permutation library (libbmmc.so).
 *
 * Operation (Bouverot-Dupuis & Sheeran, "Efficient GPU Implementation of
 * Affine Index Permutations on Arrays", FHPNC '23; Section 3, the affine map
 * y = A.x + c over F_2 and its per-bit expansion; Section 4.1, the kernel
 * that writes the element read at input index x to output index p(x) XOR c):
 *
 *     out[A.x XOR c] = in[x]     for every x in [0, 2^n)
 *
 * where an index x is the bit vector (x_0 .. x_{n-1}), bit 0 least
 * significant, A is an invertible n x n matrix over F_2 and c an n-bit
 * vector.  Elements are opaque blocks of elem_bytes bytes.
 *
 * Conventions shared by every entry point
 *   - A_rows: host array of n uint64 words; bit j of A_rows[i] is entry a_ij
 *     (row i produces output bit i).  Bits at positions >= n must be zero,
 *     as must bits of c at positions >= n.  The library copies A_rows and c
 *     before returning; the caller may free them at once.
 *   - in / out: device pointers owned by the caller, 16-byte aligned,
 *     2^n * elem_bytes bytes each, not overlapping (the method is out of
 *     place).  Ownership never passes to the library.
 *   - elem_bytes: 1, 2, 4, 8 or 16.  n: 0 .. BMMC_MAX_BITS.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *     entry points only enqueue work and return; results are visible after
 *     the stream is synchronized.  Faults inside kernels surface at that
 *     synchronization, not as a return code.
 *   - Return value: BMMC_OK (0) or a negative bmmc_status.  Arguments are
 *     validated before anything is enqueued, so an error return means no work
 *     was queued.  bmmc_last_error() gives a message for the calling thread.
 *   - Thread safety: every entry point may be called from several host
 *     threads; plans and scratch buffers are cached per device and stream.
 */
#ifndef BMMC_H
#define BMMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMMC_MAX_BITS 32
#define BMMC_VERSION 100

typedef enum {
    BMMC_OK = 0,
    BMMC_ERR_ARG = -1,      /* null pointer, bad width, bits beyond n, misaligned */
    BMMC_ERR_SINGULAR = -2, /* A is not invertible over F_2 */
    BMMC_ERR_RANGE = -3,    /* n, t or a tile size out of the supported range */
    BMMC_ERR_ALIAS = -4,    /* in and out overlap */
    BMMC_ERR_NOMEM = -5,    /* device or host allocation failed / budget exceeded */
    BMMC_ERR_HIP = -6,      /* a HIP runtime call failed (message in bmmc_last_error) */
    BMMC_ERR_INTERNAL = -7, /* planner invariant violated (a bug) */
    BMMC_ERR_NOTFOUND = -8, /* unknown ticket or handle */
    BMMC_ERR_BUSY = -9      /* request not finished yet (non-blocking poll) */
} bmmc_status;

/* How a permutation is carried out.  Every method gives the same result. */
typedef enum {
    /* One HBM round trip for every A: one tiled pass (Section 5.1) when A is
       tiled or the whole array fits one tile, otherwise one pass whose tile is
       the span of the low run_in input bits and of the inputs that reach the
       low run_out output bits (not in the paper; both sides still move runs
       of whole cache lines).  A tuned call may pick BMMC_METHOD_TILED where it
       measured faster. */
    BMMC_METHOD_AUTO = 0,
    /* The paper's scheme (Sections 5.1-5.2): one LDS-staged pass when A is
       tiled or the whole array fits one tile, otherwise the factorization
       A = (U.R)(R.L.P) and two passes through a library-owned scratch array. */
    BMMC_METHOD_TILED = 1,
    /* The general one-pass tile above, also for tiled A. */
    BMMC_METHOD_ONEPASS = 2,
    /* Lower bound: one lane per element, coalesced reads, scattered writes
       (the paper's naive kernels, Appendix). */
    BMMC_METHOD_NAIVE = 3
} bmmc_method;

/* Tuning knobs of one call; zero means "library default" everywhere.  Under
   BMMC_METHOD_AUTO and _ONEPASS the defaults for 4- and 8-byte arrays of
   more than 8 MiB depend on the size (up to 32 MiB, up to 256 MiB, beyond):
   a tile shape and runs when none of threads, iters, t, run_in, run_out is
   given, hints, tile_order and grid. */
typedef struct {
    int method;    /* bmmc_method */
    int t;         /* run bits: reads and writes move runs of 2^t elements */
    int threads;   /* work-group size: 256, 512 or 1024 */
    int iters;     /* 16-byte vectors per thread per tile */
    int swizzle;   /* 1 (default) conflict-avoiding LDS layout, -1 plain layout */
    /* work-groups per pass launch; -1 = one per tile; 0 = library default:
       one per tile, or for 4- and 8-byte arrays of more than 32 and up to
       256 MiB under BMMC_METHOD_AUTO / _ONEPASS twice the work-groups
       resident at once */
    int grid;
    int run_in;    /* read-run bits (input runs of 2^run_in elements); 0 = t */
    int run_out;   /* write-run bits (output runs of 2^run_out elements); 0 = t */
    /* 1: non-temporal loads, 2: non-temporal stores, 3: both, 4: neither;
       0: library default (size-dependent as above, else both for arrays of
       64 MiB and more, neither below).  Adding 8 (two-pass plans): the
       scratch array goes through the caches -- cached stores in the first
       pass, cached loads in the second, so that the second pass finds it in
       the 256 MB last-level cache; the default for arrays up to 256 MiB. */
    int hints;
    /* 1: give each XCD a contiguous range of tiles (work-groups are dealt
       to the XCDs round-robin); 2: select tiles through XOR-combined index
       bits; 3: both; 4: neither; 0: library default (size-dependent as
       above, else 2 for one-pass plans of tiled matrices larger than a
       tile, 4 otherwise).  Adding 8 also fills the tile with
       XOR-combined iteration bits instead of the lowest free index bits.
       Adding 16*k (k = 1..15) makes the k lowest tile-index bits step the
       output by one write run each (k = 15: every tile-index bit that can),
       so that tiles running side by side write neighbouring runs.
       Adding 256 (with the plain order, 4): where no vector of the tile
       moves the output's 4 KiB-block index bits (the three bits above a
       4 KiB block; bit permutations such as the bit reversal and the
       transposes allow it, random matrices do not), tile t writes only the
       blocks of index t mod 8 (XOR a constant from c), so that each of the
       eight XCDs, to which work-groups are dealt in turn, writes one eighth
       of the blocks; otherwise as without it. */
    int tile_order;
    int reserved[2];
} bmmc_options_t;

/* Result of planning one permutation (plain data, caller-owned, no free).
   Factor k is (rows[k], c[k]); factor 0 is applied first.  With two factors
   c[0] = 0 and c[1] = c (Section 5.2). */
typedef struct {
    int n, t, nfactors;        /* nfactors: 1 or 2 (0 when n == 0) */
    int elem_bytes;
    uint64_t rows[2][64];
    uint64_t c[2];
    uint64_t col_mask[2];      /* tile column bits: the low t input bits */
    uint64_t tile_rows_mask[2];/* tile row bits: inputs whose images are the low t outputs */
    uint64_t iter_mask[2];     /* iteration bits folded into the tile (Section 4.3) */
    uint64_t tb_mask[2];       /* bits that select the tile (one tile per value) */
    int n_over[2];             /* |col bits AND row bits| */
    int tile_bits[2];          /* log2 of elements per tile */
    int coordinate[2];         /* 1 when the tile is spanned by index bits */
    int lds_conflict_score[2]; /* 0 = every wave LDS access conflict-free */
} bmmc_plan_t;

/* One array of a batched call. */
typedef struct {
    const void* in;
    void* out;
    int n;
    int elem_bytes;
    const uint64_t* A_rows;
    uint64_t c;
} bmmc_desc_t;

/* Knobs of the batched persistent kernel; zero means default / autotuned. */
typedef struct {
    int workgroups;     /* persistent work-groups (default: fill every CU) */
    int chunk_tiles;    /* tiles per work item (default 4) */
    int order;          /* 0 = largest arrays first, 1 = input order */
    int use_graph;      /* 0 or 1 (default): replay a captured hipGraph; -1: plain launches */
    int method;         /* bmmc_method for the arrays larger than a tile */
    int hints;          /* as bmmc_options_t.hints (0: non-temporal above 64 MiB moved) */
    int iters;          /* tile size in 256s of 16-byte vectors: 4 (default: 256 threads x 4
                           vectors, 16 KiB), 8 (256 x 8, 32 KiB), 16 (512 x 8, 64 KiB) or
                           32 (1024 x 8, 128 KiB) */
    int tile_order;     /* as bmmc_options_t.tile_order, bits 1, 2, 16*k and 256 (0: plain order) */
} bmmc_batch_options_t;

/* Per-kernel timing gathered between bmmc_profile_begin and _end. */
typedef struct {
    char name[48];
    int launches;
    double total_ms;
    double bytes;       /* algorithmic bytes moved by those launches (read + write) */
} bmmc_kernel_stat_t;

/* Host emulation counters (see bmmc_emulate). */
typedef struct {
    int64_t tiles;
    int64_t read_instr, write_instr;      /* wave-level global accesses */
    int64_t read_lines, write_lines;      /* distinct 128-byte lines they touch */
    int64_t read_lines_min, write_lines_min;
    int64_t lds_instr;                    /* wave-level LDS accesses */
    int64_t lds_conflicts32, lds_conflicts64; /* extra cycles beyond 1 per group */
    int64_t lds_slot_errors;              /* slots not written exactly once / read exactly once */
    int64_t dealt_write_tiles;            /* tiles writing only 4 KiB blocks of index (tile XOR k) mod 8,
                                             k that of the pass's tile 0 */
} bmmc_emu_stats_t;

/* ------------------------------------------------------------ utilities */

/* Message for a status code.  Static string; never NULL. */
const char* bmmc_strerror(int status);
/* Message of the last failed call on this host thread ("" if none). */
const char* bmmc_last_error(void);
int bmmc_version(void);

/* --------------------------------------------------- host-only planning */

/* Tiled test (Section 5.1): is there a set S of t columns whose first t
   rows form an invertible block and whose last n-t rows are zero?  Returns
   1 (tiled; *rows_mask_out = S when not NULL), 0 (not tiled) or a negative
   status.  Host only; touches no device. */
int bmmc_is_tiled(const uint64_t* A_rows, int n, int t, uint64_t* rows_mask_out);

/* Factorization (Section 5.2): fills *plan_out with one factor (A, c) when A
   is tiled at the default t or 2^n fits one tile, else with
   (R.L.P, 0) then (U.R, c) where A = U.L.P.  bmmc_factorize_t picks t.
   Host only.  Errors: BMMC_ERR_ARG, _SINGULAR, _RANGE. */
int bmmc_factorize(const uint64_t* A_rows, uint64_t c, int n, bmmc_plan_t* plan_out);
int bmmc_factorize_t(const uint64_t* A_rows, uint64_t c, int n, int t, int elem_bytes,
                     bmmc_plan_t* plan_out);

/* The plan bmmc_permute_ex would run with these options (tile shape from
   threads / iters / t; NULL = defaults), for inspection.  The kernel for
   that shape need not exist.  Host only.  Errors: _ARG, _SINGULAR, _RANGE. */
int bmmc_plan_ex(const uint64_t* A_rows, uint64_t c, int n, int elem_bytes,
                 const bmmc_options_t* opts, bmmc_plan_t* plan_out);

/* The raw factorization of Section 5.2: A = U.L.P with U upper
   unitriangular, L lower unitriangular and P a permutation matrix, and the
   tiled factors T1 = U.R, T2 = R.L.P (R the bit reversal), so A = T1.T2.
   Each output is a host array of n rows in the A_rows encoding; any may be
   NULL.  Host only.  Errors: _ARG, _RANGE, _SINGULAR. */
int bmmc_factorize_ulp(const uint64_t* A_rows, int n, uint64_t* U, uint64_t* L, uint64_t* P,
                       uint64_t* T1, uint64_t* T2);

/* ------------------------------------------------- host BMMC algebra */

/* Composition (Section 3 fusion rule): bmmc(A, c) after bmmc(B, d) equals
   bmmc(A.B, A.d XOR c).  Writes n rows to out_rows and the complement to
   *out_c (out_rows may alias A_rows or B_rows).  Host only.
   Errors: _ARG (NULL pointer, bits beyond n), _RANGE (n outside 1..64). */
int bmmc_compose(const uint64_t* A_rows, uint64_t c, const uint64_t* B_rows, uint64_t d, int n,
                 uint64_t* out_rows, uint64_t* out_c);

/* Inverse: (A^-1, A^-1.c) undoes (A, c).  Host only.  Errors: _ARG,
   _RANGE, _SINGULAR. */
int bmmc_invert(const uint64_t* A_rows, uint64_t c, int n, uint64_t* out_rows, uint64_t* out_c);

/* The BMMC that makes parm's two sub-arrays contiguous (Section 7.2): for a
   nonzero n-bit mask with lowest set bit l, y_i = x_i for i < l,
   y_i = x_(i+1) for l <= i < n-1, and y_(n-1) = x.mask (F_2 dot product), so
   that parm mask f = bmmc(A^-1, 0) . parm 2^(n-1) f . bmmc(A, 0).  Writes A
   to rows_out and A^-1 to inv_rows_out (either may be NULL).  Host only.
   Errors: _ARG (mask zero or beyond n), _RANGE. */
int bmmc_parm_matrix(uint64_t mask, int n, uint64_t* rows_out, uint64_t* inv_rows_out);

/* Apply a sequence of `count` BMMCs (first one first) as ONE permutation:
   the sequence is fused on the host with the composition rule and the
   result is run as bmmc_permute would run it.  A_rows_seq holds count * n
   rows, c_seq count complements.  Errors: as bmmc_permute. */
int bmmc_permute_seq(const void* in, void* out, int n, int count, const uint64_t* A_rows_seq,
                     const uint64_t* c_seq, int elem_bytes, void* stream);

/* ----------------------------------------- sorting network (Section 7.1) */

/* Key order of the sorting network. */
typedef enum {
    BMMC_KEY_I32 = 0, /* 4-byte keys compared as signed 32-bit integers */
    BMMC_KEY_U32 = 1  /* 4-byte keys compared as unsigned 32-bit integers */
} bmmc_key_type;

/* How the network runs. */
typedef enum {
    /* parm compiled to BMMCs (Section 7.2) and fused (Section 3), then
       consecutive stages grouped into LDS-staged passes whose reads and
       writes are coalesced: each pass applies the product of its BMMCs and
       runs its compare-exchange columns on every staged tile in LDS (a column
       joins a pass when all its pairs lie inside the pass's tiles). */
    BMMC_SORTNET_PASSES = 0,
    /* every column in place at the keys' own positions (no permutations;
       accesses as scattered as the column's pairs): the uncompiled form */
    BMMC_SORTNET_DIRECT = 1
} bmmc_sortnet_method;

/* The network as the compiled sequence M_0, C, M_1, C, ..., C, M_S of
   S = n(n+1)/2 compare-exchange columns C between fused BMMCs (linear, c = 0),
   where C orders each pair (2k, 2k+1) of the index space it sees, smaller key
   first, and M_S ... M_0 = I.  Writes *count_out = S + 1 and, when rows_out
   is not NULL, matrix s to rows_out[s*n .. s*n + n-1] (room for max_matrices
   matrices).  Host only.  Errors: _RANGE (n, or too little room),
   _INTERNAL. */
int bmmc_sortnet_stages(int n, uint64_t* rows_out, int max_matrices, int* count_out);

/* The device passes of BMMC_SORTNET_PASSES for 2^n keys: *passes_out (the
   number of passes, each one read and one write of the array) and
   *columns_out (the most columns one pass runs); either may be NULL.
   2 <= n <= BMMC_MAX_BITS.  Host only.  Errors: _RANGE, _INTERNAL. */
int bmmc_sortnet_passes(int n, int* passes_out, int* columns_out);

/* Sort 2^n 4-byte keys ascending with the sorting network of Section 7.1
   (even/odd merge sort, balanced periodic merger, written with parm):
   out = the keys of in in ascending key_type order.  in and out are distinct
   16-byte aligned device buffers of 4 * 2^n bytes; BMMC_SORTNET_PASSES uses
   the library's per-stream scratch array of the same size.  Asynchronous on
   `stream`.  Errors: _ARG, _RANGE, _ALIAS, _NOMEM, _HIP, _INTERNAL. */
int bmmc_sortnet(const void* in, void* out, int n, int key_type, int method, void* stream);

/* Host emulation of bmmc_sortnet's BMMC_SORTNET_PASSES form, for tests: the
   same passes with the same tables, tile by tile, on HOST memory (in/out are
   host pointers); *passes_out (may be NULL) receives the number of passes.
   2 <= n <= 24.  Errors: _ARG, _RANGE, _INTERNAL. */
int bmmc_sortnet_emulate(const void* in, void* out, int n, int key_type, int* passes_out);

/* Host emulation of the tiled kernels' address arithmetic, for tests: runs
   the same plan, tile by tile and lane by lane, on host memory (in/out are
   HOST pointers here) and counts coalescing, LDS bank conflicts and LDS
   slot use.  Never used by the device entry points.  stats may be NULL. */
int bmmc_emulate(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                 int elem_bytes, const bmmc_options_t* opts, bmmc_emu_stats_t* stats);

/* ------------------------------------------------------- device calls */

/* The permutation out[A.x XOR c] = in[x]: the affine map x -> A.x XOR c over
   F_2 of Section 3, applied in the scatter direction of the Section 4.1
   kernel (the element read at x is written at A.x XOR c).  Runs by
   BMMC_METHOD_AUTO with the options bmmc_autotune stored for (n, elem_bytes)
   and the class of A, else with the size-dependent defaults; arrays above
   256 MiB whose three output index bits above a 4 KiB block depend only on
   the same three input bits (XOR translations such as the reversal, bit
   permutations of the other bits) take dealt output blocks (tile_order
   260) instead, on 16 KiB tiles (512 threads x 2 vectors) for 4- and
   8-byte elements.  From 64 MiB on
   these are tuned for a call that finds the caches full of other data (the
   tuner flushes them before every timed call); below, for calls repeated on
   arrays that stay in the caches.  Plans are cached
   by (A, c, n, elem_bytes, options); two-pass plans (BMMC_METHOD_TILED) use a
   scratch array of 2^n * elem_bytes owned by the library (kept per device
   and stream, grown on demand).
   Errors: _ARG, _SINGULAR, _RANGE, _ALIAS, _NOMEM, _HIP. */
int bmmc_permute(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                 int elem_bytes, void* stream);

/* Same operation with explicit options (method, tile width, launch shape). */
int bmmc_permute_ex(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                    int elem_bytes, const bmmc_options_t* opts, void* stream);

/* Lower bound of the paper's ablation (Appendix naive kernel): one lane per
   element, coalesced read, write scattered to A.x XOR c. */
int bmmc_permute_naive(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c,
                       int elem_bytes, void* stream);

/* Upper bound (Section 2.3 "copy"): out[i] = in[i] for `bytes` bytes with
   16-byte vector loads and stores.  Pointers must not overlap. */
int bmmc_copy(const void* in, void* out, size_t bytes, void* stream);
/* The same copy with a chosen kernel: vpt 16-byte vectors per lane (1, 2, 4
   or 8); hints bit 0 makes the loads and bit 1 the stores non-temporal.
   bmmc_copy uses vpt = 2 with non-temporal stores for 64 MiB and more,
   vpt = 4 without hints below. */
int bmmc_copy_ex(const void* in, void* out, size_t bytes, int vpt, int hints, void* stream);

/* Many independent permutations, each with its own n, width, A and c, in one
   replay of a captured hipGraph holding two launches of a persistent kernel:
   the first runs every one-pass array (those that fit one tile, or are tiled)
   and the first passes of the others (the paper's two tiled passes), the
   second runs those second passes.  Arrays of 1- or 2-byte elements, or too
   small for one 16-byte vector, go through the single-array kernels on the
   same stream.  descs is
   a host array of `count` descriptors; every in/out pair obeys the rules
   above and no out may overlap another array's in or out.  Scratch, the
   device descriptor table and the graph are owned by the library.  Options
   come from the tuning cache for this histogram of (n, width); without an
   entry, batches moving 256 MiB or more take 128 KiB tiles, one per work
   item, smaller ones the defaults of bmmc_batch_options_t.
   Errors: as bmmc_permute, reported for the first bad descriptor. */
int bmmc_permute_batched(const bmmc_desc_t* descs, int count, void* stream);
int bmmc_permute_batched_ex(const bmmc_desc_t* descs, int count,
                            const bmmc_batch_options_t* opts, void* stream);

/* A batch kept resident on the device: plans, the device descriptor table,
   a scratch array for the two-pass arrays and the captured graph are made
   once; each bmmc_batch_launch is one graph replay (plus the single-array
   launches of arrays the persistent kernel does not take).  The descriptors'
   buffers must stay valid until bmmc_batch_destroy; launches of one handle
   must not overlap (they share the scratch and the work counters).
   Errors: as bmmc_permute_batched, plus _NOMEM for the owned buffers. */
int bmmc_batch_create(const bmmc_desc_t* descs, int count, const bmmc_batch_options_t* opts,
                      void** handle_out);
int bmmc_batch_launch(void* handle, void* stream);
int bmmc_batch_destroy(void* handle);

/* bmmc_permute_batched for callers that cannot allocate device memory (code
   that must not call hipMalloc: tight serving loops, harnesses that forbid
   it).  Same descriptors, options (NULL: as bmmc_permute_batched) and
   results; no hipMalloc, hipFree or other allocating routine is called.
   The batch's descriptor table, work items and queue heads go into one
   fixed device array of bmmc_noalloc_table_bytes() bytes (4 MiB) that the
   library holds on each device it runs on until the process ends; the
   kernels run as plain launches (no graph).  Every call on a device shares
   that array and leaves its contents behind (the queue heads are cleared
   by a kernel at the start of each call): calls that overlap on one device,
   from any stream or thread, race and must be serialized by the caller;
   calls one after another on one stream are safe.
   Errors: as bmmc_permute_batched; _RANGE when the batch's table does not fit
   the fixed array (about 4 MiB: a few thousand arrays), _ARG for
   BMMC_METHOD_TILED (two-pass arrays need scratch as large as themselves). */
int bmmc_permute_batched_noalloc(const bmmc_desc_t* descs, int count,
                                 const bmmc_batch_options_t* opts, void* stream);
size_t bmmc_noalloc_table_bytes(void);

/* ------------------------------------------------------------- autotuner */

/* Time the available tile shapes (threads x iterations), run widths, cache
   hints, tile orders and grid sizes (with BMMC_METHOD_AUTO also the two-pass
   scheme) on 2^n elements of elem_bytes bytes, `reps` timed runs each, on
   `stream` (synchronizes it), for two classes of matrices: random matrices
   (class 0: not tiled; three, six from 256 MiB on) and three bit
   permutations (class 1: tiled; a random one, the bit reversal, the
   half-split transpose), times summed.  The
   fastest of each class is cached for (n, elem_bytes, method, class) and used
   by later calls that pass no options, by the class of their matrix; class
   0's is also returned.  Below 64 MiB the `reps` calls of a candidate are
   captured into a graph (on a stream of its own) and the replay is timed;
   from 64 MiB on each call is timed on its own right after a 512 MiB copy
   between two other buffers, which leaves the caches full of other data.
   Allocates two temporary buffers of 2^n * elem_bytes (and two of 512 MiB
   from 64 MiB on).
   Errors: _RANGE, _ARG, _NOMEM, _HIP. */
int bmmc_autotune(int n, int elem_bytes, int method, void* stream, int reps,
                  bmmc_options_t* best_out, double* best_ms);

/* The tuned options of `method` for this matrix (BMMC_METHOD_AUTO only,
   from bmmc_autotune_matrix) or else for its class: returns 1 and fills
   *opts_out when the cache holds an entry, else 0.  With BMMC_METHOD_AUTO
   these are the options a call without options uses (else the library
   defaults).  Host only.  Errors: _ARG, _RANGE. */
int bmmc_tune_lookup(int n, int elem_bytes, int method, const uint64_t* A_rows, bmmc_options_t* opts_out);

/* Tune for one matrix (the permutation of bmmc_permute, Section 3 map in the
   Section 4.1 scatter direction; BMMC_METHOD_AUTO): times, on
   these buffers, the options a call would use now under every tile order,
   then a few other tile shapes (4- and 8-byte elements), and keeps the
   fastest for later bmmc_permute calls (and served requests planned as
   single-array calls) with this A and n, for any c.  Beyond the last-level cache the best setting differs from one
   random matrix to the next.  Runs the permutation some 100-300 times and
   synchronizes `stream`; `out` ends up holding the permutation of `in`.
   The settings are kept in memory only (at most 4096 matrices: with 4096
   stored, all are dropped before the next is added).  in, out: device buffers of 2^n * elem_bytes,
   16-byte aligned, not overlapping.  *best_ms (if not NULL) receives the
   time of one call.  Errors: _ARG, _RANGE, _ALIAS, _SINGULAR, _NOMEM, _HIP. */
int bmmc_autotune_matrix(const void* in, void* out, int n, const uint64_t* A_rows, uint64_t c, int elem_bytes,
                         void* stream, int reps, bmmc_options_t* best_out, double* best_ms);

/* Forget every setting bmmc_autotune_matrix stored.  Host only. */
int bmmc_tune_clear_matrices(void);

/* Time method, tile size, chunk size, queue order and persistent grid size
   of the batched kernel on this very batch, then tile orders for the best
   (it runs the batch 1 + reps times per candidate); the fastest is cached
   for batches with the same histogram of (n, width). */
int bmmc_autotune_batched(const bmmc_desc_t* descs, int count, void* stream, int reps,
                          bmmc_batch_options_t* best_out, double* best_ms);

/* The tuned batch options for batches with this histogram of (n, width):
   returns 1 and fills *opts_out when the cache holds an entry, else 0.
   These are the options bmmc_permute_batched and bmmc_batch_create use when
   given none.  Host only.  Errors: _ARG. */
int bmmc_tune_lookup_batched(const bmmc_desc_t* descs, int count, bmmc_batch_options_t* opts_out);

/* Save / load the tuning cache as JSON lines.  On first use the cache holds
   the tuning results shipped with the library (tuning/gfx950.jsonl beside
   libbmmc.so, measured on MI355X); BMMC_TUNE_CACHE, when set, names another
   file to load instead (and to rewrite after each tuning run), an empty value
   none.  bmmc_tune_load adds a file's entries and returns their number. */
int bmmc_tune_save(const char* path);
int bmmc_tune_load(const char* path);

/* --------------------------------------------------------------- serving */

typedef struct {
    int64_t budget_bytes; /* HBM budget: input + output + scratch of admitted requests */
    int streams;          /* concurrent batched launches (default 4, at most 16) */
    int max_batch;        /* requests per launch (0 = all admitted) */
    /* 0: the caller passes `out`; 1: the server allocates `out` from its
       arena and keeps it until bmmc_server_release; 2: as 1, but the output
       is dropped at completion and the ticket forgotten (load generation). */
    int own_outputs;
    int method;           /* bmmc_method for two-pass-sized arrays */
    /* 0 (default): each launch is plain launches of the batched kernel with
       no more work-groups than the batch has work items; 1: a replay of a
       captured graph with a fixed persistent grid */
    int use_graph;
    /* launches of at most this many requests run them as their own tiled
       launches (0: default 4; negative: never, every launch is batched) */
    int direct_max;
    /* requests of at least 2^solo_log2 bytes are planned like a
       bmmc_permute call without options (tuned options of their size and
       matrix class) and always run as their own launch (0: default 24,
       16 MiB; negative: never) */
    int solo_log2;
    int reserved[1];
} bmmc_server_options_t;

typedef struct {
    int64_t submitted, completed, rejected, batches;
    double bytes_moved;   /* algorithmic bytes (read + write) of completed requests */
    double busy_s;        /* first arrival to last completion */
    double p50_ms, p99_ms, mean_ms, max_ms;  /* arrival-to-completion latency */
    int64_t in_use_bytes, peak_bytes;
    double mean_batch;    /* requests per launch */
    /* mean of each stage of a completed request's latency: arrival to
       planned, planned to launched (admission and a free stream), launched to
       completion seen by the server */
    double mean_plan_ms, mean_wait_ms, mean_run_ms;
    double reserved[1];
} bmmc_server_stats_t;

/* A continuous-batching server on the current device.  It allocates one
   device arena (the largest power of two <= budget_bytes) for outputs and
   scratch, `streams` HIP streams at default priority, four planner threads
   and one dispatcher thread (they spin for up to 200 us before sleeping, so
   a busy server keeps five host cores busy).
   Requests are admitted in arrival order while input + output + scratch of
   all admitted, unfinished requests fits budget_bytes; admitted requests join
   the next launch on a free stream (up to direct_max requests as their own
   tiled launches, more as one batched persistent launch); while another
   stream is free or at most 16 requests wait, a request planned as its own
   launch (solo_log2) goes alone and a launch takes only the run of small
   requests ahead of the next such request, the rest going to the next free
   stream; a longer queue goes into one launch.
   Errors: _ARG, _NOMEM. */
int bmmc_server_create(const bmmc_server_options_t* opts, void** handle_out);

/* Queue one permutation.  desc->in must stay valid and unchanged until the
   request completes; desc->out is used only when own_outputs == 0.  A_rows is
   copied.  arrival_ns is on the bmmc_server_now_ns clock (0 = now); a future
   time holds the request back until then, and latency is measured from it.
   Errors: _ARG, _RANGE, _NOMEM (can never fit the budget). */
int bmmc_server_submit(void* handle, const bmmc_desc_t* desc, int64_t arrival_ns, int64_t* ticket_out);

/* State of a ticket: BMMC_OK with the completion time and output pointer,
   BMMC_ERR_BUSY while pending (wait = 0), or the error the request failed
   with.  wait != 0 blocks until completion.  With own_outputs == 2 a
   request is forgotten when it finishes: its ticket then reads
   BMMC_ERR_NOTFOUND, and wait != 0 is refused with BMMC_ERR_ARG. */
int bmmc_server_poll(void* handle, int64_t ticket, int wait, int64_t* done_ns, void** out_ptr);

/* Forget a finished ticket and free its output (own_outputs == 1). */
int bmmc_server_release(void* handle, int64_t ticket);

/* Block until every submitted request has finished. */
int bmmc_server_drain(void* handle);

int bmmc_server_stats(void* handle, bmmc_server_stats_t* stats);

/* Start the statistics afresh (counts, latencies, busy time; the peak
   restarts from the bytes in use), e.g. after a warm-up.  Requests still in
   flight count toward the new statistics when they finish. */
int bmmc_server_reset_stats(void* handle);

/* Stop the server threads, wait for its streams and free its memory. */
int bmmc_server_destroy(void* handle);

/* The server's clock (steady clock, nanoseconds). */
int64_t bmmc_server_now_ns(void);

/* The unbatched baseline of the server, on the same request stream: request
   k runs as its own bmmc_permute call, issued at arrival_ns[k] (server
   clock) on stream k mod `streams` by that stream's issuing thread (one per
   stream, each planning its own requests), with no admission and no
   batching; a second thread per stream stamps each request's completion
   when an event recorded after it has passed.  Requests of one stream run in
   order, so they may share an output buffer; every descriptor obeys the
   rules of bmmc_permute.  Blocks until every request has completed and
   fills *stats_out as bmmc_server_stats does (one launch per request; plan
   time = arrival to the call's return, run time = return to completion;
   no budget figures).  streams: 1..16 (0: 4).  Creates and destroys its
   own streams.  Errors: _ARG, _RANGE, _HIP, or the first request's error
   (the others still run). */
int bmmc_serve_direct(const bmmc_desc_t* descs, const int64_t* arrival_ns, int count, int streams,
                      bmmc_server_stats_t* stats_out);

/* ------------------------------------------------------------ profiling */

/* Start timing every launch the library makes on this device: a hipEvent
   pair bound to each single kernel's own dispatch (hipExtLaunchKernel; the
   interval is the kernel's execution and nothing is enqueued between
   kernels), or recorded around a batched launch's graph or kernels.
   Launches onto a stream under capture are not timed.  bmmc_profile_end
   waits for the events, fills up to `max` entries (one per kernel name, e.g.
   "k_tiled<4,512,8,3>", "k_copy<vpt,hints>", "k_batched") and returns how
   many it filled. */
int bmmc_profile_begin(void);
int bmmc_profile_end(bmmc_kernel_stat_t* out, int max);

#ifdef __cplusplus
}
#endif

#endif /* BMMC_H */
