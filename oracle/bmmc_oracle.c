/*
 * bmmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU definition of a BMMC permutation, used
 * to check the GPU library.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, header,
 * table or helper with the GPU library and includes nothing from it.
 *
 * What is computed (paper, Section 3 "Key ideas", the affine map and its
 * per-bit expansion): an index x in [0, 2^n) is the vector (x_0 .. x_{n-1}) of
 * its bits, bit 0 being the least significant.  For an n x n matrix A over F_2
 * and a vector c,
 *
 *       y_i = (sum_j a_ij * x_j  mod 2)  XOR  c_i          for i = 0 .. n-1.
 *
 * Direction (paper, Section 4.1 kernel, where the tile element read from
 * input position x is written to output position p(x) XOR c; and Section 7.2,
 * where the element found at index x is sent to index y): the permutation is a
 * scatter,
 *
 *       out[A.x XOR c] = in[x]      for every x.
 *
 * Matrix encoding used at this interface: rows[i] is a 64-bit word whose bit j
 * is a_ij (row i produces output bit i).  The dense helpers below work on one
 * byte per matrix entry, a[i*n + j] = a_ij, and never use packed rows, so that
 * they stay independent of any packed-row code elsewhere.
 *
 * Elements are opaque blocks of w bytes; no arithmetic is done on them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Output bit i of A.x XOR c, evaluated entry by entry (Section 3, per-bit form). */
static inline uint64_t apply_bitwise(const uint64_t *rows, uint64_t c, int n, uint64_t x)
{
    uint64_t y = 0;
    for (int i = 0; i < n; i++) {
        /* sum over j of a_ij * x_j, mod 2: the parity of (row_i AND x). */
        int s = __builtin_parityll(rows[i] & x);
        int ci = (int)((c >> i) & 1u);
        y |= (uint64_t)(s ^ ci) << i;
    }
    return y;
}

uint64_t oracle_apply(const uint64_t *rows, uint64_t c, int n, uint64_t x)
{
    return apply_bitwise(rows, c, n, x);
}

/* ys[k] = A.xs[k] XOR c for k < count (used to check sampled outputs at full size). */
void oracle_apply_many(const uint64_t *rows, uint64_t c, int n,
                       const uint64_t *xs, uint64_t *ys, int64_t count)
{
    for (int64_t k = 0; k < count; k++)
        ys[k] = apply_bitwise(rows, c, n, xs[k]);
}

/* The same per-bit definition written with the double sum spelled out
 * (no parity builtin); used by the tests on tiny n to check the fast form. */
uint64_t oracle_apply_sum(const uint64_t *rows, uint64_t c, int n, uint64_t x)
{
    uint64_t y = 0;
    for (int i = 0; i < n; i++) {
        int s = 0;
        for (int j = 0; j < n; j++) {
            int aij = (int)((rows[i] >> j) & 1u);
            int xj = (int)((x >> j) & 1u);
            s = (s + aij * xj) % 2;
        }
        y |= (uint64_t)((s + (int)((c >> i) & 1u)) % 2) << i;
    }
    return y;
}

/*
 * out[A.x XOR c] = in[x] for every x in [0, 2^n), elements of w bytes.
 * Returns 0, or -1 on bad arguments.  A must be invertible for the result to
 * be a permutation; that is the caller's business here (the tests check
 * bijectivity separately).  nthreads <= 0 means "OpenMP default".
 */
int oracle_permute(const void *in, void *out, int n, const uint64_t *rows, uint64_t c,
                   int w, int nthreads)
{
    if (n < 0 || n > 40 || w <= 0 || in == NULL || out == NULL || rows == NULL)
        return -1;
    const unsigned char *src = (const unsigned char *)in;
    unsigned char *dst = (unsigned char *)out;
    const int64_t size = (int64_t)1 << n;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* Each destination is written once because the map is a bijection, so the
       iterations are independent. */
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < size; x++) {
        uint64_t y = apply_bitwise(rows, c, n, (uint64_t)x);
        memcpy(dst + (int64_t)y * w, src + x * w, (size_t)w);
    }
    return 0;
}

/* Number of threads an OpenMP parallel region would use with this request. */
int oracle_threads(int nthreads)
{
#ifdef _OPENMP
    int got = 1;
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        got = omp_get_num_threads();
    }
    return got;
#else
    (void)nthreads;
    return 1;
#endif
}

/* ---------------- dense F_2 helpers (one byte per entry) ---------------- */

/* out = a.b over F_2: (ab)_ij = sum_k a_ik b_kj mod 2. */
void oracle_mul(const uint8_t *a, const uint8_t *b, uint8_t *out, int n)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int s = 0;
            for (int k = 0; k < n; k++)
                s ^= (a[i * n + k] & b[k * n + j]) & 1;
            out[i * n + j] = (uint8_t)s;
        }
}

/* Rank over F_2 by Gaussian elimination on a copy. */
int oracle_rank(const uint8_t *a, int n_rows, int n_cols)
{
    uint8_t *m = (uint8_t *)malloc((size_t)n_rows * n_cols + 1);
    memcpy(m, a, (size_t)n_rows * n_cols);
    int rank = 0;
    for (int col = 0; col < n_cols && rank < n_rows; col++) {
        int piv = -1;
        for (int r = rank; r < n_rows; r++)
            if (m[r * n_cols + col]) { piv = r; break; }
        if (piv < 0)
            continue;
        if (piv != rank)
            for (int j = 0; j < n_cols; j++) {
                uint8_t t = m[piv * n_cols + j];
                m[piv * n_cols + j] = m[rank * n_cols + j];
                m[rank * n_cols + j] = t;
            }
        for (int r = 0; r < n_rows; r++)
            if (r != rank && m[r * n_cols + col])
                for (int j = 0; j < n_cols; j++)
                    m[r * n_cols + j] ^= m[rank * n_cols + j];
        rank++;
    }
    free(m);
    return rank;
}

/* Inverse by Gauss-Jordan on [a | I].  Returns 0, or -1 if a is singular. */
int oracle_inverse(const uint8_t *a, uint8_t *inv, int n)
{
    int w = 2 * n;
    uint8_t *m = (uint8_t *)calloc((size_t)n * w + 1, 1);
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++)
            m[i * w + j] = a[i * n + j] & 1;
        m[i * w + n + i] = 1;
    }
    for (int col = 0; col < n; col++) {
        int piv = -1;
        for (int r = col; r < n; r++)
            if (m[r * w + col]) { piv = r; break; }
        if (piv < 0) { free(m); return -1; }
        if (piv != col)
            for (int j = 0; j < w; j++) {
                uint8_t t = m[piv * w + j];
                m[piv * w + j] = m[col * w + j];
                m[col * w + j] = t;
            }
        for (int r = 0; r < n; r++)
            if (r != col && m[r * w + col])
                for (int j = 0; j < w; j++)
                    m[r * w + j] ^= m[col * w + j];
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            inv[i * n + j] = m[i * w + n + j];
    free(m);
    return 0;
}

/*
 * Tiled condition at width t (paper, Section 5.1): there are t columns
 * i_1..i_t such that the block of the first t rows on those columns is
 * invertible and the block of the last n-t rows on those columns is zero.
 * Written literally: collect the columns whose last n-t rows are zero, then try
 * every t-subset of them.  Returns 1 if tiled, 0 if not; if cols_out is not
 * NULL it receives a bit mask of the first qualifying subset found.
 */
int oracle_is_tiled(const uint8_t *a, int n, int t, uint64_t *cols_out)
{
    if (t < 0 || t > n)
        return 0;
    int cand[64], nc = 0;
    for (int j = 0; j < n; j++) {
        int zero_bottom = 1;
        for (int i = t; i < n; i++)
            if (a[i * n + j]) { zero_bottom = 0; break; }
        if (zero_bottom)
            cand[nc++] = j;
    }
    if (nc < t)
        return 0;
    if (t == 0) {
        if (cols_out) *cols_out = 0;
        return 1;
    }
    /* enumerate t-subsets of cand in lexicographic order */
    int idx[64];
    for (int k = 0; k < t; k++)
        idx[k] = k;
    uint8_t *blk = (uint8_t *)malloc((size_t)t * t);
    for (;;) {
        for (int r = 0; r < t; r++)
            for (int k = 0; k < t; k++)
                blk[r * t + k] = a[r * n + cand[idx[k]]];
        if (oracle_rank(blk, t, t) == t) {
            if (cols_out) {
                uint64_t mask = 0;
                for (int k = 0; k < t; k++)
                    mask |= (uint64_t)1 << cand[idx[k]];
                *cols_out = mask;
            }
            free(blk);
            return 1;
        }
        int k = t - 1;
        while (k >= 0 && idx[k] == nc - t + k)
            k--;
        if (k < 0)
            break;
        idx[k]++;
        for (int m = k + 1; m < t; m++)
            idx[m] = idx[m - 1] + 1;
    }
    free(blk);
    return 0;
}
