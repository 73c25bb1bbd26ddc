/*
 * gf2ref.c -- CPU oracle for dense matrix multiplication over GF(2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * What it computes is the plain definition of the product (Section 1 and
 * Section 2.3 of the paper): over GF(2) addition is XOR and multiplication
 * is AND, so for A (m x k) and B (k x n)
 *
 *     C[i][j] = XOR over t < k of (A[i][t] AND B[t][j]).
 *
 * It is evaluated row by row on the flat row-major packed layout of
 * Section 2.1 (64 entries per word): row i of C is the XOR of the rows t of
 * B for which bit t of row i of A is set, each row addition being a
 * word-wise XOR (Section 2.2).  No Gray-code tables, no blocking, no
 * Strassen-Winograd, no transposes.
 *
 * Layout: column j of a row is bit (j & 63) of word (j >> 6); rows are ld
 * words apart.  Bits at columns >= cols of a row's last word are padding:
 * inputs' padding is ignored; gf2ref_mul writes C's padding as zero;
 * accumulate mode (C ^= A*B) leaves it unchanged.  Words between
 * ceil(cols/64) and ld are never read or written.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static uint64_t last_word_mask(int64_t cols) {
    int r = (int)(cols & 63);
    return r == 0 ? ~(uint64_t)0 : (((uint64_t)1 << r) - 1);
}

/* One row of the product: acc = XOR of rows t of B with A[i][t] = 1. */
static void product_row(uint64_t* acc, const uint64_t* arow, const uint64_t* B, int64_t ldb,
                        int64_t k, int64_t W) {
    for (int64_t w = 0; w < W; ++w) acc[w] = 0;
    for (int64_t t = 0; t < k; ++t) {
        if ((arow[t >> 6] >> (t & 63)) & 1) {
            const uint64_t* brow = B + t * ldb;
            for (int64_t w = 0; w < W; ++w) acc[w] ^= brow[w];
        }
    }
}

static void store_row(uint64_t* crow, const uint64_t* acc, int64_t W, uint64_t mask, int accumulate) {
    for (int64_t w = 0; w < W; ++w) {
        uint64_t v = acc[w];
        if (w == W - 1) v &= mask;             /* padding bits of B never reach C */
        crow[w] = accumulate ? (crow[w] ^ v) : v;
    }
}

static int set_threads(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* C := A*B (accumulate = 0) or C := C + A*B (accumulate = 1).  Returns 0, or -1 on bad arguments. */
int gf2ref_mul(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
               int64_t m, int64_t k, int64_t n, int accumulate, int nthreads) {
    if (m < 0 || k < 0 || n < 0) return -1;
    int64_t W = (n + 63) >> 6;
    if (m == 0 || n == 0) return 0;
    if (ldc < W || (k > 0 && (lda < ((k + 63) >> 6) || ldb < W))) return -1;
    uint64_t mask = last_word_mask(n);
    int nt = set_threads(nthreads);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        uint64_t* acc = (uint64_t*)malloc((size_t)W * sizeof(uint64_t));
        if (!acc) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 8)
            for (int64_t i = 0; i < m; ++i) {
                product_row(acc, A + i * lda, B, ldb, k, W);
                store_row(C + i * ldc, acc, W, mask, accumulate);
            }
            free(acc);
        }
    }
    return fail ? -2 : 0;
}

/* Selected rows only: Cout row r (ldc words apart) receives row rows[r] of A*B.
 * Used to check very large products on sampled rows. */
int gf2ref_mul_rows(uint64_t* Cout, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                    int64_t m, int64_t k, int64_t n, const int64_t* rows, int64_t nrows, int nthreads) {
    if (m < 0 || k < 0 || n < 0 || nrows < 0) return -1;
    int64_t W = (n + 63) >> 6;
    if (n == 0 || nrows == 0) return 0;
    for (int64_t r = 0; r < nrows; ++r) if (rows[r] < 0 || rows[r] >= m) return -1;
    uint64_t mask = last_word_mask(n);
    int nt = set_threads(nthreads);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        uint64_t* acc = (uint64_t*)malloc((size_t)W * sizeof(uint64_t));
        if (!acc) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t r = 0; r < nrows; ++r) {
                product_row(acc, A + rows[r] * lda, B, ldb, k, W);
                store_row(Cout + r * ldc, acc, W, mask, 0);
            }
            free(acc);
        }
    }
    return fail ? -2 : 0;
}

/* Element-wise definition on unpacked 0/1 bytes (row-major, dense): the twin used
 * to pin the packed routine on small inputs. */
int gf2ref_mul_bruteforce(uint8_t* C, const uint8_t* A, const uint8_t* B, int64_t m, int64_t k, int64_t n) {
    if (m < 0 || k < 0 || n < 0) return -1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            uint8_t s = 0;
            for (int64_t t = 0; t < k; ++t) s ^= (uint8_t)(A[i * k + t] & B[t * n + j] & 1);
            C[i * n + j] = s;
        }
    return 0;
}

/* Matrix-vector product b' = A*v (Section 2.3): word-wise AND of row i with the
 * vector stored as a row, XOR-accumulate, then the parity of the word.  Output
 * is packed (bit i of word i>>6). */
int gf2ref_matvec(uint64_t* y, const uint64_t* A, int64_t lda, const uint64_t* v, int64_t m, int64_t k) {
    if (m < 0 || k < 0) return -1;
    int64_t Wk = (k + 63) >> 6, Wm = (m + 63) >> 6;
    uint64_t km = last_word_mask(k);
    for (int64_t w = 0; w < Wm; ++w) y[w] = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t p = 0;
        for (int64_t w = 0; w < Wk; ++w) {
            uint64_t a = A[i * lda + w] & v[w];
            if (w == Wk - 1) a &= km;
            p ^= a;
        }
        int par = 0;
        while (p) { par ^= 1; p &= p - 1; }
        y[i >> 6] |= (uint64_t)par << (i & 63);
    }
    return 0;
}

int gf2ref_max_threads(void) { return set_threads(0); }
