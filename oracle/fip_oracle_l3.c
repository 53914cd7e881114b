/*
 * TEST INFRASTRUCTURE ONLY -- the oracle of the other level-3 operations.
 *
 * Plain, slow references for the symmetric rank-k update (SYRK) and the
 * triangular matrix multiply (TRMM) the library runs through the same
 * fused-pack tile kernel.  The paper builds every level-3 operation of BLIS
 * on the one packing and microkernel layer (Sec. 2.2) and names carrying the
 * fused packing over to those operations as future work (Sec. 5); what the
 * operations compute is the BLAS definition, written out here in binary64.
 * Only the test suite may load this file's shared object; it shares no code
 * with the GPU library.
 *
 *   SYRK   C := alpha * op(A) * op(A)^T + beta * C, op(A) n x k (A for 'N',
 *          A^T for 'T'/'C'), on the uplo triangle of C ('L': i >= j, 'U':
 *          i <= j) only; the other triangle of C is neither read nor written.
 *   TRMM   C := alpha * op(T) * B + beta * C   (side 'L', T m x m), or
 *          C := alpha * B * op(T) + beta * C   (side 'R', T n x n),
 *          B and C m x n; T is the uplo triangle of the stored A ('L': stored
 *          row >= column, 'U': row <= column), its diagonal taken as 1 and not
 *          read when diag is 'U'; the other triangle of A is not read.  (BLAS
 *          overwrites B; here the product goes to a separate C, with beta.)
 *
 * Each entry is a sequential sum in ascending p over the terms the definition
 * has (for TRMM only the referenced entries of T, so a structural zero is never
 * multiplied), then alpha * sum + beta * C0 with beta == 0 not reading C0 and
 * alpha == 0 (or k == 0) not reading A or B.  The bound D is the same sum of
 * absolute values, |alpha| * sum |.| |.| + |beta| * |C0|.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>

#define L3_COL 0

static int l3_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static int l3_lower(char u) { return u == 'L' || u == 'l'; }
static int l3_left(char s) { return s == 'L' || s == 'l'; }
static int l3_unit(char d) { return d == 'U' || d == 'u'; }

/* Stored element (r, c) of a matrix with leading dimension ld. */
static double l3_stored(const double* X, int layout, int64_t ld, int64_t r, int64_t c)
{
    return layout == L3_COL ? X[r + c * ld] : X[r * ld + c];
}

static int64_t l3_index(int layout, int64_t ld, int64_t r, int64_t c)
{
    return layout == L3_COL ? r + c * ld : r * ld + c;
}

/* op(A)[r, c] of SYRK's n x k operand. */
static double syrk_op(const double* A, int layout, int64_t lda, char trans, int64_t r, int64_t c)
{
    return l3_trans(trans) ? l3_stored(A, layout, lda, c, r) : l3_stored(A, layout, lda, r, c);
}

/*
 * SYRK reference.  Cref and D use C's storage; only the uplo triangle of the
 * n x n result is written (the caller pre-fills Cref, e.g. with C0).
 */
void oracle_syrk(int layout, char uplo, char trans, int64_t n, int64_t k, double alpha,
                 const double* A, int64_t lda, double beta, const double* C0, int64_t ldc,
                 double* Cref, double* D)
{
    const int lower = l3_lower(uplo);
    const int use_a = alpha != 0.0 && k > 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i0 = lower ? j : 0, i1 = lower ? n : j + 1;
        for (int64_t i = i0; i < i1; ++i) {
            double s = 0.0, d = 0.0;
            if (use_a) {
                for (int64_t p = 0; p < k; ++p) {
                    const double a = syrk_op(A, layout, lda, trans, i, p);
                    const double b = syrk_op(A, layout, lda, trans, j, p);
                    s = s + a * b;
                    d = d + fabs(a) * fabs(b);
                }
            }
            const int64_t ci = l3_index(layout, ldc, i, j);
            double c = use_a ? alpha * s : 0.0;
            double dd = use_a ? fabs(alpha) * d : 0.0;
            if (beta != 0.0) {
                c = c + beta * C0[ci];
                dd = dd + fabs(beta) * fabs(C0[ci]);
            }
            Cref[ci] = c;
            D[ci] = dd;
        }
    }
}

/*
 * op(T)[r, c] of TRMM's triangular operand, and whether it is a referenced
 * entry (1) or a structural zero (0).  T is the uplo triangle of the stored A.
 */
static int trmm_op(const double* A, int layout, int64_t lda, char uplo, char trans, char diag,
                   int64_t r, int64_t c, double* v)
{
    const int64_t sr = l3_trans(trans) ? c : r, sc = l3_trans(trans) ? r : c;
    if (sr == sc && l3_unit(diag)) { *v = 1.0; return 1; }
    if (l3_lower(uplo) ? sr < sc : sr > sc) { *v = 0.0; return 0; }
    *v = l3_stored(A, layout, lda, sr, sc);
    return 1;
}

/*
 * TRMM reference (out of place).  B, Cref, D use their own storage; only the
 * m x n entries of Cref and D are written.
 */
void oracle_trmm(int layout, char side, char uplo, char transA, char diag, int64_t m, int64_t n,
                 double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double beta, const double* C0, int64_t ldc, double* Cref, double* D)
{
    const int left = l3_left(side);
    const int64_t k = left ? m : n;
    const int use_ab = alpha != 0.0 && k > 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0, d = 0.0;
            if (use_ab) {
                for (int64_t p = 0; p < k; ++p) {
                    double t, b;
                    int ref;
                    if (left) {
                        ref = trmm_op(A, layout, lda, uplo, transA, diag, i, p, &t);
                        if (!ref) continue;
                        b = l3_stored(B, layout, ldb, p, j);
                    } else {
                        ref = trmm_op(A, layout, lda, uplo, transA, diag, p, j, &t);
                        if (!ref) continue;
                        b = l3_stored(B, layout, ldb, i, p);
                    }
                    const double prod = left ? t * b : b * t;
                    s = s + prod;
                    d = d + fabs(t) * fabs(b);
                }
            }
            const int64_t ci = l3_index(layout, ldc, i, j);
            double c = use_ab ? alpha * s : 0.0;
            double dd = use_ab ? fabs(alpha) * d : 0.0;
            if (beta != 0.0) {
                c = c + beta * C0[ci];
                dd = dd + fabs(beta) * fabs(C0[ci]);
            }
            Cref[ci] = c;
            D[ci] = dd;
        }
    }
}
