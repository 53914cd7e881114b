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
 *   TRSM   solve op(T) * X = alpha * B (side 'L', T m x m) or
 *          X * op(T) = alpha * B (side 'R', T n x n) for X, B m x n; T as for
 *          TRMM.  The solution is written to a separate X (BLAS overwrites B).
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

/*
 * TRSM reference: substitution, one right-hand side at a time (a column of B
 * for side 'L', a row for side 'R'), in the order the triangle dictates.
 * With S the matrix acting on that right-hand side (S = op(T) for side 'L',
 * S = op(T)^T for side 'R', since X op(T) = alpha B is op(T)^T x = alpha b for
 * each row x of X), the unknowns are solved from the end of S's nonzero band
 * inward:
 *   x_r = (alpha * b_r - sum_c S[r, c] x_c) / S[r, r]
 * where c runs over the already solved unknowns (c < r for lower S, c > r for
 * upper S) in the order they were solved, and the division is skipped for a
 * unit diagonal.  alpha == 0 gives X = 0 without reading A or B.  X uses B's
 * storage convention (layout, ldx).
 */
void oracle_trsm(int layout, char side, char uplo, char transA, char diag, int64_t m, int64_t n,
                 double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double* X, int64_t ldx)
{
    const int left = l3_left(side);
    const int64_t k = left ? m : n;        /* order of T */
    const int64_t nrhs = left ? n : m;
    /* S lower?  op(T) is lower when uplo is lower and not transposed, or upper
       and transposed; side 'R' acts with op(T)^T, which flips it. */
    const int op_lower = l3_lower(uplo) != l3_trans(transA);
    const int s_lower = left ? op_lower : !op_lower;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t v = 0; v < nrhs; ++v) {
        for (int64_t t = 0; t < k; ++t) {
            const int64_t r = s_lower ? t : k - 1 - t;
            const int64_t xi = left ? r : v, xj = left ? v : r;
            if (alpha == 0.0) { X[l3_index(layout, ldx, xi, xj)] = 0.0; continue; }
            double s = alpha * l3_stored(B, layout, ldb, xi, xj);
            for (int64_t u = 0; u < t; ++u) {
                const int64_t c = s_lower ? u : k - 1 - u;
                /* S[r, c] = op(T)[r, c] (left) or op(T)[c, r] (right) */
                double tv;
                if (left) trmm_op(A, layout, lda, uplo, transA, diag, r, c, &tv);
                else trmm_op(A, layout, lda, uplo, transA, diag, c, r, &tv);
                const int64_t ci = left ? c : v, cj = left ? v : c;
                s = s - tv * X[l3_index(layout, ldx, ci, cj)];
            }
            if (!l3_unit(diag)) {
                double dv;
                trmm_op(A, layout, lda, uplo, transA, diag, r, r, &dv);
                s = s / dv;
            }
            X[l3_index(layout, ldx, xi, xj)] = s;
        }
    }
}
