/*
 * TEST INFRASTRUCTURE ONLY -- the oracle of the complex GEMM.
 *
 * A plain, slow reference for the complex-domain product the library runs
 * through its real-domain fused-pack tile kernel by the 1m method.  The paper
 * points to the 1m method as an example of a transformation carried out by
 * the packing stage (Sec. 5): the definition of complex multiplication is
 * encoded in how the operands are packed, and the real microkernel does the
 * rest.  What is computed is the BLAS zgemm/cgemm definition, written out
 * here in binary64 complex arithmetic on (re, im) pairs; the 1m expansion is
 * written out separately so that the tests can check the packed operands.
 * Only the test suite may load this file's shared object; it shares no code
 * with the GPU library.
 *
 * Storage: element (r, c) of a complex matrix with leading dimension ld is the
 * pair X[2q], X[2q + 1] (re, im) with q = r + c*ld (column-major) or r*ld + c
 * (row-major).
 *
 *   Cref[i,j] = alpha * sum_{p=0}^{k-1} opA[i,p] * opB[p,j] + beta * C0[i,j]
 *
 * op(X) is X ('N'), X^T ('T') or the conjugate transpose X^H ('C').  Each
 * complex product a*b is (ar*br - ai*bi, ar*bi + ai*br) and the sum runs in
 * ascending p, each component sequentially.  alpha == 0 (or k == 0): A and B
 * are not read; beta == 0: C0 is not read.  Complex scalars multiply the same
 * way: alpha*s = (alr*sr - ali*si, alr*si + ali*sr).
 *
 * Bound: D[i,j] = |alpha|_1 * sum_p |opA[i,p]|_1 |opB[p,j]|_1 + |beta|_1 |C0[i,j]|_1
 * with |z|_1 = |re| + |im|.  Each real component of the sum is a sum of 2k
 * real products whose absolute values add up to at most this, so D bounds the
 * rounding error of either component in the usual way (gamma_{2k} D, plus the
 * epilogue's few roundings).
 *
 * 1m expansion (the formats of the 1m method): with z = opA[i,p], the real
 * 2m x 2k matrix A1e holds the 2 x 2 block [[re z, -im z], [im z, re z]] at
 * rows 2i, 2i+1 and columns 2p, 2p+1; with w = opB[p,j], the real 2k x n
 * matrix B1r holds re w, im w at rows 2p, 2p+1 of column j.  Then the real
 * product A1e * B1r holds re and im of opA*opB at rows 2i, 2i+1: the real view
 * of a column-major complex C.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define CX_COL 0

static int cx_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static int cx_conj(char t) { return t == 'C' || t == 'c'; }

/* op(X)[r, c] as (re, im). */
static void cx_op(const double* X, int layout, int64_t ld, char t, int64_t r, int64_t c,
                  double* re, double* im)
{
    const int64_t sr = cx_trans(t) ? c : r, sc = cx_trans(t) ? r : c;
    const int64_t q = layout == CX_COL ? sr + sc * ld : sr * ld + sc;
    *re = X[2 * q];
    *im = cx_conj(t) ? -X[2 * q + 1] : X[2 * q + 1];
}

static int64_t cx_cindex(int layout, int64_t ldc, int64_t i, int64_t j)
{
    return layout == CX_COL ? i + j * ldc : i * ldc + j;
}

/* One entry: alpha * sum_p opA[i,p] opB[p,j] + beta * C0[i,j] and its bound. */
static void cx_entry(int layout, int64_t k, double alr, double ali, const double* A, int64_t lda,
                     char tA, const double* B, int64_t ldb, char tB, double ber, double bei,
                     const double* C0, int64_t ldc, int64_t i, int64_t j, double* out, double* d)
{
    const int use_ab = (alr != 0.0 || ali != 0.0) && k > 0;
    double sr = 0.0, si = 0.0, sd = 0.0;
    if (use_ab) {
        for (int64_t p = 0; p < k; ++p) {
            double ar, ai, br, bi;
            cx_op(A, layout, lda, tA, i, p, &ar, &ai);
            cx_op(B, layout, ldb, tB, p, j, &br, &bi);
            const double tr = ar * br - ai * bi;
            const double ti = ar * bi + ai * br;
            sr = sr + tr;
            si = si + ti;
            sd = sd + (fabs(ar) + fabs(ai)) * (fabs(br) + fabs(bi));
        }
    }
    double cr = 0.0, ci = 0.0, dd = 0.0;
    if (use_ab) {
        cr = alr * sr - ali * si;
        ci = alr * si + ali * sr;
        dd = (fabs(alr) + fabs(ali)) * sd;
    }
    if (ber != 0.0 || bei != 0.0) {
        const int64_t q = cx_cindex(layout, ldc, i, j);
        const double c0r = C0[2 * q], c0i = C0[2 * q + 1];
        cr = cr + (ber * c0r - bei * c0i);
        ci = ci + (ber * c0i + bei * c0r);
        dd = dd + (fabs(ber) + fabs(bei)) * (fabs(c0r) + fabs(c0i));
    }
    out[0] = cr;
    out[1] = ci;
    *d = dd;
}

/*
 * Full complex GEMM reference.  Cref (pairs) and D (one bound per complex
 * entry) use C's storage (layout, ldc); only the m x n entries are written.
 * Parallel over columns j.
 */
void oracle_zgemm(int layout, int64_t m, int64_t n, int64_t k, double alr, double ali,
                  const double* A, int64_t lda, char transA, const double* B, int64_t ldb,
                  char transB, double ber, double bei, const double* C0, int64_t ldc,
                  double* Cref, double* D)
{
    if (m <= 0 || n <= 0) return;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            const int64_t q = cx_cindex(layout, ldc, i, j);
            cx_entry(layout, k, alr, ali, A, lda, transA, B, ldb, transB, ber, bei, C0, ldc, i, j,
                     Cref + 2 * q, D + q);
        }
}

/* The same definition on a list of entries (rows[t], cols[t]): out holds
   pairs, d one bound per entry; equal bit for bit to oracle_zgemm's. */
void oracle_zgemm_entries(int layout, int64_t k, double alr, double ali, const double* A,
                          int64_t lda, char transA, const double* B, int64_t ldb, char transB,
                          double ber, double bei, const double* C0, int64_t ldc, int64_t count,
                          const int64_t* rows, const int64_t* cols, double* out, double* d)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t)
        cx_entry(layout, k, alr, ali, A, lda, transA, B, ldb, transB, ber, bei, C0, ldc, rows[t],
                 cols[t], out + 2 * t, d + t);
}

/*
 * The 1m expansion of op(X) as a dense column-major real matrix.
 *   is_b = 0: op(X) is m x k (m = mn); out is A1e, 2mn x 2k.
 *   is_b = 1: op(X) is k x n (n = mn); out is B1r, 2k x mn.
 */
void oracle_expand_1m(int is_b, int layout, char trans, int64_t mn, int64_t k, const double* X,
                      int64_t ld, double* out)
{
    if (!is_b) {
        const int64_t rows = 2 * mn;
        for (int64_t p = 0; p < k; ++p)
            for (int64_t i = 0; i < mn; ++i) {
                double re, im;
                cx_op(X, layout, ld, trans, i, p, &re, &im);
                out[(2 * i) + (2 * p) * rows] = re;
                out[(2 * i + 1) + (2 * p) * rows] = im;
                out[(2 * i) + (2 * p + 1) * rows] = -im;
                out[(2 * i + 1) + (2 * p + 1) * rows] = re;
            }
    } else {
        const int64_t rows = 2 * k;
        for (int64_t j = 0; j < mn; ++j)
            for (int64_t p = 0; p < k; ++p) {
                double re, im;
                cx_op(X, layout, ld, trans, p, j, &re, &im);
                out[(2 * p) + j * rows] = re;
                out[(2 * p + 1) + j * rows] = im;
            }
    }
}
