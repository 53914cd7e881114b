/*
 * TEST INFRASTRUCTURE ONLY -- the oracle.
 *
 * A plain, slow, obviously correct CPU reference for what the fused-pack GEMM
 * library computes.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file's shared object.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes (all arithmetic in IEEE binary64):
 *
 *   Cref[i,j] = alpha * sum_{p=0}^{k-1} opA[i,p] * opB[p,j]  +  beta * C0[i,j]
 *
 * Paper, Sec. 2.1: the prototypical product is C := A B + C with A m x k,
 * B k x n, C m x n (the alpha = beta = 1, no-transpose case).  alpha, beta,
 * op() in {N, T, C} and row/column-major storage follow the BLAS gemm
 * statement the paper targets (Sec. 1).  The paper's method (Sec. 3) changes
 * only where operands live (packed vs unpacked memory, Sec. 2.1), never the
 * value being computed, so this plain definition is the reference.
 *
 * Conventions taken where the paper is silent (BLAS semantics):
 *   - alpha == 0: A and B are not read.  beta == 0: C0 is not read.
 *   - 'C' (conjugate transpose) equals 'T' for real data.
 *   - The sum over p runs in ascending p, each entry sequentially.
 *
 * The per-entry bound
 *   D[i,j] = |alpha| * sum_p |opA[i,p]| * |opB[p,j]|  +  |beta| * |C0[i,j]|
 * is computed in the same loop; it scales the tolerance of every comparison.
 *
 * Packing (Sec. 2.1, Fig. "pack2fit"; fringe padding Sec. 2.2): the reference
 * pack copies op(X) element bits into contiguous micropanels, zero-padding
 * fringes.  The contiguous layout (one block per (tile, k-step), k-major with
 * the tile's MN extent contiguous) is this library's contract; the paper fixes
 * only "contiguous micropanels, m_R values per k, zero padded".
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_COL 0
#define OR_ROW 1

/* Stored element (r, c) of a matrix with leading dimension ld. */
static double stored_at(const double* X, int layout, int64_t ld, int64_t r, int64_t c)
{
    return layout == OR_COL ? X[r + c * ld] : X[r * ld + c];
}

static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

/* op(X)[r, c]: for 'N' the stored (r, c); for 'T'/'C' the stored (c, r). */
static double op_at(const double* X, int layout, int64_t ld, char t, int64_t r, int64_t c)
{
    return is_trans(t) ? stored_at(X, layout, ld, c, r) : stored_at(X, layout, ld, r, c);
}

static int64_t c_index(int layout, int64_t ldc, int64_t i, int64_t j)
{
    return layout == OR_COL ? i + j * ldc : i * ldc + j;
}

/* Threads the OpenMP loops below will use. */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Materialise op(X) (rows x cols) as a dense column-major binary64 array. */
void oracle_materialize_op(int layout, char trans, int64_t rows, int64_t cols,
                           const double* X, int64_t ld, double* out)
{
    for (int64_t c = 0; c < cols; ++c)
        for (int64_t r = 0; r < rows; ++r)
            out[r + c * rows] = op_at(X, layout, ld, trans, r, c);
}

/*
 * Full GEMM reference.  Cref and D use C's own storage (layout, ldc); only the
 * m x n entries are written, so the caller pre-fills Cref (e.g. with C0) and
 * can check that padding is left alone.  Loop order j -> p -> i over a
 * column-major copy of op(A): i is innermost, so each entry's sum is still
 * taken sequentially in ascending p.  Parallel over columns j (independent).
 * Returns 0, or -1 when scratch allocation fails.
 */
int oracle_gemm(int layout, int64_t m, int64_t n, int64_t k, double alpha,
                const double* A, int64_t lda, char transA,
                const double* B, int64_t ldb, char transB,
                double beta, const double* C0, int64_t ldc,
                double* Cref, double* D)
{
    if (m <= 0 || n <= 0) return 0;
    const int use_ab = (alpha != 0.0) && k > 0;
    double* opA = NULL;
    if (use_ab) {
        opA = (double*)malloc(sizeof(double) * (size_t)m * (size_t)k);
        if (!opA) return -1;
        oracle_materialize_op(layout, transA, m, k, A, lda, opA);
    }
    int failed = 0;
#pragma omp parallel
    {
        double* s = (double*)malloc(sizeof(double) * (size_t)m);
        double* d = (double*)malloc(sizeof(double) * (size_t)m);
        double* bcol = use_ab ? (double*)malloc(sizeof(double) * (size_t)k) : NULL;
        if (!s || !d || (use_ab && !bcol)) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t j = 0; j < n; ++j) {
                for (int64_t i = 0; i < m; ++i) { s[i] = 0.0; d[i] = 0.0; }
                if (use_ab) {
                    for (int64_t p = 0; p < k; ++p) bcol[p] = op_at(B, layout, ldb, transB, p, j);
                    for (int64_t p = 0; p < k; ++p) {
                        const double b = bcol[p];
                        const double ab = fabs(b);
                        const double* a = opA + p * m;
                        for (int64_t i = 0; i < m; ++i) {
                            s[i] = s[i] + a[i] * b;
                            d[i] = d[i] + fabs(a[i]) * ab;
                        }
                    }
                }
                for (int64_t i = 0; i < m; ++i) {
                    const int64_t ci = c_index(layout, ldc, i, j);
                    double c = use_ab ? alpha * s[i] : 0.0;
                    double dd = use_ab ? fabs(alpha) * d[i] : 0.0;
                    if (beta != 0.0) {
                        c = c + beta * C0[ci];
                        dd = dd + fabs(beta) * fabs(C0[ci]);
                    }
                    Cref[ci] = c;
                    D[ci] = dd;
                }
            }
        }
        free(s); free(d); free(bcol);
    }
    free(opA);
    return failed ? -1 : 0;
}

/*
 * The same definition on a list of entries (i_t, j_t), for sizes where the
 * full triple loop is too slow.  Same ascending-p order per entry, so each
 * value equals the corresponding entry of oracle_gemm bit for bit.
 */
void oracle_gemm_entries(int layout, int64_t m, int64_t n, int64_t k, double alpha,
                         const double* A, int64_t lda, char transA,
                         const double* B, int64_t ldb, char transB,
                         double beta, const double* C0, int64_t ldc,
                         int64_t count, const int64_t* rows, const int64_t* cols,
                         double* cref_out, double* d_out)
{
    (void)m; (void)n;
    const int use_ab = (alpha != 0.0) && k > 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        double s = 0.0, d = 0.0;
        if (use_ab) {
            for (int64_t p = 0; p < k; ++p) {
                const double a = op_at(A, layout, lda, transA, i, p);
                const double b = op_at(B, layout, ldb, transB, p, j);
                s = s + a * b;
                d = d + fabs(a) * fabs(b);
            }
        }
        double c = use_ab ? alpha * s : 0.0;
        double dd = use_ab ? fabs(alpha) * d : 0.0;
        if (beta != 0.0) {
            const double c0 = C0[c_index(layout, ldc, i, j)];
            c = c + beta * c0;
            dd = dd + fabs(beta) * fabs(c0);
        }
        cref_out[t] = c;
        d_out[t] = dd;
    }
}

/*
 * Freivalds probe of the whole product: for a vector x (length n),
 *   y     = alpha * opA (opB x) + beta * C0 x
 *   bound = |alpha| |opA| (|opB| |x|) + |beta| |C0| |x|
 * in O(mk + kn + mn) operations.  A result C satisfies the GEMM tolerance
 * entry-wise only if |C x - y| <= tol * bound row by row (plus the probe's own
 * rounding), so this checks every entry of C in aggregate.
 */
int oracle_freivalds(int layout, int64_t m, int64_t n, int64_t k, double alpha,
                     const double* A, int64_t lda, char transA,
                     const double* B, int64_t ldb, char transB,
                     double beta, const double* C0, int64_t ldc,
                     const double* x, double* y, double* bound)
{
    const int use_ab = (alpha != 0.0) && k > 0;
    double* t = NULL; double* ta = NULL;
    if (use_ab) {
        t = (double*)calloc((size_t)k, sizeof(double));
        ta = (double*)calloc((size_t)k, sizeof(double));
        if (!t || !ta) { free(t); free(ta); return -1; }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < k; ++p) {
            double s = 0.0, sa = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const double b = op_at(B, layout, ldb, transB, p, j);
                s = s + b * x[j];
                sa = sa + fabs(b) * fabs(x[j]);
            }
            t[p] = s; ta[p] = sa;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0, sa = 0.0;
        if (use_ab) {
            for (int64_t p = 0; p < k; ++p) {
                const double a = op_at(A, layout, lda, transA, i, p);
                s = s + a * t[p];
                sa = sa + fabs(a) * ta[p];
            }
        }
        double yi = use_ab ? alpha * s : 0.0;
        double bi = use_ab ? fabs(alpha) * sa : 0.0;
        if (beta != 0.0) {
            double cs = 0.0, ca = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const double c0 = C0[c_index(layout, ldc, i, j)];
                cs = cs + c0 * x[j];
                ca = ca + fabs(c0) * fabs(x[j]);
            }
            yi = yi + beta * cs;
            bi = bi + fabs(beta) * ca;
        }
        y[i] = yi;
        bound[i] = bi;
    }
    free(t); free(ta);
    return 0;
}

/*
 * Which index of op(X) is contiguous in X's storage.  op(X)[r, c] is stored
 * element (r, c) for 'N' and (c, r) for 'T'/'C'; a column-major matrix is
 * contiguous along its row index, a row-major one along its column index.
 * For op(A) (m x k) the MN index is the row index r; for op(B) (k x n) it is
 * the column index c.  Returns 1 when storage runs along the MN index.
 */
int oracle_mn_contiguous(int is_b, int layout, char trans)
{
    /* index of op(X) (0 = row r, 1 = column c) that runs along storage:
       column-major N -> r, column-major T -> c, row-major N -> c, row-major T -> r */
    const int contiguous_index = (layout == OR_ROW) ^ is_trans(trans);
    const int mn_index = is_b ? 1 : 0; /* op(A): rows are M; op(B): columns are N */
    return contiguous_index == mn_index;
}

/*
 * Reference pack (a bit copy).  X holds elements of elem_size bytes; the
 * operand is op(X) with extent mn along its M (for A) or N (for B) index and
 * k along the contraction index.  is_b selects which index of op(X) is the
 * contraction index: op(A) is mn x k (contraction = column), op(B) is k x mn
 * (contraction = row).  The packed buffer holds ceil(mn/MNT) * ceil(k/KT)
 * contiguous blocks of KT * MNT elements, block (t, q) at position
 * t * ceil(k/KT) + q.  Inside a block the tile keeps the orientation op(X) has
 * in storage: if storage runs along the MN index, element (x, p) sits at
 * (p % KT) * MNT + (x % MNT) (each k-slice contiguous); otherwise at
 * (x % MNT) * KT + (p % KT) (each MN-row's k-run contiguous).  Entries outside
 * op(X) are all-zero bytes.  Element bits are copied untouched (NaN payloads,
 * -0.0, subnormals).
 */
/* The pack with an explicit block orientation: kmajor = 1 stores each block
   K-major ((i % MNT)*KT + p % KT), 0 MN-major ((p % KT)*MNT + i % MNT), -1
   follows the operand's storage (the FP64/FP32 contract).  The mixed-precision
   forms always pack K-major. */
void oracle_pack_oriented(int elem_size, int is_b, int layout, char trans, int64_t mn, int64_t k,
                          const void* X, int64_t ld, int64_t MNT, int64_t KT, int kmajor,
                          void* out)
{
    const unsigned char* src = (const unsigned char*)X;
    unsigned char* dst = (unsigned char*)out;
    const int64_t nt = (mn + MNT - 1) / MNT, nk = (k + KT - 1) / KT;
    const int tr = is_trans(trans);
    const int mn_major = kmajor < 0 ? oracle_mn_contiguous(is_b, layout, trans) : !kmajor;
    for (int64_t t = 0; t < nt; ++t)
        for (int64_t q = 0; q < nk; ++q)
            for (int64_t pp = 0; pp < KT; ++pp)
                for (int64_t xx = 0; xx < MNT; ++xx) {
                    const int64_t x = t * MNT + xx, p = q * KT + pp;
                    const int64_t inner = mn_major ? pp * MNT + xx : xx * KT + pp;
                    unsigned char* d = dst + ((t * nk + q) * KT * MNT + inner) * elem_size;
                    if (x >= mn || p >= k) { memset(d, 0, (size_t)elem_size); continue; }
                    /* op(X)[r, c] with (r, c) = (x, p) for A, (p, x) for B */
                    const int64_t r = is_b ? p : x, c = is_b ? x : p;
                    const int64_t sr = tr ? c : r, sc = tr ? r : c; /* stored indices */
                    const int64_t off = layout == OR_COL ? sr + sc * ld : sr * ld + sc;
                    memcpy(d, src + off * elem_size, (size_t)elem_size);
                }
}

void oracle_pack(int elem_size, int is_b, int layout, char trans, int64_t mn, int64_t k,
                 const void* X, int64_t ld, int64_t MNT, int64_t KT, void* out)
{
    oracle_pack_oriented(elem_size, is_b, layout, trans, mn, k, X, ld, MNT, KT, -1, out);
}
