// Diagonal-block solve of the blocked triangular solve (TRSM) for gfx950.
//
// The library solves op(T) X = alpha B (or X op(T) = alpha B) by recursive
// blocking: the off-diagonal updates are GEMMs run by the fused-pack tile
// kernel (paper Sec. 2.2: BLIS casts the level-3 operations onto one packing
// and microkernel layer; Sec. 5: fused packing for them), and what remains
// are solves with diagonal blocks of at most kTrsmBlock rows, done here.
//
// One thread per right-hand side: a column of B (side L) or a row (side R).
// The block's triangle S (NB x NB, S = op(T) for side L, op(T)^T for side R)
// sits in LDS; each thread substitutes through it with its unknowns in
// registers (fully unrolled, so every index is a constant), in place in B:
//   x_r = (alpha b_r - sum_c S[r, c] x_c) / S[r, r]
// over the already solved c (ascending for lower S, descending for upper S);
// no division for a unit diagonal.  Only the referenced triangle of the stored
// matrix is read (and not the diagonal when it is unit).  A block of nb < NB
// rows is padded with identity rows and zero right-hand sides, which solve to
// zeros and are not stored.
#include "fip_internal.h"

namespace fip {
namespace {

template <typename T, int NB, bool LOWER>
__global__ void __launch_bounds__(64) trsm_block_kernel(const T* __restrict__ A, int64_t lda,
                                                        int s_trans, int unit, int nb, T* B,
                                                        int64_t s_e, int64_t s_v, int64_t nrhs,
                                                        T alpha)
{
    __shared__ T S[NB][NB + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < NB * NB; idx += 64) {
        const int r = idx / NB, c = idx - r * NB;
        const bool in_tri = LOWER ? c <= r : c >= r;
        T v = T(0);
        if (r < nb && c < nb && in_tri) {
            if (r == c) v = unit ? T(1) : (s_trans ? A[c + (int64_t)r * lda] : A[r + (int64_t)c * lda]);
            else v = s_trans ? A[c + (int64_t)r * lda] : A[r + (int64_t)c * lda];
        } else if (r == c) {
            v = T(1);   // padding rows: identity
        }
        S[r][c] = v;
    }
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 64 + tid;
    if (v >= nrhs) return;
    T* b = B + v * s_v;
    // The sum of row r is split over four accumulators (terms c = 0, 1, 2, 3
    // mod 4 of the solved unknowns, in solve order), so four independent
    // chains of LDS reads and FMAs are in flight instead of one.
    T x[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int r = LOWER ? t : NB - 1 - t;
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int u = 0; u < t; ++u) {
            const int c = LOWER ? u : NB - 1 - u;
            acc[u & 3] = acc[u & 3] + S[r][c] * x[c];
        }
        const T s = (r < nb ? alpha * b[r * s_e] : T(0)) - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        x[r] = unit ? s : s / S[r][r];
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
        if (r < nb) b[r * s_e] = x[r];
}

template <typename T>
hipError_t launch_t(const TrsmBlockDesc& d)
{
    const dim3 grid((unsigned)((d.nrhs + 63) / 64)), block(64);
    const T* A = static_cast<const T*>(d.A);
    T* B = static_cast<T*>(d.B);
    if (d.s_lower)
        trsm_block_kernel<T, kTrsmBlock, true><<<grid, block, 0, d.stream>>>(
            A, d.lda, d.s_trans, d.unit, d.nb, B, d.s_e, d.s_v, d.nrhs, (T)d.alpha);
    else
        trsm_block_kernel<T, kTrsmBlock, false><<<grid, block, 0, d.stream>>>(
            A, d.lda, d.s_trans, d.unit, d.nb, B, d.s_e, d.s_v, d.nrhs, (T)d.alpha);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_trsm_block(const TrsmBlockDesc& d)
{
    clear_stale_error();
    if (d.nrhs <= 0 || d.nb <= 0) return hipSuccess;
    return d.elem == 8 ? launch_t<double>(d) : launch_t<float>(d);
}

}  // namespace fip
