// Diagonal-block solve of the blocked triangular solve (TRSM) for gfx950.
//
// The library solves op(T) X = alpha B (or X op(T) = alpha B) by recursive
// blocking: the off-diagonal updates are GEMMs run by the fused-pack tile
// kernel (paper Sec. 2.2: BLIS casts the level-3 operations onto one packing
// and microkernel layer; Sec. 5: fused packing for them), and what remains
// are solves with diagonal blocks of at most kTrsmBlock rows, done here.
//
// Sixteen lanes per right-hand side (a column of B for side L, a row for
// side R), 16 right-hand sides per 256-thread workgroup, so that a few
// thousand right-hand sides give every SIMD a wave or two (TRSM measured
// 2-4 % faster than with eight lanes).  The block's triangle S
// (NB x NB, S = op(T) for side L, op(T)^T for side R) sits in LDS with zeros
// outside the triangle.  Lane q of a group owns rows r = q + 16i: it holds
// their b and, once solved, their x (zero before), and for every row r forms
// the partial sum over its columns c = q + 16i of S[r, c] x_c, minus alpha
// b_r on the lane that owns r; four DPP steps add the sixteen partials
// (every lane ends with the same bits, the additions commute), and
//   x_r = (alpha b_r - sum_c S[r, c] x_c) * (1 / S[r, r])
// over the already solved c (ascending r for lower S, descending for upper
// S), with the reciprocals of the diagonal formed once per block, as BLIS
// packs them for its TRSM microkernel, so no division sits on the chain from
// one unknown to the next; nothing for a unit diagonal.  Unsolved x_c are zero and so are the
// entries of S outside the triangle, so terms that fall outside add exact
// zeros.  Only the referenced triangle of the stored matrix is read (and not
// the diagonal when it is unit).  A block of nb < NB rows is padded with
// identity rows and zero right-hand sides, which solve to zeros and are not
// stored.
#include "fip_internal.h"

namespace fip {
namespace {

constexpr int kLanes = 16;      // lanes per right-hand side
constexpr int kThreads = 256;

// DPP moves within a row of sixteen lanes: quad_perm [1,0,3,2] (lane ^ 1),
// quad_perm [2,3,0,1] (lane ^ 2), row_half_mirror (lane 7 - l of each eight)
// and row_ror:8 (the other half of the row).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <typename T, int NB, bool LOWER, bool UNIT>
__global__ void __launch_bounds__(kThreads) trsm_block_kernel(const T* __restrict__ A, int64_t lda,
                                                              int s_trans, int nb, T* B,
                                                              int64_t s_e, int64_t s_v,
                                                              int64_t nrhs, T alpha)
{
    constexpr int NI = NB / kLanes;     // rows owned per lane
    static_assert(NB % kLanes == 0, "rows split evenly over the lanes");
    __shared__ T S[NB][NB + 1];
    __shared__ T Dinv[NB];   // 1 / S[r, r]
    const int tid = threadIdx.x;
    for (int idx = tid; idx < NB * NB; idx += kThreads) {
        // consecutive threads walk contiguous memory of A
        const int u = idx % NB, w = idx / NB;
        const int r = s_trans ? w : u, c = s_trans ? u : w;
        const bool in_tri = LOWER ? c <= r : c >= r;
        T v = T(0);
        if (r < nb && c < nb && in_tri) {
            if (r == c) v = UNIT ? T(1) : (s_trans ? A[c + (int64_t)r * lda] : A[r + (int64_t)c * lda]);
            else v = s_trans ? A[c + (int64_t)r * lda] : A[r + (int64_t)c * lda];
        } else if (r == c) {
            v = T(1);   // padding rows: identity
        }
        S[r][c] = v;
        if (r == c) Dinv[r] = T(1) / v;
    }
    __syncthreads();
    // a group of sixteen lanes shares its right-hand side, so a group is live
    // or returns as a whole and the DPP moves only read live lanes
    const int q = tid & (kLanes - 1);
    const int64_t v = (int64_t)blockIdx.x * (kThreads / kLanes) + tid / kLanes;
    if (v >= nrhs) return;
    T* b = B + v * s_v;
    T bq[NI], xq[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int r = q + kLanes * i;
        bq[i] = r < nb ? alpha * b[r * s_e] : T(0);
        xq[i] = T(0);
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int r = LOWER ? t : NB - 1 - t;
        const int own = r / kLanes;
        T acc = q == (r & (kLanes - 1)) ? -bq[own] : T(0);
        // columns q + 16i that can precede r in the solve order, the most
        // recently solved last
        if constexpr (LOWER) {
#pragma unroll
            for (int i = 0; i <= own; ++i) acc = acc + S[r][q + kLanes * i] * xq[i];
        } else {
#pragma unroll
            for (int i = NI - 1; i >= own; --i) acc = acc + S[r][q + kLanes * i] * xq[i];
        }
        acc = acc + dpp<kDppXor1>(acc);
        acc = acc + dpp<kDppXor2>(acc);
        acc = acc + dpp<kDppHalfMirror>(acc);
        acc = acc + dpp<kDppRor8>(acc);
        const T x = UNIT ? -acc : -acc * Dinv[r];
        if (q == (r & (kLanes - 1))) xq[own] = x;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int r = q + kLanes * i;
        if (r < nb) b[r * s_e] = xq[i];
    }
}

template <typename T>
hipError_t launch_t(const TrsmBlockDesc& d)
{
    constexpr int per_block = kThreads / kLanes;
    const dim3 grid((unsigned)((d.nrhs + per_block - 1) / per_block)), block(kThreads);
    const T* A = static_cast<const T*>(d.A);
    T* B = static_cast<T*>(d.B);
#define FIP_TRSM_LAUNCH(LO, UN)                                                               \
    trsm_block_kernel<T, kTrsmBlock, LO, UN><<<grid, block, 0, d.stream>>>(                  \
        A, d.lda, d.s_trans, d.nb, B, d.s_e, d.s_v, d.nrhs, (T)d.alpha)
    if (d.s_lower) {
        if (d.unit) FIP_TRSM_LAUNCH(true, true);
        else FIP_TRSM_LAUNCH(true, false);
    } else {
        if (d.unit) FIP_TRSM_LAUNCH(false, true);
        else FIP_TRSM_LAUNCH(false, false);
    }
#undef FIP_TRSM_LAUNCH
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
