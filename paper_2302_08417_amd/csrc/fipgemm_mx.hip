// Mixed-precision fused-pack GEMM (gfx950): dispatch over the forms and tiles,
// the alpha = 0 / k = 0 scaling and FP8 E4M3 quantization.  The kernels and
// the launch template are in fip_mx_impl.h; the E4M3 256 x 256 tile is
// instantiated in fipgemm_mx_fp8big.hip.
#include "fip_mx_impl.h"

namespace fip {
namespace {

// C := beta*C for the alpha = 0 / k = 0 quick path.
__global__ void __launch_bounds__(256) scale_mx_kernel(char* C, int c_bf16, int64_t M, int64_t N,
                                                       int64_t ldc, float beta)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % M, j = idx / M;
        if (c_bf16) {
            uint16_t* p = reinterpret_cast<uint16_t*>(C) + i + j * ldc;
            *p = beta == 0.f ? (uint16_t)0 : (uint16_t)bf16_bits(beta * bf16_float(*p));
        } else {
            float* p = reinterpret_cast<float*>(C) + i + j * ldc;
            *p = beta == 0.f ? 0.f : beta * *p;
        }
    }
}

// ---- FP8 E4M3 quantization ---------------------------------------------------
// E4M3 code of a binary32 (OCP "FN": bias 7, no infinities, 0x7F NaN, largest
// finite 448): round to nearest even on the bit pattern, saturating at 448.
__device__ __forceinline__ uint32_t e4m3_code(float v)
{
    const uint32_t u = __float_as_uint(v);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return 0x7Fu;                    // NaN
    if (a > 0x43E00000u) return sign | 0x7Eu;             // |v| > 448: saturate
    const int e = (int)(a >> 23) - 127;
    if (e >= -6) {
        // normal range: keep 3 fraction bits, ties to even; a carry moves into
        // the exponent field by itself
        const uint32_t r = (a + 0x7FFFFu + ((a >> 20) & 1u)) >> 20;
        uint32_t code = r - ((127u - 7u) << 3);
        if (code > 0x7Eu) code = 0x7Eu;
        return sign | code;
    }
    // below 2^-6: multiples of 2^-9 (code m = value / 2^-9, m = 8 is 2^-6)
    if (a < 0x00800000u) return sign;                     // binary32 subnormal: rounds to 0
    const uint32_t mant = (a & 0x7FFFFFu) | 0x800000u;    // value = mant * 2^(e - 23)
    const int sh = 14 - e;                                // value / 2^-9 = mant >> sh
    if (sh > 24) return sign;                             // below 2^-10 ... actually < half unit
    uint32_t m = mant >> sh;
    const uint32_t rem = mant & ((1u << sh) - 1u), half = 1u << (sh - 1);
    if (rem > half || (rem == half && (m & 1u))) ++m;
    return sign | m;
}

// Exponent e of the line scale 2^e: the largest e with amax * 2^e <= 448
// (448 = 0.875 * 2^9); 0 when amax is 0, not finite; clamped to [-126, 126].
__device__ __forceinline__ int fp8_scale_exp(float amax)
{
    if (!(amax > 0.f) || !(amax < __builtin_huge_valf())) return 0;
    int E;
    const float f = frexpf(amax, &E);   // amax = f * 2^E, f in [0.5, 1)
    int e = (f <= 0.875f ? 9 : 8) - E;
    return e < -126 ? -126 : e > 126 ? 126 : e;
}

// Pass 1: zero the per-line maxima (bit patterns of |x|, stored in scales).
__global__ void __launch_bounds__(256) fp8_zero_kernel(uint32_t* amax, int64_t lines)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < lines; i += (int64_t)gridDim.x * 256)
        amax[i] = 0u;
}

// Pass 2: per-line max of |x| by atomic max on the bit pattern (monotone for
// non-negative binary32); NaNs are skipped.  Threads walk the stored matrix in
// storage order (coalesced).
__global__ void __launch_bounds__(256) fp8_amax_kernel(int col, int64_t rows, int64_t cols,
                                                       const float* X, int64_t ld, int axis,
                                                       uint32_t* amax)
{
    const int64_t inner = col ? rows : cols, outer = col ? cols : rows;
    const int64_t total = inner * outer;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t in = idx % inner, out = idx / inner;
        const int64_t r = col ? in : out, c = col ? out : in;
        const uint32_t a = __float_as_uint(X[in + out * ld]) & 0x7FFFFFFFu;
        if (a > 0x7F800000u || a == 0u) continue;
        atomicMax(amax + (axis == 0 ? r : c), a);
    }
}

// Pass 3: quantize every element with its line's scale.
__global__ void __launch_bounds__(256) fp8_quant_kernel(int col, int64_t rows, int64_t cols,
                                                        const float* X, int64_t ld, int axis,
                                                        const uint32_t* amax, uint8_t* Q,
                                                        int64_t ldq)
{
    const int64_t inner = col ? rows : cols, outer = col ? cols : rows;
    const int64_t total = inner * outer;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t in = idx % inner, out = idx / inner;
        const int64_t r = col ? in : out, c = col ? out : in;
        const int e = fp8_scale_exp(__uint_as_float(amax[axis == 0 ? r : c]));
        Q[in + out * ldq] = (uint8_t)e4m3_code(ldexpf(X[in + out * ld], e));
    }
}

// Pass 4: turn each line's maximum into its scale 2^e, in place.
__global__ void __launch_bounds__(256) fp8_scale_kernel(uint32_t* amax_scale, int64_t lines)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < lines; i += (int64_t)gridDim.x * 256) {
        const int e = fp8_scale_exp(__uint_as_float(amax_scale[i]));
        amax_scale[i] = __float_as_uint(ldexpf(1.f, e));
    }
}

hipError_t dispatch_mx(const MxLaunchDesc& d, bool pack)
{
    const bool big = d.mt == 256;
    switch (d.form) {
    case kMxBF16: return big ? launch_form<kMxBF16, 256>(d, pack) : launch_form<kMxBF16, 128>(d, pack);
    case kMxFP8: return big ? launch_mx_fp8_big(d, pack) : launch_form<kMxFP8, 128>(d, pack);
    case kMxX3: return launch_form<kMxX3, 128>(d, pack);
    case kMxX3Fast: return launch_form<kMxX3Fast, 128>(d, pack);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_gemm_mx(const MxLaunchDesc& d)
{
    clear_stale_error();
    return dispatch_mx(d, false);
}

hipError_t launch_pack_mx(const MxLaunchDesc& d)
{
    clear_stale_error();
    return dispatch_mx(d, true);
}

hipError_t launch_scale_mx(int c_bf16, int64_t M, int64_t N, void* C, int64_t ldc, float beta,
                           hipStream_t stream)
{
    clear_stale_error();
    scale_mx_kernel<<<dim3(grid_for(M * N)), dim3(256), 0, stream>>>(static_cast<char*>(C), c_bf16,
                                                                      M, N, ldc, beta);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(int layout_col, int64_t rows, int64_t cols, const float* X,
                               int64_t ldx, int axis, uint8_t* Q, int64_t ldq, float* scales,
                               hipStream_t stream)
{
    clear_stale_error();
    const int64_t lines = axis == 0 ? rows : cols;
    uint32_t* amax = reinterpret_cast<uint32_t*>(scales);
    fp8_zero_kernel<<<dim3(grid_for(lines)), dim3(256), 0, stream>>>(amax, lines);
    fp8_amax_kernel<<<dim3(grid_for(rows * cols)), dim3(256), 0, stream>>>(layout_col, rows, cols,
                                                                           X, ldx, axis, amax);
    fp8_quant_kernel<<<dim3(grid_for(rows * cols)), dim3(256), 0, stream>>>(
        layout_col, rows, cols, X, ldx, axis, amax, Q, ldq);
    fp8_scale_kernel<<<dim3(grid_for(lines)), dim3(256), 0, stream>>>(amax, lines);
    return hipGetLastError();
}

}  // namespace fip
