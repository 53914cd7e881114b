// Register/LDS staging of FP64/FP32 operand chunks and the 16x16x4 MFMA, shared
// by the fused-pack tile kernel (fipgemm_kernels.hip) and the batched kernel
// (fipgemm_batched.hip).  Internal; included only by HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fip {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Types;
// vec: 16-byte vector (16-byte aligned); uvec: the same vector with only
// element alignment, for unpacked operands whose leading dimension or base is
// not a multiple of 16 bytes (gfx950 global loads accept dword-aligned
// multi-dword accesses, so this is still one 16-byte load).
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
template <> struct Types<double> { typedef d2 vec; typedef d2u uvec; typedef d4 acc; static constexpr int VEC = 2; };
template <> struct Types<float> { typedef f4 vec; typedef f4u uvec; typedef f4 acc; static constexpr int VEC = 4; };

// One 16x16x4 MFMA on fragments a (lane l: A[i = l%16][k = l/16]) and b (lane l:
// B[k = l/16][j = l%16]) of a 16x16 C block.  Output layouts differ by type:
//   f32 (v_mfma_f32_16x16x4_f32): item r of lane l is C[4*(l/16) + r][l%16];
//   f64 (v_mfma_f64_16x16x4_f64): item r of lane l would be C[4*r + l/16][l%16].
// For f64 the operands are swapped so the instruction produces the transposed
// block: item r of lane l is then C[l%16][4*r + l/16], i.e. each lane keeps one
// row and 16 consecutive lanes cover 16 consecutive rows of a column-major C.
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS pitch of an MN-major tile ([k][mn]): the tile extent plus padding so
// that the four k-rows one MFMA fragment read touches start 16 elements apart
// modulo the 64 4-byte banks (conflict-free 16x4 fragment reads).
template <typename T, int MNT>
constexpr int lds_pitch_mn()
{
    constexpr int mod = 256 / (int)sizeof(T);
    return MNT + (((16 - MNT) % mod) + mod) % mod;
}
// LDS pitch of a K-major tile ([mn][k]): KT plus padding so that the 16 rows
// one fragment read touches land on distinct banks: a row stride of 36 banks
// (f64: KT + 2 = 18 elements, f32: KT + 4 = 36); rows stay 16-byte aligned.
// One operand chunk (MNT x KT) held in registers while it moves from HBM to
// LDS (and, for a producer, to the pack buffer).  KC: the operand is K-major
// (contiguous along k); otherwise MN-major.  The chunk keeps that orientation
// everywhere: in the unpacked operand, in LDS and in the packed copy, so no
// step transposes it.  Register vector i holds chunk elements o .. o+VEC-1,
// o = (tid + i*NTHR)*VEC, in the orientation's linear order:
//   MN-major: (x, p) = (o % MNT, o / MNT),  packed position p*MNT + x
//   K-major:  (x, p) = (o / KT, o % KT),    packed position x*KT + p
// so the packed position of register vector i is always o.
template <typename T, int MNT, int KT, int NTHR, bool KC>
struct Chunk {
    typedef typename Types<T>::vec V;
    static constexpr int VEC = Types<T>::VEC;
    static constexpr int NV = MNT * KT / (NTHR * VEC);
    static constexpr int LDP = KC ? (sizeof(T) == 8 ? KT + 2 : KT + 4) : lds_pitch_mn<T, MNT>();
    static constexpr int LDS_ELEMS = KC ? MNT * LDP : KT * LDP;
    static_assert(NV * NTHR * VEC == MNT * KT, "chunk must split evenly over the threads");
    static_assert(MNT % VEC == 0 && KT % VEC == 0, "vector width must divide the chunk");

    V r[NV];

    __device__ __forceinline__ static int elem_o(int i, int tid) { return (tid + i * NTHR) * VEC; }
    __device__ __forceinline__ static int x_of(int o) { return KC ? o / KT : o % MNT; }
    __device__ __forceinline__ static int p_of(int o) { return KC ? o % KT : o / MNT; }
    // LDS element index of chunk element (x, p)
    __device__ __forceinline__ static int lds_at(int x, int p) { return KC ? x * LDP + p : p * LDP + x; }

    // Unpacked source, interior chunk: every element exists and vector loads
    // are aligned.  Element (x, p) sits at X[x + p*ld] (MN-major) or
    // X[x*ld + p] (K-major).  The chunk origin is uniform across the
    // workgroup; each lane adds loop-invariant 32-bit byte offsets (the host
    // guarantees they fit), so loads use the scalar-base addressing form and
    // the code is straight-line with no masks.
    __device__ __forceinline__ static uint32_t fast_offset(int i, int tid, int64_t ld)
    {
        const int o = elem_o(i, tid);
        const int64_t x = x_of(o), p = p_of(o);
        return (uint32_t)((KC ? x * ld + p : x + p * ld) * (int64_t)sizeof(T));
    }
    __device__ __forceinline__ void load_at(const char* __restrict__ base, const uint32_t* off)
    {
        typedef typename Types<T>::uvec U;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const U u = *reinterpret_cast<const U*>(base + off[i]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) r[i][e] = u[e];
        }
    }
    __device__ __forceinline__ void load_fast(const T* __restrict__ origin, const uint32_t* off)
    {
        typedef typename Types<T>::uvec U;
        const char* base = reinterpret_cast<const char*>(origin);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const U u = *reinterpret_cast<const U*>(base + off[i]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) r[i][e] = u[e];
        }
    }

    // Unpacked source, fringe chunk (Sec. 2.2 zero padding done in registers):
    // elements outside the MN x K operand read as +0.0; one vector load where
    // the whole vector exists, element loads otherwise.
    __device__ __forceinline__ void load_edge(const T* __restrict__ X, int64_t ld, int64_t MN,
                                              int64_t K, int64_t x0, int64_t p0, bool vec_ok,
                                              int tid)
    {
        typedef typename Types<T>::uvec U;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = elem_o(i, tid);
            const int64_t x = x0 + x_of(o), p = p0 + p_of(o);
            if (!KC) {
                const T* src = X + x + p * ld;
                if (vec_ok && p < K && x + VEC <= MN) {
                    const U u = *reinterpret_cast<const U*>(src);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) r[i][e] = u[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) r[i][e] = (p < K && x + e < MN) ? src[e] : T(0);
                }
            } else {
                const T* src = X + x * ld + p;
                if (vec_ok && x < MN && p + VEC <= K) {
                    const U u = *reinterpret_cast<const U*>(src);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) r[i][e] = u[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) r[i][e] = (x < MN && p + e < K) ? src[e] : T(0);
                }
            }
        }
    }

    // Triangle of a TRMM operand, applied in registers: element (x, p) of the
    // chunk at (x0, p0) is kept when x >= p (keep_ge) or x <= p, else +0.0;
    // with unit, the diagonal x == p inside the MN x K operand is 1 (the zero
    // padding outside it stays +0.0).  Vector element e runs along MN
    // (MN-major) or along k (K-major).
    __device__ __forceinline__ void mask_tri(int64_t x0, int64_t p0, int keep_ge, int unit,
                                             int64_t MN, int64_t K, int tid)
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = elem_o(i, tid);
            const int64_t xb = x0 + x_of(o), pb = p0 + p_of(o);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int64_t x = xb + (KC ? 0 : e), p = pb + (KC ? e : 0);
                const bool keep = keep_ge ? x >= p : x <= p;
                T v = keep ? r[i][e] : T(0);
                if (unit && x == p && x < MN && p < K) v = T(1);
                r[i][e] = v;
            }
        }
    }

    // Packed source: one contiguous, zero-padded chunk; always vector loads.
    __device__ __forceinline__ void load_packed(const T* __restrict__ chunk, int tid)
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) r[i] = *reinterpret_cast<const V*>(chunk + elem_o(i, tid));
    }

    __device__ __forceinline__ void store_lds(T* lds, int tid) const
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = elem_o(i, tid);
            *reinterpret_cast<V*>(lds + lds_at(x_of(o), p_of(o))) = r[i];
        }
    }

    __device__ __forceinline__ void store_pack(T* __restrict__ chunk, int tid) const
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) *reinterpret_cast<V*>(chunk + elem_o(i, tid)) = r[i];
    }
};

}  // namespace
}  // namespace fip
