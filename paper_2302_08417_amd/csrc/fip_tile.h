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
    // Whether register vector i of a chunk at MN origin x0 lies inside an
    // operand of extent MN (no vector straddles the edge: K-major vectors run
    // along k, MN-major ones need MN to be a multiple of VEC).
    __device__ __forceinline__ static bool vec_inside(int i, int tid, int64_t x0, int64_t MN)
    {
        return x0 + x_of(elem_o(i, tid)) < MN;
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

    // ---- Complex operands through the 1m method ---------------------------
    // The kernel multiplies real matrices; a complex operand reaches it in the
    // expanded formats of the 1m method (the paper's Sec. 5 example of
    // arithmetic encoded in the packing).  SIDE 0 (kernel A side): real
    // element (x, p) is entry (x % 2, p % 2) of the 2 x 2 block
    // [[re, -im], [im, re]] of complex element (x/2, p/2).  SIDE 1 (kernel B
    // side): real element (x, p) is component p % 2 (re, im) of complex element
    // (p/2, x).  Complex element (r, q) (r along MN, q along k) is the pair
    // X[2(r*ld + q)] (K-major) or X[2(r + q*ld)] (MN-major), conjugated on
    // request.  A register vector then covers VEC/2 whole complex elements
    // (16 bytes) in every case but the MN-major B side, where it takes one
    // component of VEC complex elements (32 bytes).
    //
    // Byte offset of register vector i's first complex element from the
    // chunk's first one (loop-invariant per lane).
    template <int SIDE>
    __device__ __forceinline__ static uint32_t cx_offset(int i, int tid, int64_t ld)
    {
        const int o = elem_o(i, tid);
        const int64_t x = x_of(o), p = p_of(o);
        const int64_t r = SIDE == 0 ? x / 2 : x, q = p / 2;
        return (uint32_t)((KC ? r * ld + q : r + q * ld) * (int64_t)(2 * sizeof(T)));
    }
    // The parity that selects vector i's arrangement: p % 2 (the block column,
    // or the component) except on the K-major A side, where it is x % 2 (the
    // block row); unused on the K-major B side.
    template <int SIDE>
    __device__ __forceinline__ static bool cx_par(int i, int tid)
    {
        const int o = elem_o(i, tid);
        return (SIDE == 0 && KC) ? (x_of(o) & 1) : (p_of(o) & 1);
    }
    // In-place arrangement of one vector that holds VEC/2 whole complex
    // elements as loaded (every case but the MN-major B side).
    template <int SIDE>
    __device__ __forceinline__ static void cx_arrange(V& v, bool par, bool cj)
    {
        constexpr int H = VEC / 2;   // complex elements in 16 bytes
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const T re = v[2 * h], im = cj ? -v[2 * h + 1] : v[2 * h + 1];
            T a0, a1;
            if constexpr (SIDE == 1) { a0 = re; a1 = im; }                        // (re, im) along k
            else if constexpr (!KC) { a0 = par ? -im : re; a1 = par ? re : im; }  // a block column
            else { a0 = par ? im : re; a1 = par ? re : -im; }                     // a block row
            v[2 * h] = a0;
            v[2 * h + 1] = a1;
        }
    }
    // Whether a vector arranges in place (so it can be loaded raw and
    // arranged later, after the step's MFMAs, off the loads' latency).
    template <int SIDE>
    __device__ __forceinline__ static constexpr bool cx_in_place() { return !(SIDE == 1 && !KC); }
    template <int SIDE>
    __device__ __forceinline__ void cx_fix(uint32_t par, bool cj)
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) cx_arrange<SIDE>(r[i], (par >> i) & 1u, cj);
    }
    template <int SIDE>
    __device__ __forceinline__ void cx_vec(int i, const char* __restrict__ src, bool par, bool cj)
    {
        typedef typename Types<T>::uvec U;
        constexpr int H = VEC / 2;
        const U u = *reinterpret_cast<const U*>(src);
        if constexpr (SIDE == 1 && !KC) {
            const U u2 = *reinterpret_cast<const U*>(src + 16);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T v = e < H ? (par ? u[2 * e + 1] : u[2 * e]) : (par ? u2[2 * (e - H) + 1] : u2[2 * (e - H)]);
                r[i][e] = (cj && par) ? -v : v;
            }
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) r[i][e] = u[e];
            cx_arrange<SIDE>(r[i], par, cj);
        }
    }
    // Full chunk through the loop-invariant offsets (interior chunks).
    template <int SIDE>
    __device__ __forceinline__ void load_cx_at(const char* __restrict__ base, const uint32_t* off,
                                               uint32_t par, bool cj)
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) cx_vec<SIDE>(i, base + off[i], (par >> i) & 1u, cj);
    }
    // Fringe chunk: element by element, +0.0 outside the MNc x Kc complex
    // operand (x0, p0: the chunk origin in real indices).
    template <int SIDE>
    __device__ __forceinline__ void load_cx_edge(const T* __restrict__ X, int64_t ld, int64_t MNc,
                                                 int64_t Kc, int64_t x0, int64_t p0, bool cj, int tid)
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int o = elem_o(i, tid);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int64_t x = x0 + x_of(o) + (KC ? 0 : e), p = p0 + p_of(o) + (KC ? e : 0);
                const int64_t rr = SIDE == 0 ? x >> 1 : x, q = p >> 1;
                T v = T(0);
                if (rr < MNc && q < Kc) {
                    const T* z = X + 2 * (KC ? rr * ld + q : rr + q * ld);
                    if constexpr (SIDE == 0) {
                        const int s = (int)(x & 1), t = (int)(p & 1);
                        if (s == t) {
                            v = z[0];
                        } else {
                            const T im = cj ? -z[1] : z[1];
                            v = s == 0 ? -im : im;
                        }
                    } else {
                        const bool t = p & 1;
                        v = t ? (cj ? -z[1] : z[1]) : z[0];
                    }
                }
                r[i][e] = v;
            }
        }
    }

    // ---- Direct global -> LDS loads (LDS DMA) ---------------------------------
    // gfx950's global_load_lds_dwordx4 takes a 16-byte global address per lane
    // and writes the 64 lanes' data to 64 consecutive 16-byte LDS slots from a
    // wave-uniform base: lane l to slot base + l.  The chunk's LDS region is
    // ROWS rows of SPR slots (the padded pitch), DPR of them holding data; it
    // is covered by NI such wave loads at slot bases 64 g (the last one pulled
    // back so that it ends with the region: the overlap is written twice with
    // the same data).  A lane whose slot is row padding fetches the row's first
    // element again (a cache hit), so the padding receives copies of data that
    // no fragment read uses.
    static constexpr int SPR = LDP / VEC;
    static constexpr int DPR = (KC ? KT : MNT) / VEC;
    static constexpr int ROWS = KC ? MNT : KT;
    static constexpr int SLOTS = ROWS * SPR;
    static constexpr int NI = (SLOTS + 63) / 64;
    static constexpr int NIW = (NI + NTHR / 64 - 1) / (NTHR / 64);   // wave loads per wave
    static_assert(LDP % VEC == 0 && SLOTS >= 64, "LDS rows must hold whole slots");
    __device__ __forceinline__ static int dma_base(int g) { return 64 * g + 64 <= SLOTS ? 64 * g : SLOTS - 64; }
    // chunk element (x, p) that lane `lane` of wave load g brings
    __device__ __forceinline__ static void dma_elem(int g, int lane, int& x, int& p)
    {
        const int s = dma_base(g) + lane;
        const int row = s / SPR;
        int col = s - row * SPR;
        if (col >= DPR) col = 0;
        if (KC) { x = row; p = col * VEC; } else { p = row; x = col * VEC; }
    }
    // Issue this wave's loads of a chunk into the LDS buffer `lds` (wave loads
    // g = wave, wave + waves, ...).  Packed source (ld < 0): element (x, p) at
    // its packed position.  Unpacked source: at x + p*ld (MN-major) or
    // x*ld + p (K-major) from the chunk origin, and at the origin itself when
    // x0 + x is beyond MN (rows a fringe tile computes but never stores).
    // The offsets are recomputed per load rather than kept in registers.
    __device__ __forceinline__ static void dma_issue(T* lds, const char* __restrict__ base,
                                                     int64_t ld, int64_t x0, int64_t MN, int wave,
                                                     int lane)
    {
#pragma unroll
        for (int j = 0; j < NIW; ++j) {
            const int g = wave + j * (NTHR / 64);
            if (g < NI) {
                int x, p;
                dma_elem(g, lane, x, p);
                uint32_t off;
                if (ld < 0) off = (uint32_t)((KC ? x * KT + p : p * MNT + x) * (int)sizeof(T));
                else if (x0 + x < MN) off = (uint32_t)((KC ? x * ld + p : x + p * ld) * (int64_t)sizeof(T));
                else off = 0u;
                __builtin_amdgcn_global_load_lds(base + off, reinterpret_cast<char*>(lds) + dma_base(g) * 16,
                                                 16, 0, 0);
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
