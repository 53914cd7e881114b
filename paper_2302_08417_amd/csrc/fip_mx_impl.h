// Kernels, staging and launch template of the mixed-precision fused-pack GEMM
// (gfx950, CDNA4), shared by the translation units that instantiate them:
// fipgemm_mx.hip (every form and tile but the E4M3 256 x 256 tile) and
// fipgemm_mx_fp8big.hip (that tile, whose instantiation alone takes as long
// to compile as all the others, so the two compile side by side).
//
// The paper expects its fused packing to carry over to other precisions, and
// notes that the packing stage can encode a transformation of the data on its
// way into the packed buffer (Sec. 5, the 1m method).  Here the pack is where
// the conversion happens, once per panel:
//   BF16      A, B stored as bfloat16; the pack copies the bits.
//   FP8       A, B stored as OCP E4M3 codes (with optional power-of-two scales
//             per row of op(A) / column of op(B), applied in the epilogue);
//             the pack copies the bytes.
//   BF16X3    A, B stored as binary32; the first pass splits every element
//             into x0 + x1 + x2 (three bfloat16 terms, x0 = bf16(x),
//             x1 = bf16(x - x0), x2 = bf16(x - x0 - x1)) and packs the three
//             planes; later passes read the split planes instead of splitting
//             again.  Six bfloat16 MFMA products per block (terms i + j <= 2),
//             the small ones in their own accumulator, added to x0*y0 last.
//   BF16X3F   the same with two terms and three products.
// Accumulation is binary32 in every form (MFMA 16x16x32 bf16, 16x16x128 fp8;
// 32x32x16 bf16 for the 256 tile).
//
// Structure (shared with the FP64/FP32 kernel): one workgroup per MT x MT C
// tile, 2 x 2 waves of MT/2 x MT/2, k-steps of KT, two LDS buffers.  MT = 128
// for every form (two workgroups per CU).  bfloat16 also has MT = 256 (128 x
// 128 per wave, accumulators in the AGPRs, one workgroup per CU): half the LDS
// and L2 bytes per flop of the 128 tile, with one wave per SIMD, so its k-loop
// is software-pipelined by hand (fragment reads one k-block ahead of the
// MFMAs, one barrier per k-step placed before the last block, global loads
// two k-steps ahead).  Fused
// packing per operand panel: first toucher per XCD claims and packs, publishes
// a completion flag once its stores are acknowledged; other workgroups read
// the packed copy from the moment they see the flag, the unpacked operand
// before that.  Packed and unpacked sources fill the same thread's registers
// with the same elements, so each wave may choose its source independently.
//
// Packed layout (every form): chunk (tile t, k-step q) is block t*nK + q of
// PLANES * MT * KT elements; plane t of a block holds the chunk in the
// operand's storage orientation: element (x, p) at x*KT + p (K-major) or
// p*MT + x (MN-major).  A chunk goes from HBM (packed or not) to registers,
// LDS and the pack buffer as 16-byte vectors in that orientation; the MFMA
// fragments of MN-major chunks are read from LDS with the transposing loads
// (ds_read_b64_tr_b16 / _b8), so no pass transposes in registers.
#pragma once
#include <type_traits>

#include "fip_internal.h"
#include "fip_device.h"

namespace fip {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
// Element-aligned (4-byte) forms for unpacked operands: one 8- or 16-byte
// global load on gfx950 as long as the address is dword aligned.
typedef unsigned u4a __attribute__((ext_vector_type(4), aligned(4)));
typedef unsigned u2a __attribute__((ext_vector_type(2), aligned(4)));

constexpr int NTHR = 256;     // 2 x 2 waves; C tile MT x MT (128 or 256), per wave MT/2

// Per-form constants.  KT: k-step; SB: bytes per source element; PL: packed
// planes; EB: bytes per packed element; VK: k extent of a thread's micro-block
// (a micro-block is NR rows x VK k-values of the operand chunk; 256 threads
// cover the MT x KT chunk, NR = 4 for MT = 128, 8 for MT = 256); WPR: 32-bit
// words per micro-block row and plane.
template <int FORM> struct Form;
template <> struct Form<kMxBF16> {
    typedef uint16_t S;
    static constexpr int KT = 64, SB = 2, PL = 1, EB = 2, VK = 8;
};
template <> struct Form<kMxFP8> {
    typedef uint8_t S;
    static constexpr int KT = 128, SB = 1, PL = 1, EB = 1, VK = 16;
};
template <> struct Form<kMxX3> {
    typedef float S;
    static constexpr int KT = 32, SB = 4, PL = 3, EB = 2, VK = 4;
};
template <> struct Form<kMxX3Fast> {
    typedef float S;
    static constexpr int KT = 32, SB = 4, PL = 2, EB = 2, VK = 4;
};

template <int FORM, int MT_> struct Geo {
    typedef Form<FORM> Fm;
    static constexpr int MT = MT_;
    static constexpr int KT = Fm::KT, PL = Fm::PL, EB = Fm::EB, VK = Fm::VK, SB = Fm::SB;
    static constexpr int WPR = VK * EB / 4;
    static constexpr int KGROUPS = KT / VK;               // micro-blocks along k (8)
    static constexpr int NR = MT * KT / (NTHR * VK);      // rows per thread's micro-block
    static constexpr int WT = MT / 2;                     // per-wave C sub-tile
    static constexpr int FB = WT / 16;                    // 16 x 16 MFMA blocks per wave side
    static constexpr int PITCH = KT * EB + 16;            // LDS row pitch in bytes
    static constexpr int LDS_PLANE = MT * PITCH;
    static constexpr int LDS_OPERAND = PL * LDS_PLANE;    // one buffer of one operand
    static constexpr int PACK_PLANE = MT * KT * EB;       // bytes of one plane of a chunk
    static constexpr int PACK_CHUNK = PL * PACK_PLANE;
    // MN-major chunks (operand contiguous along m or n) sit in LDS as KT rows
    // of MT elements.  Pitch: the transposing fragment reads fetch 4 rows x 32
    // bytes (16-bit forms) or 8 rows x 16 bytes (E4M3) per 16 lanes; a row
    // stride of 32 (mod 128) or 16 (mod 128) bytes puts them on distinct banks.
    static constexpr int PITCH_MN = MT * EB + (FORM == kMxFP8 ? 16 : 32);
    static constexpr int LDS_PLANE_MN = KT * PITCH_MN;
    // LDS row of row p (a k index) of an MN-major chunk.  E4M3 swaps the two
    // 2-bit fields of p = 32g + 8h + i (row 32h + 8g + i): one transposing
    // fragment read then spans 32 consecutive rows (8 per lane group g)
    // instead of four groups 32 rows apart, and a 144-byte pitch spreads any
    // 16 consecutive rows over all 64 banks.  The other forms keep the order.
    __device__ __forceinline__ static int lds_row_mn(int p)
    {
        if constexpr (FORM == kMxFP8) return (p & ~127) | ((p & 24) << 2) | ((p & 96) >> 2) | (p & 7);
        else return p;
    }
    template <bool KC> static constexpr int lds_operand() { return PL * (KC ? LDS_PLANE : LDS_PLANE_MN); }
    static_assert(KGROUPS * (MT / NR) == NTHR, "micro-blocks must cover the chunk");
    static_assert(FORM != kMxFP8 || KT == 128, "E4M3 row permutation covers one 128-row chunk");
    static_assert(WPR == 2 || WPR == 4, "8- or 16-byte rows");
};

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// bfloat16 of a binary32, round to nearest even (the hardware conversion).
__device__ __forceinline__ uint32_t bf16_bits(float v)
{
    const __bf16 h = (__bf16)v;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_float(uint32_t h) { return __uint_as_float(h << 16); }

typedef float mx_f2 __attribute__((ext_vector_type(2)));
typedef __bf16 mx_bf2 __attribute__((ext_vector_type(2)));
// Two binary32 values as one word of two bfloat16 (lo in the low half), round
// to nearest even: one packed hardware conversion.
__device__ __forceinline__ uint32_t bf16x2_bits(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(mx_f2{lo, hi}, mx_bf2));
}
// The bfloat16 split of two binary32 values (elements e and e + 1 of a run):
// word t holds term t of both, x0 = bf16(x), x1 = bf16(x - x0) and, with three
// terms, x2 = bf16(x - x0 - x1); each difference is exact in binary32.
template <int PL>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t (&h)[3])
{
    h[0] = bf16x2_bits(a, b);
    const float ra = a - __uint_as_float(h[0] << 16), rb = b - __uint_as_float(h[0] & 0xFFFF0000u);
    h[1] = bf16x2_bits(ra, rb);
    h[2] = 0u;
    if constexpr (PL == 3)
        h[2] = bf16x2_bits(ra - __uint_as_float(h[1] << 16), rb - __uint_as_float(h[1] & 0xFFFF0000u));
}

// Registers of one K-major operand chunk (operand contiguous along k) on their
// way from HBM to LDS (and, for a producer, to the pack buffer): thread b holds
// rows x0 .. x0+NR-1 (x0 = NR*(b/8)) and k-values p0 .. p0+VK-1 (p0 =
// VK*(b%8)) of the chunk, already in packed form: for each plane and row, WPR
// words of consecutive k.  MN-major operands use the specialisation below.
template <int FORM, bool KC, int MT>
struct Stage {
    static_assert(KC, "MN-major chunks: Stage<FORM, false, MT>");
    typedef Geo<FORM, MT> G;
    static constexpr int NR = G::NR;
    typedef typename Form<FORM>::S S;
    static constexpr int PL = G::PL, WPR = G::WPR, VK = G::VK, EB = G::EB, SB = G::SB;
    static constexpr bool SPLIT = FORM == kMxX3 || FORM == kMxX3Fast;
    // Two-term split: unpacked binary32 words stay raw until finish(), so the
    // loads of the next chunk remain in flight across the current MFMAs; the
    // four raw words of row j wait in w[0][j] and w[1][j] (no extra
    // registers), and the caller knows (uniformly) which chunks came in raw.
    // The three-term split converts at load time: deferring it measured
    // slower for that form's packed path (its kernel is the most
    // register- and schedule-bound).
    static constexpr bool DEFER = FORM == kMxX3Fast;
    uint32_t w[PL][NR][WPR];

    __device__ __forceinline__ static int x0_of(int tid) { return NR * (tid / G::KGROUPS); }
    __device__ __forceinline__ static int p0_of(int tid) { return VK * (tid % G::KGROUPS); }
    // This thread's first source byte of the chunk at (xc, k = 0); ldb: bytes per row.
    __device__ __forceinline__ static const char* thread_src(const char* X, int64_t xc, int64_t ldb,
                                                             int tid)
    {
        return X + (xc + x0_of(tid)) * ldb + (int64_t)p0_of(tid) * SB;
    }
    // Byte step from one chunk to the next along k.
    __device__ __forceinline__ static int64_t chunk_step(int64_t ldb) { return (int64_t)G::KT * SB; }
    // Deferred forms: turn the raw binary32 words that load_full left into
    // the packed planes (only for a chunk that came through load_full).
    __device__ __forceinline__ void finish()
    {
        if constexpr (DEFER) {
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const float a = __uint_as_float(w[0][j][0]), b = __uint_as_float(w[0][j][1]),
                            c = __uint_as_float(w[1][j][0]), d = __uint_as_float(w[1][j][1]);
                put_pair(j, 0, a, b);
                put_pair(j, 2, c, d);
            }
        }
    }

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int j = 0; j < NR; ++j)
#pragma unroll
                for (int u = 0; u < WPR; ++u) w[t][j][u] = 0;
    }

    // Place source element (row j, k i) of the micro-block (bfloat16 / E4M3);
    // w must start cleared.
    __device__ __forceinline__ void put(int j, int i, S v)
    {
        static_assert(!SPLIT, "split forms place pairs");
        if constexpr (FORM == kMxBF16) {
            w[0][j][i >> 1] |= (uint32_t)v << (16 * (i & 1));
        } else {
            w[0][j][i >> 2] |= (uint32_t)v << (8 * (i & 3));
        }
    }
    // Split forms: elements (row j, k i) and (row j, k i + 1), i even, make
    // word i/2 of row j in every plane.
    __device__ __forceinline__ void put_pair(int j, int i, float a, float b)
    {
        uint32_t h[3];
        split_pair<PL>(a, b, h);
#pragma unroll
        for (int t = 0; t < PL; ++t) w[t][j][i >> 1] = h[t];
    }

    // Unpacked source, every element of the micro-block present and vector
    // loads dword aligned.  src: this thread's element (x0, p0) of the chunk;
    // ldb: leading dimension in bytes.
    __device__ __forceinline__ void load_full(const char* __restrict__ src, int64_t ldb)
    {
        if constexpr (KC) {
            // rows are contiguous along k: one 16-byte load per row
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const u4 v = *reinterpret_cast<const u4a*>(src + j * ldb);
                if constexpr (FORM == kMxBF16 || FORM == kMxFP8) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[0][j][u] = v[u];
                } else if constexpr (DEFER) {
                    static_assert(WPR == 2 && PL >= 2, "raw words fit planes 0 and 1");
                    w[0][j][0] = v[0];
                    w[0][j][1] = v[1];
                    w[1][j][0] = v[2];
                    w[1][j][1] = v[3];
                } else {
                    put_pair(j, 0, __uint_as_float(v[0]), __uint_as_float(v[1]));
                    put_pair(j, 2, __uint_as_float(v[2]), __uint_as_float(v[3]));
                }
            }
        }
    }

    // Unpacked source, fringe chunk (or unaligned operand): element loads with
    // predicates; elements outside the MN x K operand are +0 (Sec. 2.2
    // padding done in registers).  X: operand base; (xc, pc): chunk origin.
    __device__ __forceinline__ void load_edge(const S* __restrict__ X, int64_t ld, int64_t MN,
                                              int64_t K, int64_t xc, int64_t pc, int tid)
    {
        const int64_t x0 = xc + x0_of(tid), p0 = pc + p0_of(tid);
        if constexpr (SPLIT) {
#pragma unroll
            for (int j = 0; j < NR; ++j)
#pragma unroll
                for (int i = 0; i < VK; i += 2) {
                    const int64_t x = x0 + j, p = p0 + i;
                    float a = 0.f, b = 0.f;
                    if (x < MN && p < K) a = X[x * ld + p];
                    if (x < MN && p + 1 < K) b = X[x * ld + p + 1];
                    put_pair(j, i, a, b);
                }
        } else {
            clear();
#pragma unroll
            for (int j = 0; j < NR; ++j)
#pragma unroll
                for (int i = 0; i < VK; ++i) {
                    const int64_t x = x0 + j, p = p0 + i;
                    S v = S(0);
                    if (x < MN && p < K) v = X[x * ld + p];
                    put(j, i, v);
                }
        }
    }

    // Packed source: the chunk's planes, K-major; this thread's rows are
    // WPR-word runs at ((x0 + j)*KT + p0)*EB.
    __device__ __forceinline__ void load_packed(const char* __restrict__ chunk, int tid)
    {
        const int off = (x0_of(tid) * G::KT + p0_of(tid)) * EB;
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const char* p = chunk + t * G::PACK_PLANE + off + j * G::KT * EB;
                if constexpr (WPR == 4) {
                    const u4 v = *reinterpret_cast<const u4*>(p);
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[t][j][u] = v[u];
                } else {
                    const u2 v = *reinterpret_cast<const u2*>(p);
                    w[t][j][0] = v[0];
                    w[t][j][1] = v[1];
                }
            }
    }

    __device__ __forceinline__ void store_pack(char* __restrict__ chunk, int tid) const
    {
        const int off = (x0_of(tid) * G::KT + p0_of(tid)) * EB;
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                char* p = chunk + t * G::PACK_PLANE + off + j * G::KT * EB;
                if constexpr (WPR == 4) {
                    *reinterpret_cast<u4*>(p) = u4{w[t][j][0], w[t][j][1], w[t][j][2], w[t][j][3]};
                } else {
                    *reinterpret_cast<u2*>(p) = u2{w[t][j][0], w[t][j][1]};
                }
            }
    }

    __device__ __forceinline__ void store_lds(char* lds, int tid) const
    {
        const int off = x0_of(tid) * G::PITCH + p0_of(tid) * EB;
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                char* p = lds + t * G::LDS_PLANE + off + j * G::PITCH;
                if constexpr (WPR == 4) {
                    *reinterpret_cast<u4*>(p) = u4{w[t][j][0], w[t][j][1], w[t][j][2], w[t][j][3]};
                } else {
                    *reinterpret_cast<u2*>(p) = u2{w[t][j][0], w[t][j][1]};
                }
            }
    }
};

// Registers of one MN-major operand chunk (operand contiguous along m or n):
// the chunk's KT rows (one k each) of MT elements stay in that orientation,
// in HBM, in registers, in the pack and in LDS; the MFMA fragments are read
// from LDS with the transposing loads (ds_read_b64_tr_b16 / _b8), so no pass
// ever transposes in registers.  Eight threads cover 128 contiguous bytes of a
// row: thread b takes 16-byte source vectors (h, j) at row 32h + b/8, element
// VE*(b%8 + 8j) (VE = elements per 16 bytes).
template <int FORM, int MT>
struct Stage<FORM, false, MT> {
    typedef Geo<FORM, MT> G;
    typedef typename Form<FORM>::S S;
    static constexpr int KT = G::KT, PL = G::PL, EB = G::EB, SB = G::SB;
    static constexpr int VE = 16 / SB;                    // elements per source vector
    static constexpr int VT = MT * SB / 16 / 8;           // vectors per thread per row
    static constexpr int NP = KT / 32;                    // rows per thread
    static constexpr int NV = NP * VT;
    static constexpr int WPV = VE * EB / 4;               // packed words per vector and plane
    static_assert(VT >= 1 && NP >= 1 && (WPV == 2 || WPV == 4), "MN-major staging shape");
    static constexpr bool SPLIT = FORM == kMxX3 || FORM == kMxX3Fast;
    static constexpr bool DEFER = SPLIT;
    uint32_t w[PL][NV][WPV];
    // Split forms: unpacked binary32 words stay raw until finish(), so the
    // loads of the next chunk remain in flight across the current MFMAs.  The
    // four raw words of vector v wait in w[0][v] and w[1][v] (no extra
    // registers).  The caller knows (uniformly) which chunks came in raw.

    __device__ __forceinline__ static int row_of(int v, int tid) { return 32 * (v / VT) + (tid >> 3); }
    __device__ __forceinline__ static int x_of(int v, int tid) { return VE * ((tid & 7) + 8 * (v % VT)); }
    __device__ __forceinline__ static const char* thread_src(const char* X, int64_t xc, int64_t ldb,
                                                             int tid)
    {
        return X + (xc + x_of(0, tid)) * SB + (int64_t)row_of(0, tid) * ldb;
    }
    __device__ __forceinline__ static int64_t chunk_step(int64_t ldb) { return (int64_t)G::KT * ldb; }

    // Place the VE source elements of vector v (all planes).
    __device__ __forceinline__ void put_vec(int v, const uint32_t (&src)[4])
    {
        if constexpr (FORM == kMxBF16 || FORM == kMxFP8) {
#pragma unroll
            for (int u = 0; u < 4; ++u) w[0][v][u] = src[u];
        } else {
#pragma unroll
            for (int e = 0; e < VE; e += 2) {
                uint32_t h[3];
                split_pair<PL>(__uint_as_float(src[e]), __uint_as_float(src[e + 1]), h);
#pragma unroll
                for (int t = 0; t < PL; ++t) w[t][v][e >> 1] = h[t];
            }
        }
    }

    // Unpacked source, whole chunk present, dword-aligned rows.  src: this
    // thread's first source byte of the chunk; ldb: bytes per row (k).
    __device__ __forceinline__ void load_full(const char* __restrict__ src, int64_t ldb)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const u4 x = *reinterpret_cast<const u4a*>(src + (int64_t)(32 * (v / VT)) * ldb +
                                                       16 * 8 * (v % VT));
            if constexpr (SPLIT) {
                static_assert(WPV == 2 && PL >= 2, "raw words fit planes 0 and 1");
                w[0][v][0] = x[0];
                w[0][v][1] = x[1];
                w[1][v][0] = x[2];
                w[1][v][1] = x[3];
            } else {
                const uint32_t a[4] = {x[0], x[1], x[2], x[3]};
                put_vec(v, a);
            }
        }
    }

    // Split forms: turn the raw binary32 words that load_full left into the
    // packed planes (only for a chunk that came through load_full).
    __device__ __forceinline__ void finish()
    {
        if constexpr (SPLIT) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const uint32_t a[4] = {w[0][v][0], w[0][v][1], w[1][v][0], w[1][v][1]};
                put_vec(v, a);
            }
        }
    }

    // Unpacked source, fringe chunk or unaligned operand: element loads with
    // predicates; elements outside the operand are +0.
    __device__ __forceinline__ void load_edge(const S* __restrict__ X, int64_t ld, int64_t MN,
                                              int64_t K, int64_t xc, int64_t pc, int tid)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int64_t p = pc + row_of(v, tid), x0 = xc + x_of(v, tid);
            uint32_t a[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const int64_t x = x0 + e;
                uint32_t b = 0u;
                if (x < MN && p < K) {
                    if constexpr (SB == 4) b = __float_as_uint(X[x + p * ld]);
                    else b = (uint32_t)X[x + p * ld];
                }
                a[e * SB / 4] |= b << (8 * ((e * SB) & 3));
            }
            put_vec(v, a);
        }
    }

    // Packed source (MN-major planes): element (x, p) of plane t at (p*MT + x)*EB.
    __device__ __forceinline__ void load_packed(const char* __restrict__ chunk, int tid)
    {
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const char* q = chunk + t * G::PACK_PLANE + (row_of(v, tid) * MT + x_of(v, tid)) * EB;
                if constexpr (WPV == 4) {
                    const u4 x = *reinterpret_cast<const u4*>(q);
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[t][v][u] = x[u];
                } else {
                    const u2 x = *reinterpret_cast<const u2*>(q);
                    w[t][v][0] = x[0];
                    w[t][v][1] = x[1];
                }
            }
    }

    __device__ __forceinline__ void store_pack(char* __restrict__ chunk, int tid) const
    {
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                char* q = chunk + t * G::PACK_PLANE + (row_of(v, tid) * MT + x_of(v, tid)) * EB;
                if constexpr (WPV == 4)
                    *reinterpret_cast<u4*>(q) = u4{w[t][v][0], w[t][v][1], w[t][v][2], w[t][v][3]};
                else
                    *reinterpret_cast<u2*>(q) = u2{w[t][v][0], w[t][v][1]};
            }
    }

    __device__ __forceinline__ void store_lds(char* lds, int tid) const
    {
#pragma unroll
        for (int t = 0; t < PL; ++t)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                char* q = lds + t * G::LDS_PLANE_MN + G::lds_row_mn(row_of(v, tid)) * G::PITCH_MN +
                          x_of(v, tid) * EB;
                if constexpr (WPV == 4)
                    *reinterpret_cast<u4*>(q) = u4{w[t][v][0], w[t][v][1], w[t][v][2], w[t][v][3]};
                else
                    *reinterpret_cast<u2*>(q) = u2{w[t][v][0], w[t][v][1]};
            }
    }
};

typedef short s4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef int i2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) s4v lds_s4v;
typedef __attribute__((address_space(3))) i2v lds_i2v;

// MFMA operand fragments from one LDS plane.  Every fragment is "lane l gives
// element x = x0 + (l % R) and a run of k starting at k0 + run(l)".
//   K-major plane (rows x, pitch PITCH): one or two 16-byte reads.
//   MN-major plane (rows k, pitch PITCH_MN): transposing reads.  Within each
//   16 lanes, ds_read_b64_tr_b16 gives lane i, item r, element i%4 of the
//   8 bytes that lane 4r + i/4 addressed (tr_b8: byte i%8 of lane 2r + i/8),
//   so lane c addressing row k + c/4 (c/2), column x + 4*(c%4) (8*(c%2))
//   hands lane i the k-run of column x + i.
template <int FORM, int MT, bool KC>
struct Frag {
    typedef Geo<FORM, MT> G;

    __device__ __forceinline__ static s4v tr16(const char* p)
    {
        return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4v*)(p));
    }
    __device__ __forceinline__ static i2v tr8(const char* p)
    {
        return __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i2v*)(p));
    }
    // 8 bfloat16 k-values: x = x0 + l%16 (sixteen-row form) or x0 + l%32
    // (thirty-two-row form, R = 32), k = k0 + 8*(l/R) .. +8.
    template <int R>
    __device__ __forceinline__ static bf8v bf16(const char* plane, int x0, int k0, int lane)
    {
        const int x = x0 + (lane & (R - 1)), run = lane / R;
        if constexpr (KC) {
            return *reinterpret_cast<const bf8v*>(plane + x * G::PITCH + (k0 + 8 * run) * 2);
        } else {
            const int c = lane & 15;
            const int xb = x0 + (lane & (R - 1) & ~15) + 4 * (c & 3);
            const char* q = plane + (k0 + 8 * run + (c >> 2)) * G::PITCH_MN + xb * 2;
            const s4v lo = tr16(q), hi = tr16(q + 4 * G::PITCH_MN);
            const s8v v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            return __builtin_bit_cast(bf8v, v);
        }
    }
    // 32 E4M3 k-values: x = x0 + l%16, k = k0 + 32*(l/16) .. +32 (sixteen-row
    // form), or x = x0 + l%32, k = k0 + 32*(l/32) .. +32 (R = 32).
    template <int R>
    __device__ __forceinline__ static i8v fp8(const char* plane, int x0, int k0, int lane)
    {
        const int run = lane / R;
        if constexpr (KC) {
            return *reinterpret_cast<const i8v*>(plane + (x0 + (lane & (R - 1))) * G::PITCH + k0 + 32 * run);
        } else {
            // k = k0 + 32*run + 8h + c/2 (h = 0..3, k0 a multiple of 32) sits
            // at LDS row 32h + 8*((k0 + 32*run) / 32) + c/2 (lds_row_mn)
            const int c = lane & 15;
            const int xb = x0 + (lane & (R - 1) & ~15) + 8 * (c & 1);
            const char* q = plane + (8 * ((k0 >> 5) + run) + (c >> 1)) * G::PITCH_MN + xb;
            i8v v;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const i2v t = tr8(q + 32 * h * G::PITCH_MN);
                v[2 * h] = t[0];
                v[2 * h + 1] = t[1];
            }
            return v;
        }
    }
};

struct MxParams {
    const char* A; const char* B; char* C;
    int64_t a_ld, b_ld, ldc;        // in elements
    int64_t M, N, K;
    float alpha, beta;
    const float* a_scale; const float* b_scale;
    char* apack; char* bpack;
    int64_t apack_copy, bpack_copy;  // bytes per copy
    uint64_t* aflag; uint64_t* bflag; uint64_t* aclaim; uint64_t* bclaim;
    unsigned long long* stats;
    uint64_t epoch;
    int tilesM, tilesN, nK, group_m;
    int mode, pack_a, pack_b, no_publish, do_stats, order;
    int a_pack_from, b_pack_from;  // first tile row / column whose panel is packed
    int shared_copy;  // 1: one pack copy for all XCDs (copy 0), else one per XCD
    int a_vec, b_vec;                // unpacked vector loads allowed (dword alignment)
    int c_bf16;
    int split, slice_ksteps;         // k slices (1: none) and k-steps per slice
    float* part;                     // slice partials [split][N][M] when split > 1
};

// One MFMA k-substep on LDS buffers la (A-side rows) and lb (B-side rows).
// Fragment of a 16 x 16 block: lane l supplies row l%16 and a contiguous run
// of k (8 bf16 = 16 bytes, or 32 fp8 bytes) starting at run (l/16); A and B
// use the same k assignment, which is all the product needs.  Output item r
// of lane l is C[4*(l/16) + r][l%16].
template <int FORM, int MT>
struct Mma {
    typedef Geo<FORM, MT> G;
    static constexpr int NACC = (FORM == kMxX3 || FORM == kMxX3Fast) ? 2 : 1;
    static constexpr int FB = G::FB;
    typedef f4 Acc[NACC][FB][FB];

    __device__ __forceinline__ static void zero(Acc& acc)
    {
#pragma unroll
        for (int t = 0; t < NACC; ++t)
#pragma unroll
            for (int a = 0; a < FB; ++a)
#pragma unroll
                for (int b = 0; b < FB; ++b) acc[t][a][b] = f4{0.f, 0.f, 0.f, 0.f};
    }

    // Visit the result as runs of four consecutive rows of one column:
    // fn(v, row offset, column offset) within the wave's sub-tile.
    template <class Fn>
    __device__ __forceinline__ static void pieces(const Acc& acc, int lane, Fn&& fn)
    {
#pragma unroll
        for (int a = 0; a < FB; ++a)
#pragma unroll
            for (int b = 0; b < FB; ++b) {
                f4 v = acc[0][a][b];
                if constexpr (NACC == 2) v = acc[1][a][b] + v;  // small terms first, then x0*y0
                fn(v, a * 16 + 4 * (lane >> 4), b * 16 + (lane & 15));
            }
    }

    // One k-step on the LDS buffers sa, sb (plane 0 of each operand); xa, xb:
    // the wave's first row / column.
    template <bool AKC, bool BKC>
    __device__ __forceinline__ static void step(const char* sa, const char* sb, int xa, int xb,
                                                int lane, Acc& acc)
    {
        typedef Frag<FORM, MT, AKC> FA;
        typedef Frag<FORM, MT, BKC> FB_;
        // B fragments of the whole wave row first, then one A fragment at a
        // time against all of them (FB x FB MFMAs per A fragment)
        if constexpr (FORM == kMxFP8) {
            i8v fb[FB];
#pragma unroll
            for (int b = 0; b < FB; ++b) fb[b] = FB_::template fp8<16>(sb, xb + b * 16, 0, lane);
#pragma unroll
            for (int a = 0; a < FB; ++a) {
                const i8v fa = FA::template fp8<16>(sa, xa + a * 16, 0, lane);
#pragma unroll
                for (int b = 0; b < FB; ++b)
                    acc[0][a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        fa, fb[b], acc[0][a][b], 0, 0, 0, 0, 0, 0);
            }
            // fragment reads interleaved one to one with the MFMAs (E4M3 at
            // 16384: 5.47 against 5.87 ms issuing the reads as a burst)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS reads
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMAs
            }
        } else if constexpr (FORM == kMxBF16) {
#pragma unroll
            for (int s = 0; s < G::KT / 32; ++s) {
                bf8v fb[FB];
#pragma unroll
                for (int b = 0; b < FB; ++b) fb[b] = FB_::template bf16<16>(sb, xb + b * 16, s * 32, lane);
#pragma unroll
                for (int a = 0; a < FB; ++a) {
                    const bf8v fa = FA::template bf16<16>(sa, xa + a * 16, s * 32, lane);
#pragma unroll
                    for (int b = 0; b < FB; ++b)
                        acc[0][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[b],
                                                                               acc[0][a][b], 0, 0, 0);
                }
                // reads interleaved one to one with the MFMAs (2-3 % at 4096;
                // the split forms measured slower with it and keep the
                // compiler's order)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS reads
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMAs
                }
            }
        } else {
            // split forms: KT = 32, one substep; planes PL of each operand
            constexpr int PL = G::PL;
            constexpr int PA = G::template lds_operand<AKC>() / PL;   // plane stride
            constexpr int PB = G::template lds_operand<BKC>() / PL;
            bf8v fb[PL][FB];
#pragma unroll
            for (int t = 0; t < PL; ++t)
#pragma unroll
                for (int b = 0; b < FB; ++b) fb[t][b] = FB_::template bf16<16>(sb + t * PB, xb + b * 16, 0, lane);
#pragma unroll
            for (int a = 0; a < FB; ++a) {
                bf8v fa[PL];
#pragma unroll
                for (int t = 0; t < PL; ++t) fa[t] = FA::template bf16<16>(sa + t * PA, xa + a * 16, 0, lane);
#pragma unroll
                for (int b = 0; b < FB; ++b) {
                    f4 big = acc[0][a][b], small = acc[1][a][b];
                    big = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0], fb[0][b], big, 0, 0, 0);
                    small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0], fb[1][b], small, 0, 0, 0);
                    small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1], fb[0][b], small, 0, 0, 0);
                    if constexpr (PL == 3) {
                        small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0], fb[2][b], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1], fb[1][b], small, 0, 0, 0);
                        small = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2], fb[0][b], small, 0, 0, 0);
                    }
                    acc[0][a][b] = big;
                    acc[1][a][b] = small;
                }
            }
        }
    }
};

// MT = 256 (bfloat16, E4M3): 32 x 32 MFMA blocks (v_mfma 32x32x16 bf16,
// 32x32x64 f8f6f4), 4 x 4 blocks of 16 accumulators per wave.  The 32 x 32
// form keeps a wave's 256 accumulators in the AGPRs without the register
// shuffling the compiler inserts around 64 separate 16 x 16 accumulators.
// Fragment: lane l supplies row l%32 and a run of consecutive k (8 bfloat16 or
// 32 E4M3 values) at run l/32; output item r of lane l is
// C[8*(r/4) + 4*(l/32) + r%4][l%32].
template <int FORM>
struct Mma<FORM, 256> {
    static_assert(FORM == kMxBF16 || FORM == kMxFP8, "256 x 256 tiles: bfloat16 and E4M3");
    static constexpr bool F8 = FORM == kMxFP8;
    typedef Geo<FORM, 256> G;
    static constexpr int NACC = 1;
    static constexpr int FB = G::WT / 32;   // 4
    typedef f16v Acc[FB][FB];

    __device__ __forceinline__ static void zero(Acc& acc)
    {
#pragma unroll
        for (int a = 0; a < FB; ++a)
#pragma unroll
            for (int b = 0; b < FB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
    }

    template <class Fn>
    __device__ __forceinline__ static void pieces(const Acc& acc, int lane, Fn&& fn)
    {
        static_for<0, FB * FB * 4>([&](auto k) {
            constexpr int a = decltype(k)::value / (4 * FB), b = decltype(k)::value / 4 % FB,
                          g = decltype(k)::value % 4;
            fn(f4{acc[a][b][4 * g], acc[a][b][4 * g + 1], acc[a][b][4 * g + 2], acc[a][b][4 * g + 3]},
               a * 32 + 8 * g + 4 * (lane >> 5), b * 32 + (lane & 31));
        });
    }

    // k-blocks of one MFMA: 16 (bfloat16) or 64 (E4M3) k-values; NB per k-step.
    static constexpr int KB = F8 ? 64 : 16;
    static constexpr int NB = G::KT / KB;
    typedef std::conditional_t<F8, i8v, bf8v> V;
    struct Frags {
        V a[FB], b[FB];
    };

    template <bool KC>
    __device__ __forceinline__ static V frag(const char* plane, int x0, int k0, int lane)
    {
        if constexpr (F8) return Frag<FORM, 256, KC>::template fp8<32>(plane, x0, k0, lane);
        else return Frag<FORM, 256, KC>::template bf16<32>(plane, x0, k0, lane);
    }

    // Fragments of k-block s of the wave's rows (from xa) and columns (from xb).
    template <bool AKC, bool BKC>
    __device__ __forceinline__ static void read(const char* sa, const char* sb, int xa, int xb,
                                                int lane, int s, Frags& f)
    {
#pragma unroll
        for (int b = 0; b < FB; ++b) f.b[b] = frag<BKC>(sb, xb + b * 32, s * KB, lane);
#pragma unroll
        for (int a = 0; a < FB; ++a) f.a[a] = frag<AKC>(sa, xa + a * 32, s * KB, lane);
    }

    __device__ __forceinline__ static void mma(const Frags& f, Acc& acc)
    {
#pragma unroll
        for (int a = 0; a < FB; ++a)
#pragma unroll
            for (int b = 0; b < FB; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[a], f.b[b], acc[a][b], 0, 0, 0);
    }

    // E4M3: a block's fragments are twice the bfloat16 ones (8 registers
    // each), too many to hold two blocks beside the staged chunks, so the
    // next block's fragments are read in place while this block's MFMAs run:
    // A fragments one ahead of their MFMAs, each B fragment right after its
    // last MFMA of this block.  On entry f holds the block's B fragments and
    // its first A fragment; on exit, the next block's (when NEXT).
    struct Frags8 {
        i8v b[FB];
        i8v a;
    };

    template <bool AKC, bool BKC>
    __device__ __forceinline__ static void first8(const char* sa, const char* sb, int xa, int xb,
                                                  int lane, int s, Frags8& f)
    {
#pragma unroll
        for (int b = 0; b < FB; ++b) f.b[b] = frag<BKC>(sb, xb + b * 32, s * KB, lane);
        f.a = frag<AKC>(sa, xa, s * KB, lane);
    }

    // Block s of the LDS buffer (sa); the next block is block ns of (na, nb).
    // before_next() runs after the last read of this block has been issued
    // and before the first read of the next one (the k-step's barrier goes
    // there when the next block sits in the other buffer).
    template <bool AKC, bool BKC, bool NEXT, class Hook>
    __device__ __forceinline__ static void block8(const char* sa, int s, const char* na,
                                                  const char* nb, int ns, int xa, int xb, int lane,
                                                  Frags8& f, Acc& acc, Hook&& before_next)
    {
        i8v fa[2];
        fa[0] = f.a;
#pragma unroll
        for (int a = 0; a < FB; ++a) {
            if (a + 1 < FB) {
                fa[(a + 1) & 1] = frag<AKC>(sa, xa + (a + 1) * 32, s * KB, lane);
            } else {
                __builtin_amdgcn_sched_barrier(0);
                before_next();
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (NEXT) fa[0] = frag<AKC>(na, xa, ns * KB, lane);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < FB; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    fa[a & 1], f.b[b], acc[a][b], 0, 0, 0, 0, 0, 0);
                if (a == FB - 1 && NEXT) {
                    __builtin_amdgcn_sched_barrier(0);
                    f.b[b] = frag<BKC>(nb, xb + b * 32, ns * KB, lane);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        f.a = fa[0];
    }
};

template <int FORM, int MT, bool AKC, bool BKC>
__global__ void __launch_bounds__(NTHR, (MT == 128 && (FORM == kMxBF16 || FORM == kMxFP8)) ? 2 : 1)
gemm_mx_kernel(const MxParams P)
{
    typedef Geo<FORM, MT> G;
    typedef Stage<FORM, AKC, MT> StA;
    typedef Stage<FORM, BKC, MT> StB;
    typedef typename Form<FORM>::S S;
    constexpr int KT = G::KT, SB = G::SB, WT = G::WT;

    __shared__ __attribute__((aligned(16))) char sA[2][G::template lds_operand<AKC>()];
    __shared__ __attribute__((aligned(16))) char sB[2][G::template lds_operand<BKC>()];
    __shared__ int s_role;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // Split k: workgroup w computes k-slice w / tiles of tile w % tiles, i.e.
    // chunks [q0, q1); slices of one tile are `tiles` workgroups apart.
    const int NS = MT == 128 ? P.split : 1;  // the 256 tile never splits
    const int ntiles = P.tilesM * P.tilesN;
    const int slice = NS > 1 ? (int)(blockIdx.x / (unsigned)ntiles) : 0;
    int tm, tn;
    tile_coords((int)blockIdx.x - slice * ntiles, P.tilesM, P.tilesN, P.group_m, P.order, tm, tn);
    const int64_t x0a = (int64_t)tm * MT, x0b = (int64_t)tn * MT;
    const int nK = P.nK;
    const int q0 = slice * P.slice_ksteps;
    const int q1 = q0 + P.slice_ksteps < nK ? q0 + P.slice_ksteps : nK;
    const int nKfull = (int)(P.K / KT);
    const uint64_t epoch = P.epoch;

    // Unpacked sources: this thread's element (x0, p0) of chunk 0, and the
    // byte step from one chunk to the next.
    const bool a_in = P.a_vec && x0a + MT <= P.M, b_in = P.b_vec && x0b + MT <= P.N;
    const int64_t a_ldb = P.a_ld * SB, b_ldb = P.b_ld * SB;
    const char* a_src = StA::thread_src(P.A, x0a, a_ldb, tid);
    const char* b_src = StB::thread_src(P.B, x0b, b_ldb, tid);
    const int64_t a_step = StA::chunk_step(a_ldb), b_step = StB::chunk_step(b_ldb);

    const bool consume = P.mode == kModeConsumePacked;
    bool fused = P.mode == kModeFused;
    int copy = 0;
    if (fused) {
        const unsigned x = xcc_id();
        if (P.shared_copy) copy = 0;
        else if (x < (unsigned)kCopies) copy = (int)x;
        else fused = false;
    }
    const bool useA = fused && P.pack_a && tm >= P.a_pack_from;
    const bool useB = fused && P.pack_b && tn >= P.b_pack_from;
    char* apanel = nullptr;
    char* bpanel = nullptr;
    // a copy holds the packed panels from a_pack_from / b_pack_from on
    if (useA || consume)
        apanel = P.apack + copy * P.apack_copy + (int64_t)(tm - P.a_pack_from) * nK * G::PACK_CHUNK;
    if (useB || consume)
        bpanel = P.bpack + copy * P.bpack_copy + (int64_t)(tn - P.b_pack_from) * nK * G::PACK_CHUNK;
    // one claim and one completion flag per (copy, panel, k-slice)
    const int64_t aslot = ((int64_t)copy * P.tilesM + tm) * NS + slice;
    const int64_t bslot = ((int64_t)copy * P.tilesN + tn) * NS + slice;
    uint64_t* adone = useA ? P.aflag + aslot : nullptr;
    uint64_t* bdone = useB ? P.bflag + bslot : nullptr;

    // First touch claims the panel (Sec. 3.2); thread 0 claims, the role is
    // broadcast because every thread stores its share of each packed chunk.
    if (tid == 0) {
        int role = 0;
        if (useA && __hip_atomic_exchange(P.aclaim + aslot, epoch, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) != epoch)
            role |= 1;
        if (useB && __hip_atomic_exchange(P.bclaim + bslot, epoch, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) != epoch)
            role |= 2;
        s_role = role;
    }
    __syncthreads();
    const bool prodA = s_role & 1, prodB = s_role & 2;
    const bool producer = prodA || prodB;
    const bool wantA = useA && !prodA, wantB = useB && !prodB;

    constexpr int REPOLL = 8;
    bool apk = consume, bpk = consume;
    {
        const uint64_t fa = wantA ? peek_flag(adone) : 0, fb = wantB ? peek_flag(bdone) : 0;
        apk = apk || (wantA && __builtin_amdgcn_readfirstlane((int)(fa == epoch)) != 0);
        bpk = bpk || (wantB && __builtin_amdgcn_readfirstlane((int)(fb == epoch)) != 0);
        if ((wantA && apk) || (wantB && bpk)) acquire_packed();
    }

    unsigned long long n_prod = 0, n_pk = 0, n_unpk = 0, n_polls = 0;
    StA ra;
    StB rb;
    auto count_chunk = [&]() {
        if (P.do_stats && tid == 0) {
            n_prod += (int)prodA + (int)prodB;
            n_pk += (int)(wantA && apk) + (int)(wantB && bpk) + (consume ? 2 : 0);
            n_unpk += (int)(wantA && !apk) + (int)(wantB && !bpk);
        }
    };
    // Split forms: a chunk read by load_full sits in registers as raw binary32
    // until put_chunks converts it; a_raw / b_raw say so (workgroup-uniform).
    bool a_raw = false, b_raw = false;
    auto load_chunks = [&](int c) {
        const bool kin = c < nKfull;
        a_raw = StA::DEFER && !apk && a_in && kin;
        b_raw = StB::DEFER && !bpk && b_in && kin;
        if (apk) ra.load_packed(apanel + (int64_t)c * G::PACK_CHUNK, tid);
        else if (a_in && kin) ra.load_full(a_src + (int64_t)c * a_step, a_ldb);
        else ra.load_edge(reinterpret_cast<const S*>(P.A), P.a_ld, P.M, P.K, x0a, (int64_t)c * KT, tid);
        if (bpk) rb.load_packed(bpanel + (int64_t)c * G::PACK_CHUNK, tid);
        else if (b_in && kin) rb.load_full(b_src + (int64_t)c * b_step, b_ldb);
        else rb.load_edge(reinterpret_cast<const S*>(P.B), P.b_ld, P.N, P.K, x0b, (int64_t)c * KT, tid);
        count_chunk();
    };

    typedef Mma<FORM, MT> MM;
    typename MM::Acc acc;
    MM::zero(acc);

    // Flag polls while an operand still comes unpacked: the loads are issued
    // in one place and their values used later, off the critical path.
    bool polling = false;
    uint64_t pfa = 0, pfb = 0;
    auto poll_issue = [&](int q) {
        polling = ((wantA && !apk) || (wantB && !bpk)) && q % REPOLL == REPOLL - 1;
        if (polling) {
            pfa = wantA && !apk ? peek_flag(adone) : 0;
            pfb = wantB && !bpk ? peek_flag(bdone) : 0;
        }
    };
    auto poll_finish = [&]() {
        if (polling) {
            const bool na = !apk && wantA && __builtin_amdgcn_readfirstlane((int)(pfa == epoch)) != 0;
            const bool nb = !bpk && wantB && __builtin_amdgcn_readfirstlane((int)(pfb == epoch)) != 0;
            if (na || nb) acquire_packed();
            apk = apk || na;
            bpk = bpk || nb;
            if (P.do_stats && tid == 0) ++n_polls;
        }
    };
    // Each operand takes one of two complete paths (convert then store, or
    // store), so no register value flows out of a conditional conversion.
    auto put_chunks = [&](int buf, int c) {
        // three-term split: one path (measured faster for this form)
        if constexpr (FORM == kMxX3) {
            if (a_raw) ra.finish();
            if (b_raw) rb.finish();
            ra.store_lds(sA[buf], tid);
            rb.store_lds(sB[buf], tid);
            if (prodA) ra.store_pack(apanel + (int64_t)c * G::PACK_CHUNK, tid);
            if (prodB) rb.store_pack(bpanel + (int64_t)c * G::PACK_CHUNK, tid);
            return;
        }
        if (a_raw) {
            ra.finish();
            ra.store_lds(sA[buf], tid);
            if (prodA) ra.store_pack(apanel + (int64_t)c * G::PACK_CHUNK, tid);
        } else {
            ra.store_lds(sA[buf], tid);
            if (prodA) ra.store_pack(apanel + (int64_t)c * G::PACK_CHUNK, tid);
        }
        if (b_raw) {
            rb.finish();
            rb.store_lds(sB[buf], tid);
            if (prodB) rb.store_pack(bpanel + (int64_t)c * G::PACK_CHUNK, tid);
        } else {
            rb.store_lds(sB[buf], tid);
            if (prodB) rb.store_pack(bpanel + (int64_t)c * G::PACK_CHUNK, tid);
        }
    };

    load_chunks(q0);
    put_chunks(0, q0);
    if constexpr (MT == 256 && FORM == kMxFP8) {
        // E4M3 256 tile: the next block's fragments are read during this
        // block's MFMAs (Mma::block8).  Per k-step: block 0, whose MFMAs
        // overlap the reads of block 1; the next chunk from registers to the
        // other LDS buffer and the global loads two k-steps ahead; block 1,
        // whose last A fragment is read before the barrier, and whose last
        // MFMAs overlap the reads of the next k-step's block 0 from the other
        // buffer, after the barrier.
        static_assert(MM::NB == 2, "two k-blocks per k-step");
        typename MM::Frags8 f;
        if (nK > 1) load_chunks(1);
        __syncthreads();
        const int xa = wm * WT, xb = wn * WT;
        MM::template first8<AKC, BKC>(sA[0], sB[0], xa, xb, lane, 0, f);
        auto nothing = [] {};
        auto barrier = [] { __syncthreads(); };
        // the last k-step is peeled off (MORE = false), as in the bfloat16 loop
        auto kstep = [&](int q, auto more_c) {
            constexpr bool more = decltype(more_c)::value;
            const int cur = q & 1;
            MM::template block8<AKC, BKC, true>(sA[cur], 0, sA[cur], sB[cur], 1, xa, xb, lane, f,
                                                acc, nothing);
            if constexpr (more) {
                put_chunks(cur ^ 1, q + 1);
                poll_issue(q);
                if (q + 2 < nK) load_chunks(q + 2);
                MM::template block8<AKC, BKC, true>(sA[cur], 1, sA[cur ^ 1], sB[cur ^ 1], 0, xa, xb,
                                                    lane, f, acc, barrier);
            } else {
                MM::template block8<AKC, BKC, false>(sA[cur], 1, sA[cur], sB[cur], 0, xa, xb, lane,
                                                     f, acc, nothing);
            }
            poll_finish();
        };
        for (int q = 0; q + 1 < nK; ++q) kstep(q, std::true_type{});
        kstep(nK - 1, std::false_type{});
    } else if constexpr (MT == 256) {
        // (no split k here: q0 = 0 and q1 = nK)
        // Software pipeline with one wave per SIMD: the fragments of k-block
        // s + 1 are read while the MFMAs of block s issue; the next chunk goes
        // from registers to the other LDS buffer after block NB - 2, and the
        // one barrier per k-step sits before the last block, so the next
        // k-step's first fragments arrive while that block's MFMAs run.
        // Global loads run two k-steps ahead (one chunk in registers).
        constexpr int NB = MM::NB;
        static_assert(NB >= 2, "at least two k-blocks per k-step");
        typename MM::Frags fr[2];
        if (nK > 1) load_chunks(1);
        __syncthreads();
        const int xa = wm * WT, xb = wn * WT;
        MM::template read<AKC, BKC>(sA[0], sB[0], xa, xb, lane, 0, fr[0]);
        // The last k-step is peeled off (MORE = false), so inside the loop
        // the path through the barrier is straight-line code and the MFMAs of
        // the last block do not wait for the next k-step's fragment reads.
        // sched_barrier(0) keeps the compiler from moving MFMAs across the
        // phase boundaries (it would otherwise hoist the last block's MFMAs
        // above the barrier and leave the barrier wait uncovered); within a
        // block, sched_group_barrier interleaves the reads with the MFMAs.
        auto kstep = [&](int q, auto more_c) {
            constexpr bool more = decltype(more_c)::value;
            const int cur = q & 1;
#pragma unroll
            for (int s = 0; s < NB; ++s) {
                if (s + 1 < NB) MM::template read<AKC, BKC>(sA[cur], sB[cur], xa, xb, lane, s + 1, fr[(s + 1) & 1]);
                if (s == NB - 1 && more) {
                    __builtin_amdgcn_sched_barrier(0);
                    __syncthreads();
                    MM::template read<AKC, BKC>(sA[cur ^ 1], sB[cur ^ 1], xa, xb, lane, 0, fr[0]);
                }
                // the next block's fragment reads are interleaved with this
                // block's MFMAs, two of each at a time (3-4 % faster than
                // issuing the reads as one burst ahead of the MFMAs)
                MM::mma(fr[s & 1], acc);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS reads
                    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMAs
                }
                __builtin_amdgcn_sched_barrier(0);
                if (s == NB - 2 && more) {
                    put_chunks(cur ^ 1, q + 1);
                    poll_issue(q);
                    if (q + 2 < nK) load_chunks(q + 2);
                }
                if (s == NB - 1) poll_finish();
            }
        };
        for (int q = 0; q + 1 < nK; ++q) kstep(q, std::true_type{});
        kstep(nK - 1, std::false_type{});
    } else {
        // A tile that reads both operands packed from its first chunk on (the
        // pack-then-compute baseline, or a later pass that finds both panels
        // published) has nothing to convert, store or poll: it runs a copy of
        // the loop compiled for that case alone, so the general loop's
        // conversion code does not shape its schedule.
        auto loop = [&](auto all_packed_c) {
            constexpr bool ALL_PACKED = decltype(all_packed_c)::value;
            __syncthreads();
            for (int q = q0; q < q1; ++q) {
                const int cur = (q - q0) & 1;
                const bool more = q + 1 < q1;
                if constexpr (ALL_PACKED) {
                    if (more) {
                        ra.load_packed(apanel + (int64_t)(q + 1) * G::PACK_CHUNK, tid);
                        rb.load_packed(bpanel + (int64_t)(q + 1) * G::PACK_CHUNK, tid);
                        count_chunk();
                    }
                    MM::template step<AKC, BKC>(sA[cur], sB[cur], wm * WT, wn * WT, lane, acc);
                    if (more) {
                        ra.store_lds(sA[cur ^ 1], tid);
                        rb.store_lds(sB[cur ^ 1], tid);
                    }
                } else {
                    poll_issue(q);
                    if (more) load_chunks(q + 1);
                    MM::template step<AKC, BKC>(sA[cur], sB[cur], wm * WT, wn * WT, lane, acc);
                    if (more) put_chunks(cur ^ 1, q + 1);
                    poll_finish();
                }
                __syncthreads();
            }
        };
        // apk and bpk imply that this workgroup produces neither panel; the
        // three-term split keeps the one loop (measured faster for that form)
        if (FORM != kMxX3 && apk && bpk) loop(std::true_type{});
        else loop(std::false_type{});
    }

    if (producer) {
        wait_all_memory();
        __syncthreads();
        if (tid == 0 && !P.no_publish) {
            if (prodA) publish_flag(adone, epoch);
            if (prodB) publish_flag(bdone, epoch);
        }
    }
    if (P.do_stats && tid == 0) {
        atomicAdd(P.stats + 0, n_prod);
        atomicAdd(P.stats + 1, n_pk);
        atomicAdd(P.stats + 2, n_unpk);
        atomicAdd(P.stats + 3, n_polls);
    }

    // Epilogue: the accumulators come as runs of four consecutive rows of one
    // column of the column-major C (16 x 16 blocks: rows 4*(l/16) .. +3 of
    // column l%16; 32 x 32 blocks: four such runs per block).  FP8 scales:
    // the stored codes are x*s, so the product is divided by s_row * s_col
    // (powers of two, applied one factor at a time: exact).
    const float alpha = P.alpha, beta = P.beta;
    const int64_t r0w = x0a + wm * WT, c0w = x0b + wn * WT;
    const bool c_in = x0a + MT <= P.M && x0b + MT <= P.N;
    if (MT == 128 && NS > 1) {
        // Split k: the slice's product, with the FP8 scales applied (exact),
        // goes to its own column-major M x N binary32 plane; a second kernel
        // sums the planes in slice order and applies alpha, beta and C.
        float* pp = P.part + (int64_t)slice * P.M * P.N;
        const bool vec = c_in && P.M % 4 == 0;
        MM::pieces(acc, lane, [&](f4 v, int di, int dj) {
            const int64_t i0 = r0w + di, j = c0w + dj;
            float ib = 1.f;
            if (FORM == kMxFP8 && P.b_scale != nullptr && j < P.N) ib = 1.f / P.b_scale[j];
            u4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float t = v[r];
                if (FORM == kMxFP8 && P.a_scale != nullptr && i0 + r < P.M)
                    t = t * (1.f / P.a_scale[i0 + r]);
                o[r] = __float_as_uint(t * ib);
            }
            float* cp = pp + j * P.M;
            if (vec) {
                *reinterpret_cast<u4a*>(cp + i0) = o;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (i0 + r < P.M && j < P.N) cp[i0 + r] = __uint_as_float(o[r]);
            }
        });
        return;
    }
    MM::pieces(acc, lane, [&](f4 v, int di, int dj) {
        const int64_t i0 = r0w + di, j = c0w + dj;
        float ib = 1.f;
        if (FORM == kMxFP8 && P.b_scale != nullptr && j < P.N) ib = 1.f / P.b_scale[j];
        if (P.c_bf16) {
            uint16_t* cp = reinterpret_cast<uint16_t*>(P.C) + j * P.ldc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r;
                if (c_in || (i < P.M && j < P.N)) {
                    float t = v[r];
                    if (FORM == kMxFP8 && P.a_scale != nullptr) t = t * (1.f / P.a_scale[i]);
                    t = t * ib;
                    const float c = beta != 0.f ? bf16_float(cp[i]) : 0.f;
                    const float o = beta != 0.f ? axpby(alpha, t, beta, c) : alpha * t;
                    cp[i] = (uint16_t)bf16_bits(o);
                }
            }
        } else {
            float* cp = reinterpret_cast<float*>(P.C) + j * P.ldc;
            if (c_in) {
                f4 c = f4{0.f, 0.f, 0.f, 0.f};
                if (beta != 0.f) {
                    const u4 cu = *reinterpret_cast<const u4a*>(cp + i0);
                    c = f4{__uint_as_float(cu[0]), __uint_as_float(cu[1]),
                           __uint_as_float(cu[2]), __uint_as_float(cu[3])};
                }
                u4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float t = v[r];
                    if (FORM == kMxFP8 && P.a_scale != nullptr) t = t * (1.f / P.a_scale[i0 + r]);
                    t = t * ib;
                    o[r] = __float_as_uint(beta != 0.f ? axpby(alpha, t, beta, c[r]) : alpha * t);
                }
                *reinterpret_cast<u4a*>(cp + i0) = o;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = i0 + r;
                    if (i < P.M && j < P.N) {
                        float t = v[r];
                        if (FORM == kMxFP8 && P.a_scale != nullptr) t = t * (1.f / P.a_scale[i]);
                        t = t * ib;
                        cp[i] = beta != 0.f ? axpby(alpha, t, beta, cp[i]) : alpha * t;
                    }
                }
            }
        }
    });
}

// Standalone pack of both operands into copy 0 (pack-then-compute baseline):
// one chunk per workgroup, same registers and stores as a producer.
template <int FORM, int MT, bool AKC, bool BKC>
__global__ void __launch_bounds__(NTHR) pack_mx_kernel(const MxParams P)
{
    typedef Geo<FORM, MT> G;
    typedef typename Form<FORM>::S S;
    const int tid = threadIdx.x;
    const int nK = P.nK;
    const int64_t nA = (int64_t)P.tilesM * nK;
    const int64_t b = blockIdx.x;
    if (b < nA) {
        const int64_t t = b / nK, q = b % nK;
        Stage<FORM, AKC, MT> r;
        r.load_edge(reinterpret_cast<const S*>(P.A), P.a_ld, P.M, P.K, t * MT, q * G::KT, tid);
        r.store_pack(P.apack + (t * nK + q) * G::PACK_CHUNK, tid);
    } else {
        const int64_t bb = b - nA;
        const int64_t t = bb / nK, q = bb % nK;
        Stage<FORM, BKC, MT> r;
        r.load_edge(reinterpret_cast<const S*>(P.B), P.b_ld, P.N, P.K, t * MT, q * G::KT, tid);
        r.store_pack(P.bpack + (t * nK + q) * G::PACK_CHUNK, tid);
    }
}

// Second half of a split-k call: C = alpha * (sum of the slice planes, in
// slice order 0, 1, ...) + beta * C with the tile kernel's epilogue rounding
// (C not read when beta == 0).  One thread per C element, column by column.
__global__ void __launch_bounds__(256) splitk_reduce_mx_kernel(const float* __restrict__ part,
                                                               int S, int64_t M, int64_t N,
                                                               char* C, int c_bf16, int64_t ldc,
                                                               float alpha, float beta)
{
    const int64_t MN = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < MN;
         idx += (int64_t)gridDim.x * 256) {
        float v = part[idx];
        for (int sl = 1; sl < S; ++sl) v = v + part[(int64_t)sl * MN + idx];
        const int64_t i = idx % M, j = idx / M;
        if (c_bf16) {
            uint16_t* cp = reinterpret_cast<uint16_t*>(C) + i + j * ldc;
            const float o = beta != 0.f ? axpby(alpha, v, beta, bf16_float(*cp)) : alpha * v;
            *cp = (uint16_t)bf16_bits(o);
        } else {
            float* cp = reinterpret_cast<float*>(C) + i + j * ldc;
            *cp = beta != 0.f ? axpby(alpha, v, beta, *cp) : alpha * v;
        }
    }
}

unsigned grid_for(int64_t total)
{
    int64_t b = (total + 255) / 256;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    return (unsigned)b;
}

MxParams make_mx_params(const MxLaunchDesc& d, int MT)
{
    const int KT = mx_kt(d.form), SB = mx_src_bytes(d.form);
    MxParams P{};
    P.A = static_cast<const char*>(d.A);
    P.B = static_cast<const char*>(d.B);
    P.C = static_cast<char*>(d.C);
    P.a_ld = d.a_ld; P.b_ld = d.b_ld; P.ldc = d.ldc;
    P.M = d.M; P.N = d.N; P.K = d.K;
    P.alpha = d.alpha; P.beta = d.beta;
    P.a_scale = d.a_scale; P.b_scale = d.b_scale;
    P.apack = static_cast<char*>(d.apack); P.bpack = static_cast<char*>(d.bpack);
    P.apack_copy = d.apack_copy_bytes; P.bpack_copy = d.bpack_copy_bytes;
    P.aflag = d.aflag; P.bflag = d.bflag; P.aclaim = d.aclaim; P.bclaim = d.bclaim;
    P.stats = d.stats_ptr;
    P.epoch = d.epoch;
    P.tilesM = (int)((d.M + MT - 1) / MT);
    P.tilesN = (int)((d.N + MT - 1) / MT);
    P.nK = (int)((d.K + KT - 1) / KT);
    P.group_m = kGroupM;
    P.mode = d.mode; P.pack_a = d.pack_a; P.pack_b = d.pack_b;
    P.a_pack_from = d.a_pack_from; P.b_pack_from = d.b_pack_from;
    P.shared_copy = d.shared_copy;
    P.no_publish = d.no_publish; P.do_stats = d.stats && d.stats_ptr != nullptr;
    P.order = d.order;
    // vector loads of the unpacked operand need every 4-byte group of a
    // micro-block row (K-major) or column (MN-major) dword aligned: the base
    // and the leading dimension in bytes must be multiples of 4
    P.a_vec = ((uintptr_t)d.A % 4 == 0) && ((d.a_ld * SB) % 4 == 0);
    P.b_vec = ((uintptr_t)d.B % 4 == 0) && ((d.b_ld * SB) % 4 == 0);
    P.c_bf16 = d.c_bf16;
    P.split = d.split > 1 ? d.split : 1;
    P.slice_ksteps = d.split > 1 ? d.slice_ksteps : P.nK;
    P.part = static_cast<float*>(d.part);
    return P;
}

template <int FORM, int MT>
hipError_t launch_form(const MxLaunchDesc& d, bool pack)
{
    const MxParams P = make_mx_params(d, MT);
    const bool akc = d.a_kmajor, bkc = d.b_kmajor;
    const dim3 block(NTHR);
    if (!pack) {
        // split k runs on the 128 tile only, with every slice non-empty
        if (P.split > 1 && (MT != 128 || P.part == nullptr || P.slice_ksteps < 1 ||
                            (int64_t)(P.split - 1) * P.slice_ksteps >= P.nK))
            return hipErrorInvalidValue;
        const dim3 grid((unsigned)((int64_t)P.tilesM * P.tilesN * P.split));
        if (!akc && !bkc) gemm_mx_kernel<FORM, MT, false, false><<<grid, block, 0, d.stream>>>(P);
        else if (!akc && bkc) gemm_mx_kernel<FORM, MT, false, true><<<grid, block, 0, d.stream>>>(P);
        else if (akc && !bkc) gemm_mx_kernel<FORM, MT, true, false><<<grid, block, 0, d.stream>>>(P);
        else gemm_mx_kernel<FORM, MT, true, true><<<grid, block, 0, d.stream>>>(P);
        if (P.split > 1) {
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            splitk_reduce_mx_kernel<<<dim3(grid_for(d.M * d.N)), dim3(256), 0, d.stream>>>(
                P.part, P.split, d.M, d.N, P.C, P.c_bf16, d.ldc, P.alpha, P.beta);
        }
    } else {
        const dim3 grid((unsigned)(((int64_t)P.tilesM + P.tilesN) * P.nK));
        if (!akc && !bkc) pack_mx_kernel<FORM, MT, false, false><<<grid, block, 0, d.stream>>>(P);
        else if (!akc && bkc) pack_mx_kernel<FORM, MT, false, true><<<grid, block, 0, d.stream>>>(P);
        else if (akc && !bkc) pack_mx_kernel<FORM, MT, true, false><<<grid, block, 0, d.stream>>>(P);
        else pack_mx_kernel<FORM, MT, true, true><<<grid, block, 0, d.stream>>>(P);
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace fip
