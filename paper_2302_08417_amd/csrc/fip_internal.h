// Internal interface between the C-ABI host layer (fipgemm_api.cpp) and the
// HIP kernels (fipgemm_kernels.hip).  Not installed; no torch types anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fip {

// One copy of every packed panel per XCD (MI355X: 8 XCDs, each with its own
// L2).  A packed chunk is only ever written and read by workgroups of the same
// XCD inside one launch, so the XCD's L2 is the single point of coherence.
constexpr int kCopies = 8;

enum Mode : int32_t {
    kModeFused = 0,        // pack on first touch, later passes read packed
    kModeConsumePacked = 1,// every chunk read from copy 0 (written by fip_pack)
    kModeUnpacked = 2,     // never pack
};

// Operations the FP64/FP32 tile kernel runs (LaunchDesc::kind).
enum Kind : int32_t {
    kGemm = 0,   // C := alpha op(A) op(B) + beta C
    kSyrk = 1,   // one triangle of alpha op(A) op(A)^T + beta C: the tiles of that
                 // triangle only; A and B sides are the same operand sharing one pack
    kTrmm = 2,   // C := alpha op(T) B + beta C or alpha B op(T) + beta C, T triangular:
                 // one side's chunks masked to the triangle, its zero k-steps skipped
    k1m = 3,     // complex C := alpha op(A) op(B) + beta C through the 1m method: the
                 // real product of the 2M x 2K expansion of the A side and the 2K x N
                 // expansion of the B side is the real view of column-major complex C
    kGemmDma = 4,  // (kernel variant of kGemm, chosen at launch) chunks fetched with
                   // direct global -> LDS loads
};

// Tile rows per band of the XCD-aware tile order (see tile_coords).
constexpr int kGroupM = 8;

// Tile classes: C tile MT x NT, k-step KT (KT depends on the element type).
constexpr int kNumTileClasses = 3;
inline int tile_mt(int cls) { return cls == 0 ? 128 : cls == 1 ? 64 : 32; }
inline int tile_kt(int cls, int elem) { (void)cls; return elem == 8 ? 16 : 32; }

// One launch of the tile kernel, in kernel terms: C is column-major M x N
// (C[x_a + x_b*ldc]); A-side element (x_a, p) at A[x_a*a_smn + p*a_sk];
// B-side element (x_b, p) at B[x_b*b_smn + p*b_sk].  A K-major operand has
// s_k = 1, an MN-major one s_mn = 1 (the host swaps operands for row-major C).
struct LaunchDesc {
    int elem;              // 8 (binary64) or 4 (binary32)
    int tile_class;
    int mode;              // Mode
    int pack_a, pack_b;    // fused mode: operand packed on first touch
    int a_pack_from, b_pack_from;  // ... from this tile row / column on (0: every panel)
    int shared_copy;       // 1: one pack copy shared by all XCDs, else one per XCD
    int no_publish, stats;
    int order;             // tile order inside an XCD's run (0 grouped, 1 rounds)
    int64_t M, N, K;
    const void* A; int64_t a_smn, a_sk; int a_kmajor;
    const void* B; int64_t b_smn, b_sk; int b_kmajor;
    void* C; int64_t ldc;
    double alpha, beta;
    // workspace pieces (device pointers; null when unused)
    void* apack; int64_t apack_copy_elems;
    void* bpack; int64_t bpack_copy_elems;
    uint64_t* aflag; uint64_t* bflag;   // panel complete: [copies][tiles][split]
    uint64_t* aclaim; uint64_t* bclaim; // [copies][tiles][split]
    unsigned long long* stats_ptr;      // 4 counters
    uint64_t epoch;                     // unique per fused call in this process
    // split k: `split` slices of `slice_ksteps` k-steps each (split = 1: none)
    int split, slice_ksteps;
    void* part;                         // slice partials [split][N][M] (column-major)
    // level-3 operations other than GEMM (Kind), in kernel terms
    int kind;
    int tri_upper;     // SYRK: the stored triangle of kernel C is row <= column
    int tri_side;      // TRMM: 1 = the kernel's A side is triangular, 2 = the B side
    int tri_keep_ge;   // TRMM: the triangular side keeps element (x, p) with x >= p (else x <= p)
    int tri_unit;      // TRMM: unit diagonal
    // k1m (complex): M and K above are the real extents 2m' and 2k' of the
    // expanded operands, A, B and C point at (re, im) pairs, the operand strides
    // and ldc count complex elements; alpha and beta above are the real parts
    double alpha_im, beta_im;
    int conj_a, conj_b;   // the kernel side reads conj(X)
    // GEMM: launches in which no tile produces a pack and every chunk can be
    // fetched whole run the kernel variant that loads chunks with direct
    // global -> LDS loads instead of through registers
    int dma;
    int* used_dma;     // out (nullable): whether the launch ran that variant
    hipStream_t stream;
};

// hipGetLastError also reports non-sticky errors left by any earlier runtime
// call in the process (another library's query, say); each launcher clears
// them first, so the status it returns after its launches is its own.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Enqueue the fused-pack tile kernel.  Returns a hipError_t.
hipError_t launch_gemm(const LaunchDesc& d);
// Enqueue the standalone pack of both operands into copy 0 (pack-then-compute).
hipError_t launch_pack(const LaunchDesc& d);
// Enqueue C := beta*C (beta == 0 writes zeros without reading C).
hipError_t launch_scale(int elem, int64_t M, int64_t N, void* C, int64_t ldc, double beta,
                        hipStream_t stream);

// ---- Triangular solve: diagonal blocks (fipgemm_trsm.hip) --------------------
// Rows of the largest diagonal block the blocked TRSM solves directly.
constexpr int kTrsmBlock = 64;
// Solve S x = alpha b in place for nrhs right-hand sides b (element e of
// right-hand side v at B[e*s_e + v*s_v]), S the nb x nb (nb <= kTrsmBlock)
// triangle with S(r, c) = A[r + c*lda] (s_trans = 0) or A[c + r*lda], lower
// or upper, unit diagonal (not read) or not.
struct TrsmBlockDesc {
    int elem;
    const void* A; int64_t lda;
    int s_trans, s_lower, unit, nb;
    void* B; int64_t s_e, s_v, nrhs;
    double alpha;
    hipStream_t stream;
};
hipError_t launch_trsm_block(const TrsmBlockDesc& d);

// ---- Mixed-precision forms (fipgemm_mx.hip) --------------------------------
// Operands stored as bfloat16 or FP8 E4M3, or binary32 split into bfloat16
// terms while packing; binary32 accumulation; C binary32 or bfloat16.
enum MxForm : int32_t {
    kMxBF16 = 0,     // A, B bfloat16
    kMxFP8 = 1,      // A, B E4M3 with optional per-row / per-column scales
    kMxX3 = 2,       // A, B binary32, three bfloat16 terms, six products
    kMxX3Fast = 3,   // A, B binary32, two bfloat16 terms, three products
};
constexpr int kMxTile = 128;                     // C tile 128 x 128, 2 x 2 waves
constexpr int kMxTileBig = 256;                  // bfloat16, E4M3: 128 x 128 per wave
inline int mx_kt(int form) { return form == kMxBF16 ? 64 : form == kMxFP8 ? 128 : 32; }
inline int mx_planes(int form) { return form == kMxX3 ? 3 : form == kMxX3Fast ? 2 : 1; }
inline int mx_src_bytes(int form) { return form == kMxBF16 ? 2 : form == kMxFP8 ? 1 : 4; }
inline int mx_pack_bytes(int form) { return form == kMxFP8 ? 1 : 2; }  // per plane element
// Workgroups of one mixed-precision tile kernel that fit on a CU (LDS-bound).
inline int mx_per_cu(int form, int mt) { return mt == 128 && (form == kMxBF16 || form == kMxFP8) ? 2 : 1; }
inline bool mx_has_big(int form) { return form == kMxBF16 || form == kMxFP8; }
// Forms whose planner default is the 256 tile once a call fills the device
// with 256-tiles (E4M3 measures faster on the 128 tile, two per CU).
inline bool mx_big_default(int form) { return form == kMxBF16; }

struct MxLaunchDesc {
    int form;              // MxForm
    int mt;                // tile extent: 128, or 256 (bfloat16 only)
    int mode;              // Mode
    int pack_a, pack_b, no_publish, stats, order;
    int a_pack_from, b_pack_from;  // first packed tile row / column (0: every panel)
    int shared_copy;               // 1: one pack copy for all XCDs
    int c_bf16;            // C stored as bfloat16 (else binary32)
    int64_t M, N, K;       // kernel terms (C column-major M x N)
    const void* A; int64_t a_ld; int a_kmajor;   // element (x, p): K-major X[x*ld + p],
    const void* B; int64_t b_ld; int b_kmajor;   //   MN-major X[x + p*ld]
    void* C; int64_t ldc;
    float alpha, beta;
    const float* a_scale;  // per kernel row (null = 1); FP8 only
    const float* b_scale;  // per kernel column (null = 1); FP8 only
    void* apack; int64_t apack_copy_bytes;
    void* bpack; int64_t bpack_copy_bytes;
    uint64_t* aflag; uint64_t* bflag; uint64_t* aclaim; uint64_t* bclaim;
    unsigned long long* stats_ptr;
    uint64_t epoch;
    // split k (128 tiles only): `split` slices of `slice_ksteps` k-steps each
    // (split = 1: none); binary32 slice partials [split][N][M] (column-major)
    int split, slice_ksteps;
    void* part;
    hipStream_t stream;
};

hipError_t launch_gemm_mx(const MxLaunchDesc& d);
// Standalone pack of both operands (copy 0) in the form's packed layout.
hipError_t launch_pack_mx(const MxLaunchDesc& d);
// The E4M3 256 x 256 tile (its own translation unit): GEMM (pack false) or
// standalone pack (pack true) launch.
hipError_t launch_mx_fp8_big(const MxLaunchDesc& d, bool pack);
// FP8 quantization of a binary32 matrix with power-of-two line scales.
hipError_t launch_quantize_fp8(int layout_col, int64_t rows, int64_t cols, const float* X,
                               int64_t ldx, int axis, uint8_t* Q, int64_t ldq, float* scales,
                               hipStream_t stream);
// C := beta*C for a binary32 or bfloat16 C (kernel terms).
hipError_t launch_scale_mx(int c_bf16, int64_t M, int64_t N, void* C, int64_t ldc, float beta,
                           hipStream_t stream);

// ---- Batched binary32 GEMM (fipgemm_batched.hip) ----------------------------
// One problem in kernel terms (C column-major M x N) and one tile of it.
enum VbFlags : int32_t { kVbAKmajor = 1, kVbBKmajor = 2, kVbSwapped = 4 };
struct VbProblem {
    int32_t M, N, K;
    int32_t flags;   // VbFlags: kernel A-/B-side K-major; swapped = row-major storage
    int32_t cls;     // tile class: 1 = 32 x 32, 2 = 16 x 16 (one wave per tile)
    int32_t pad[3];
};
struct VbItem {
    int32_t prob;
    uint16_t tm, tn;
};
struct VbLaunchDesc {
    unsigned long long* status;    // device: 1 + largest index of a skipped problem (0: none)
    const VbProblem* probs;        // device
    const VbItem* items;           // device: XCD x's items at [xcd_off[x], xcd_off[x+1])
    int64_t total;                 // number of items
    int64_t xcd_off[kCopies + 1];
    const float* const* A; const int64_t* lda;   // caller's device arrays
    const float* const* B; const int64_t* ldb;
    float* const* C; const int64_t* ldc;
    float alpha, beta;
    hipStream_t stream;
};
hipError_t launch_vbatched(const VbLaunchDesc& d);
hipError_t build_vbatched_graph(const VbLaunchDesc& d, hipGraphExec_t* exec);
int vbatched_grid();   // resident workgroups of the batched kernel on the device

// Scratch array of fip_dgemm_noalloc (fipgemm_scratch.hip): kScratchBytes of
// device memory per GPU, owned by the library for the life of the process.
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
// Device address of the current device's copy of the array (looked up once per
// device, with that device current).
hipError_t scratch_buffer(void** ptr);

// Enqueue the XCC-id diagnostic (one 64-thread workgroup per entry).
hipError_t launch_xcc_map(uint32_t* out, int64_t nblocks, hipStream_t stream);

}  // namespace fip
