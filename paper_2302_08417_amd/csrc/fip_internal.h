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
    uint64_t* aflag; uint64_t* bflag;   // panel complete: [copies][tiles]
    uint64_t* aclaim; uint64_t* bclaim; // [copies][tiles]
    unsigned long long* stats_ptr;      // 4 counters
    uint64_t epoch;                     // unique per fused call in this process
    hipStream_t stream;
};

// Enqueue the fused-pack tile kernel.  Returns a hipError_t.
hipError_t launch_gemm(const LaunchDesc& d);
// Enqueue the standalone pack of both operands into copy 0 (pack-then-compute).
hipError_t launch_pack(const LaunchDesc& d);
// Enqueue C := beta*C (beta == 0 writes zeros without reading C).
hipError_t launch_scale(int elem, int64_t M, int64_t N, void* C, int64_t ldc, double beta,
                        hipStream_t stream);

// Enqueue the XCC-id diagnostic (one 64-thread workgroup per entry).
hipError_t launch_xcc_map(uint32_t* out, int64_t nblocks, hipStream_t stream);

}  // namespace fip
