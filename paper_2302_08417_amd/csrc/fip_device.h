// Device helpers shared by the tile kernels (fipgemm_kernels.hip,
// fipgemm_mx.hip): XCD identity, memory completion, tile order, epilogue
// rounding.  Internal; included only by HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fip {
namespace {

// alpha*x + beta*y with one fixed rounding sequence (alpha*x rounded, then one
// fused multiply-add), written out so that no tile shape's code generation can
// contract it differently: every kernel variant then rounds C identically.
__device__ __forceinline__ double axpby(double alpha, double x, double beta, double y)
{
    return __builtin_fma(beta, y, alpha * x);
}
__device__ __forceinline__ float axpby(float alpha, float x, float beta, float y)
{
    return __builtin_fmaf(beta, y, alpha * x);
}

// Hardware id of the XCD (XCC) running this wave: hwreg XCC_ID, bits [3:0].
__device__ __forceinline__ unsigned xcc_id()
{
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));
}

// Wait until every memory operation this wave issued has completed; for
// global stores that means the XCD's L2 has acknowledged them.
__device__ __forceinline__ void wait_all_memory()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Workgroup -> tile (also replayed on the host by the planner to see which
// panels a later round reads).  Workgroups are dispatched round-robin over the 8 XCDs,
// so w % 8 is (normally) the XCD.  Each XCD gets one contiguous run of a
// grouped tile order: bands of GROUP_M tile rows, swept column by column.
// That keeps the tiles running together on an XCD compact for its L2 and most
// of the panels an XCD packs private to it.
//   order 0: inside a band, the GROUP_M tiles of one column are consecutive;
//   order 1: inside a band, consecutive tiles take distinct columns (round r,
//            slot s -> column s, row (s + r) mod GROUP_M), so the first round of
//            workgroups touches every column panel of the band once and later
//            rounds find them all packed.
__host__ __device__ inline void tile_coords(int w, int tilesM, int tilesN, int group_m, int order,
                                            int& tm, int& tn)
{
    const int T = tilesM * tilesN;
    const int xcd = w & 7, local = w >> 3;
    const int q = T >> 3, rr = T & 7;
    const int t = xcd * q + (xcd < rr ? xcd : rr) + local;
    const int per_group = group_m * tilesN;
    const int g = t / per_group;
    const int first_m = g * group_m;
    const int gsize = tilesM - first_m < group_m ? tilesM - first_m : group_m;
    const int rem = t - g * per_group;
    if (order == 0) {
        tm = first_m + rem % gsize;
        tn = rem / gsize;
    } else {
        const int round = rem / tilesN, slot = rem - round * tilesN;
        tn = slot;
        tm = first_m + (slot + round) % gsize;
    }
}

}  // namespace
}  // namespace fip
