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

// The publish protocol of a packed panel (paper Sec. 3.5: the one synchronisation).
// Producer: every thread waits for its pack stores (wait_all_memory), the
// workgroup meets at a barrier, then one thread stores the epoch into the
// panel's flag with release semantics at agent scope.  Consumer: a relaxed
// agent-scope flag load; the first time a wave sees the epoch it issues one
// acquire fence at agent scope before its first load of the packed copy.
// Producer and consumers of a copy run on one XCD, but the HIP memory model
// has no XCD scope, so both sides use agent scope (an L2 write-back on
// publish, an L1 invalidate on acquire: once per panel and once per wave).
__device__ __forceinline__ void publish_flag(uint64_t* flag, uint64_t epoch)
{
    __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t peek_flag(const uint64_t* flag)
{
    return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void acquire_packed() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Workgroup -> tile (also replayed on the host by the planner to see which
// panels a later round reads).  Workgroups are dispatched round-robin over the 8 XCDs,
// so w % 8 is (normally) the XCD.  Each XCD gets one contiguous run of a
// grouped tile order: bands of GROUP_M tile rows, swept column by column.
// That keeps the tiles running together on an XCD compact for its L2 and most
// of the panels an XCD packs private to it.
//   order 0: inside a band, the GROUP_M tiles of one column are consecutive;
//   order 1: inside a band, consecutive tiles take distinct columns (round r,
//            slot s -> column (s + rot) mod tilesN, row (s + r) mod GROUP_M), so
//            the first round of workgroups touches every column panel of the
//            band once and later rounds find them all packed.  rot staggers the
//            bands' sweeps by the XCD whose run starts the band (band start *
//            8 / tiles, times tilesN / 8): the XCDs start on different bands, so
//            with one pack copy shared by all XCDs the workgroups running at
//            once spread over the column panels instead of all XCDs reading the
//            same unpublished ones.  A band keeps one rotation, so the map stays
//            one-to-one.
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
        const int64_t starter = ((int64_t)g * per_group * 8) / T;   // 0..7
        const int rot = (int)((starter * tilesN) >> 3);
        tn = slot + rot < tilesN ? slot + rot : slot + rot - tilesN;
        tm = first_m + (slot + round) % gsize;
    }
}

}  // namespace
}  // namespace fip
