// Batched GEMM of many independent, unevenly sized binary32 problems in one
// persistent launch (gfx950).
//
// Every problem is cut into C tiles of the class the planner chose for it
// (64 x 64 or 32 x 32, picked per problem by the autotuned size threshold).
// The planner lists all tiles of all problems, longest first (LPT: k times
// tile area), a problem's tiles next to each other so that the workgroups
// running them concurrently share its panels in L2.  A grid of resident
// workgroups takes tiles from that list by atomic ticket until it runs out,
// so the batch costs one launch whatever the problem count.  The last
// workgroup to finish resets the ticket counters, which makes the launch
// replayable (as a graph node) with no clearing step.
//
// Packing: each problem follows the paper's Sec. 3.3 rule as refined for the
// GPU: a panel is worth packing only if a later pass reads it after the first
// finished.  A problem's tiles sit together in the list and run concurrently,
// so no tile of this workload starts after another finished with the same
// panel; every tile therefore takes the unpacked (SUP, Sec. 2.3) path, with
// the same loaders, LDS staging and MFMA microkernel as the fused-pack kernel.
#include "fip_internal.h"
#include "fip_device.h"
#include "fip_tile.h"

namespace fip {
namespace {

constexpr int VB_NTHR = 256;   // 2 x 2 waves
constexpr int VB_KT = 32;

struct VbParams {
    const VbProblem* probs;
    const VbItem* items;
    int64_t total;
    const float* const* A; const int64_t* lda;
    const float* const* B; const int64_t* ldb;
    float* const* C; const int64_t* ldc;
    float alpha, beta;
    int no_ab;          // alpha == 0: A and B are not read (C := beta*C)
    uint32_t* ticket;   // [0]: next item, [1]: finished workgroups
};

// LDS of the largest tile class (64 x 64): two buffers of each operand in the
// larger of the two orientations.
template <int MT>
struct VbLds {
    static constexpr int A_ELEMS = Chunk<float, MT, VB_KT, VB_NTHR, false>::LDS_ELEMS >
                                           Chunk<float, MT, VB_KT, VB_NTHR, true>::LDS_ELEMS
                                       ? Chunk<float, MT, VB_KT, VB_NTHR, false>::LDS_ELEMS
                                       : Chunk<float, MT, VB_KT, VB_NTHR, true>::LDS_ELEMS;
    static constexpr int FLOATS = 4 * A_ELEMS;
};

// One MT x MT tile of one problem (kernel terms: C column-major M x N; A-side
// element (x, p) at A[x + p*lda] (MN-major) or A[x*lda + p] (K-major)).
template <int MT, bool AKC, bool BKC>
__device__ __forceinline__ void vb_tile(const float* __restrict__ A, int64_t lda,
                                        const float* __restrict__ B, int64_t ldb,
                                        float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                        int tm, int tn, float alpha, float beta, float* lds)
{
    constexpr int KT = VB_KT, NTHR = VB_NTHR;
    typedef Chunk<float, MT, KT, NTHR, AKC> ChA;
    typedef Chunk<float, MT, KT, NTHR, BKC> ChB;
    constexpr int WT = MT / 2, FB = WT / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    float* sA[2] = {lds, lds + ChA::LDS_ELEMS};
    float* sB[2] = {lds + 2 * ChA::LDS_ELEMS, lds + 2 * ChA::LDS_ELEMS + ChB::LDS_ELEMS};
    const int64_t x0a = (int64_t)tm * MT, x0b = (int64_t)tn * MT;
    const int nK = (K + KT - 1) / KT, nKfull = K / KT;

    // interior chunks: one vector load per register vector at loop-invariant
    // 32-bit offsets (problems are at most a few thousand on a side)
    const bool a_al = ((uintptr_t)A & 3) == 0, b_al = ((uintptr_t)B & 3) == 0;
    const int64_t a_span = (AKC ? MT * lda + KT : MT + KT * lda) * (int64_t)sizeof(float);
    const int64_t b_span = (BKC ? MT * ldb + KT : MT + KT * ldb) * (int64_t)sizeof(float);
    const bool a_in = x0a + MT <= M && a_al && a_span < ((int64_t)1 << 31);
    const bool b_in = x0b + MT <= N && b_al && b_span < ((int64_t)1 << 31);
    const char* a_org = reinterpret_cast<const char*>(A + (AKC ? x0a * lda : x0a));
    const char* b_org = reinterpret_cast<const char*>(B + (BKC ? x0b * ldb : x0b));
    const int64_t a_step = (AKC ? KT : KT * lda) * (int64_t)sizeof(float);
    const int64_t b_step = (BKC ? KT : KT * ldb) * (int64_t)sizeof(float);
    uint32_t a_off[ChA::NV], b_off[ChB::NV];
#pragma unroll
    for (int i = 0; i < ChA::NV; ++i) a_off[i] = ChA::fast_offset(i, tid, lda);
#pragma unroll
    for (int i = 0; i < ChB::NV; ++i) b_off[i] = ChB::fast_offset(i, tid, ldb);

    ChA ra;
    ChB rb;
    auto load = [&](int c) {
        if (a_in && c < nKfull) ra.load_at(a_org + (int64_t)c * a_step, a_off);
        else ra.load_edge(A, lda, M, K, x0a, (int64_t)c * KT, a_al, tid);
        if (b_in && c < nKfull) rb.load_at(b_org + (int64_t)c * b_step, b_off);
        else rb.load_edge(B, ldb, N, K, x0b, (int64_t)c * KT, b_al, tid);
    };

    f4 acc[FB][FB];
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    load(0);
    ra.store_lds(sA[0], tid);
    rb.store_lds(sB[0], tid);
    __syncthreads();
    for (int q = 0; q < nK; ++q) {
        const int cur = q & 1;
        const bool more = q + 1 < nK;
        if (more) load(q + 1);
        const float* la = sA[cur] + ChA::lds_at(wm * WT + (lane & 15), lane >> 4);
        const float* lb = sB[cur] + ChB::lds_at(wn * WT + (lane & 15), lane >> 4);
#pragma unroll
        for (int s = 0; s < KT / 4; ++s) {
            float af[FB], bf[FB];
#pragma unroll
            for (int a = 0; a < FB; ++a) af[a] = la[ChA::lds_at(a * 16, 4 * s)];
#pragma unroll
            for (int b = 0; b < FB; ++b) bf[b] = lb[ChB::lds_at(b * 16, 4 * s)];
#pragma unroll
            for (int a = 0; a < FB; ++a)
#pragma unroll
                for (int b = 0; b < FB; ++b) acc[a][b] = mfma16(af[a], bf[b], acc[a][b]);
        }
        if (more) {
            ra.store_lds(sA[cur ^ 1], tid);
            rb.store_lds(sB[cur ^ 1], tid);
        }
        __syncthreads();
    }

    // epilogue: item r of lane l of block (a, b) is C[4*(l/16) + r][l%16]
    const int64_t r0 = x0a + wm * WT, c0 = x0b + wn * WT;
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) {
            const int64_t i0 = r0 + a * 16 + 4 * (lane >> 4), j = c0 + b * 16 + (lane & 15);
            if (j >= N) continue;
            float* cp = C + j * ldc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r;
                if (i < M)
                    cp[i] = beta != 0.f ? axpby(alpha, acc[a][b][r], beta, cp[i])
                                        : alpha * acc[a][b][r];
            }
        }
}

template <int MT>
__device__ __forceinline__ void vb_dispatch(int kmaj, const float* A, int64_t lda, const float* B,
                                            int64_t ldb, float* C, int64_t ldc, int M, int N,
                                            int K, int tm, int tn, float alpha, float beta,
                                            float* lds)
{
    switch (kmaj) {
    case 0: vb_tile<MT, false, false>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta, lds); break;
    case 1: vb_tile<MT, true, false>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta, lds); break;
    case 2: vb_tile<MT, false, true>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta, lds); break;
    default: vb_tile<MT, true, true>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta, lds); break;
    }
}

__global__ void __launch_bounds__(VB_NTHR) vbatched_kernel(const VbParams P)
{
    __shared__ __attribute__((aligned(16))) float lds[VbLds<64>::FLOATS];
    __shared__ int64_t s_item;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = (int64_t)atomicAdd(P.ticket, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();  // every thread has its ticket before thread 0 takes the next
        if (item >= P.total) break;
        const VbItem it = P.items[item];
        const VbProblem pr = P.probs[it.prob];
        const bool sw = pr.flags & kVbSwapped;
        // kernel A-side: the caller's A, or op(B)^T for a swapped (row-major) problem
        const float* A = sw ? P.B[it.prob] : P.A[it.prob];
        const float* B = sw ? P.A[it.prob] : P.B[it.prob];
        const int64_t lda = sw ? P.ldb[it.prob] : P.lda[it.prob];
        const int64_t ldb = sw ? P.lda[it.prob] : P.ldb[it.prob];
        const int kmaj = (pr.flags & kVbAKmajor ? 1 : 0) | (pr.flags & kVbBKmajor ? 2 : 0);
        const int K = P.no_ab ? 0 : pr.K;
        if (pr.cls == 1)
            vb_dispatch<64>(kmaj, A, lda, B, ldb, P.C[it.prob], P.ldc[it.prob], pr.M, pr.N, K,
                            it.tm, it.tn, P.alpha, P.beta, lds);
        else
            vb_dispatch<32>(kmaj, A, lda, B, ldb, P.C[it.prob], P.ldc[it.prob], pr.M, pr.N, K,
                            it.tm, it.tn, P.alpha, P.beta, lds);
    }
    // The last workgroup out resets the counters for the next launch on the
    // stream: every workgroup has taken its final ticket before it counts
    // itself finished.
    if (tid == 0) {
        const uint32_t done = atomicAdd(P.ticket + 1, 1u);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(P.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(P.ticket + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void __launch_bounds__(64) vb_zero_kernel(uint32_t* ticket)
{
    if (threadIdx.x < 2) ticket[threadIdx.x] = 0u;
}

VbParams make_vb_params(const VbLaunchDesc& d)
{
    VbParams P{};
    P.probs = d.probs; P.items = d.items; P.total = d.total;
    P.A = d.A; P.lda = d.lda; P.B = d.B; P.ldb = d.ldb; P.C = d.C; P.ldc = d.ldc;
    P.alpha = d.alpha; P.beta = d.beta;
    P.no_ab = d.alpha == 0.f;
    P.ticket = d.ticket;
    return P;
}

}  // namespace

int vbatched_grid()
{
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, cus = 256, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, vbatched_kernel, VB_NTHR, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    return grid;
}

hipError_t launch_vbatched(const VbLaunchDesc& d)
{
    const VbParams P = make_vb_params(d);
    int64_t g = vbatched_grid();
    if (g > d.total) g = d.total;
    if (g < 1) return hipSuccess;
    vbatched_kernel<<<dim3((unsigned)g), dim3(VB_NTHR), 0, d.stream>>>(P);
    return hipGetLastError();
}

hipError_t launch_vb_zero(uint32_t* ticket, hipStream_t stream)
{
    vb_zero_kernel<<<dim3(1), dim3(64), 0, stream>>>(ticket);
    return hipGetLastError();
}

// A graph of one kernel node running the batch (the counters reset themselves).
hipError_t build_vbatched_graph(const VbLaunchDesc& d, hipGraphExec_t* exec)
{
    VbParams P = make_vb_params(d);
    int64_t g = vbatched_grid();
    if (g > d.total) g = d.total;
    if (g < 1) g = 1;
    hipGraph_t graph = nullptr;
    hipError_t e = hipGraphCreate(&graph, 0);
    if (e != hipSuccess) return e;
    hipKernelNodeParams kp{};
    void* args[] = {&P};
    kp.func = reinterpret_cast<void*>(vbatched_kernel);
    kp.gridDim = dim3((unsigned)g);
    kp.blockDim = dim3(VB_NTHR);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, graph, nullptr, 0, &kp);
    if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e;
}

}  // namespace fip
