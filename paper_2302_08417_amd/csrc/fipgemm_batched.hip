// Batched GEMM of many independent, unevenly sized binary32 problems in one
// persistent launch (gfx950).
//
// Every problem is cut into C tiles of the class the planner chose for it
// (32 x 32 or 16 x 16, picked per problem by the autotuned size threshold).
// The planner deals whole problems to the 8 XCDs, balancing their cost
// (longest problem first to the least loaded XCD), and lists each XCD's tiles
// longest first (k times tile area), a problem's tiles next to each other so
// that they share the XCD's L2.  The resident one-wave workgroups of an XCD
// walk its list in a static round-robin: no shared counter (a single global
// ticket serialises at the atomic unit, about one tile per 13 ns).  A wave owns a whole tile and reads its MFMA
// fragments straight from global memory (no LDS, no barriers): small
// problems are latency-bound, and this keeps as many independent tiles in
// flight per CU as registers allow.  Nothing in device memory changes between
// launches except C, so the launch replays as a graph node as it is.
//
// Packing: each problem follows the paper's Sec. 3.3 rule as refined for the
// GPU: a panel is worth packing only if a later pass reads it after the first
// finished.  A problem's tiles sit together in the list and run concurrently,
// so no tile of this workload starts after another finished with the same
// panel; every tile therefore takes the unpacked (SUP, Sec. 2.3) path.
#include "fip_internal.h"
#include "fip_device.h"
#include "fip_tile.h"

namespace fip {
namespace {

constexpr int VB_NTHR = 64;    // one wave per workgroup: a wave owns whole tiles

struct VbParams {
    unsigned long long* status;    // 1 + the largest index of a problem that was skipped
    const VbProblem* probs;
    const VbItem* items;
    int64_t total;
    int64_t xcd_off[kCopies + 1];  // items of XCD x: [xcd_off[x], xcd_off[x+1])
    const float* const* A; const int64_t* lda;
    const float* const* B; const int64_t* ldb;
    float* const* C; const int64_t* ldc;
    float alpha, beta;
    int no_ab;          // alpha == 0: A and B are not read (C := beta*C)
};

// A matrix viewed as a buffer resource: loads at byte offsets at or beyond
// `bytes` return zeros without touching memory, so fringe lanes need no
// branch (a branch per lane would also make the compiler wait for every
// outstanding load before the MFMAs).  Offsets are 32-bit: a problem whose
// storage reaches 2 GiB is not run (vb_valid).
struct Mat {
    __amdgpu_buffer_rsrc_t r;
    uint32_t bytes;
};
constexpr uint32_t kOob = 0x80000000u;   // an offset past any operand

// Bytes spanned by an MN x K operand (kc: K-major, X[x*ld + p]; else X[x + p*ld]).
__device__ __forceinline__ int64_t mat_span(int64_t ld, int64_t MN, int64_t K, bool kc)
{
    if (MN <= 0 || K <= 0) return 0;
    return (kc ? (MN - 1) * ld + K : (K - 1) * ld + MN) * (int64_t)sizeof(float);
}
// A problem the kernel can run: every leading dimension at least the extent it strides over,
// and every matrix it reads or writes below kMaxSpan bytes (32-bit buffer offsets).
constexpr int64_t kMaxSpan = 0x7FFFFFF0;
__device__ __forceinline__ bool vb_valid(int64_t lda, int64_t ldb, int64_t ldc, int M, int N,
                                         int K, bool akc, bool bkc)
{
    if (ldc < (M > 1 ? M : 1) || mat_span(ldc, M, N, false) > kMaxSpan) return false;
    if (K == 0) return true;   // A and B are not read
    const int64_t need_a = akc ? K : M, need_b = bkc ? K : N;
    return lda >= (need_a > 1 ? need_a : 1) && ldb >= (need_b > 1 ? need_b : 1) &&
           mat_span(lda, M, K, akc) <= kMaxSpan && mat_span(ldb, N, K, bkc) <= kMaxSpan;
}

__device__ __forceinline__ Mat make_mat(const float* X, int64_t ld, int64_t MN, int64_t K, bool kc)
{
    const int64_t n = mat_span(ld, MN, K, kc);   // <= kMaxSpan (vb_valid)
    Mat m;
    m.bytes = (uint32_t)n;
    m.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X), (short)0, (int)n, 0x00020000);
    return m;
}

// One operand's fragment rows for a wave: for each 16-row block a, lane
// (r, q) reads row x = x0 + 16a + r at k = 16j + 4q + t (t = 0..3) of k-block
// j.  Byte offsets are 32-bit (operands below 2 GiB, vb_valid), set up once per tile and
// advanced by a constant per k-block; lanes whose row or k lies outside the
// operand read at kOob and get zeros from the buffer unit, so the loads need
// no branch (a branch per lane would also make the compiler wait for every
// outstanding load before the MFMAs).
//   K-major (X(x, p) at X[x*ld + p]): one 16-byte vector per row; in the last,
//     partial k-block its elements past K hold whatever follows the row and
//     are zeroed when the block is used (masking at load time would make the
//     wave wait for the load right away).
//   MN-major (X[x + p*ld]): four elements, each contiguous with the
//     neighbouring lanes' rows.
template <int FB, bool KC>
struct Frag {
    Mat m;
    uint32_t off[FB];    // byte offset of this lane's (row, k = 4q) element
    bool row_ok[FB];
    uint32_t step;       // bytes per k-block
    uint32_t kstep;      // bytes between consecutive k (MN-major)

    __device__ __forceinline__ void init(const float* X, int64_t ld, int64_t MN, int64_t K,
                                         int64_t x0, int r, int q)
    {
        m = make_mat(X, ld, MN, K, KC);
        step = (uint32_t)(16 * (KC ? 1 : ld) * sizeof(float));
        kstep = (uint32_t)(ld * sizeof(float));
#pragma unroll
        for (int a = 0; a < FB; ++a) {
            const int64_t x = x0 + 16 * a + r;
            row_ok[a] = x < MN;
            off[a] = (uint32_t)((KC ? x * ld + 4 * q : x + 4 * q * ld) * (int64_t)sizeof(float));
        }
    }
    // k-block j; k0 = 16j + 4q is this lane's first k
    __device__ __forceinline__ void load(int j, int k0, int K, f4 (&v)[FB]) const
    {
        const uint32_t base = (uint32_t)j * step;
#pragma unroll
        for (int a = 0; a < FB; ++a) {
            if (KC) {
                const uint32_t o = (row_ok[a] && k0 < K) ? off[a] + base : kOob;
                v[a] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(m.r, o, 0, 0));
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t o = (row_ok[a] && k0 + t < K) ? off[a] + base + t * kstep : kOob;
                    v[a][t] = __builtin_bit_cast(float,
                                                 __builtin_amdgcn_raw_buffer_load_b32(m.r, o, 0, 0));
                }
            }
        }
    }
};

// One TM x TM tile of one problem, computed by a single wave straight from
// global memory (no LDS).  Kernel terms: C column-major M x N; A-side element
// (x, p) at A[x + p*lda] (MN-major) or A[x*lda + p] (K-major).
// MFMA 16x16x4 fragments: lane l (r = l%16, q = l/16) supplies row r of A and
// column r of B at one k of each 4-k step; which k a lane group q supplies is
// free as long as A and B agree.  Here, in k-block j (16 values) and step t,
// group q supplies k = 16j + 4q + t, so each lane reads its four k of a block
// as one vector and a block is four MFMA steps.  Every C entry accumulates in
// the same order in both tile classes.
template <int TM, bool AKC, bool BKC>
__device__ __forceinline__ void wave_tile(const float* __restrict__ A, int64_t lda,
                                          const float* __restrict__ B, int64_t ldb,
                                          float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                          int tm, int tn, float alpha, float beta)
{
    constexpr int FB = TM / 16;
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t x0a = (int64_t)tm * TM, x0b = (int64_t)tn * TM;
    const int nJ = (K + 15) / 16;

    f4 acc[FB][FB];
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    Frag<FB, AKC> fa;
    Frag<FB, BKC> fb;
    fa.init(A, lda, M, K, x0a, r, q);
    fb.init(B, ldb, N, K, x0b, r, q);
    // Three k-blocks of fragments in registers: the one being multiplied and
    // the next two in flight.  The loop is unrolled three times so that the
    // three register sets trade roles in the code: copying a register whose
    // load is still in flight would make the wave wait for it.
    f4 a0[FB], b0[FB], a1[FB], b1[FB], a2[FB], b2[FB];
    // loads of blocks past the last one fall outside the operand (k >= K) and
    // return zeros without touching memory: issued unconditionally, so no
    // branch sits between a load and its use
    auto load = [&](int j, f4 (&ta)[FB], f4 (&tb)[FB]) {
        fa.load(j, 16 * j + 4 * q, K, ta);
        fb.load(j, 16 * j + 4 * q, K, tb);
    };
    // k-block j on register set (ta, tb); in the last, partial k-block the
    // K-major fragments' elements past K are zeroed first (uniform branch)
    auto compute = [&](int j, f4 (&ta)[FB], f4 (&tb)[FB]) {
        if (16 * j + 16 > K) {
            const int k0 = 16 * j + 4 * q;
#pragma unroll
            for (int t = 1; t < 4; ++t) {
                const bool keep = k0 + t < K;
                if (AKC) {
#pragma unroll
                    for (int a = 0; a < FB; ++a) ta[a][t] = keep ? ta[a][t] : 0.f;
                }
                if (BKC) {
#pragma unroll
                    for (int b = 0; b < FB; ++b) tb[b][t] = keep ? tb[b][t] : 0.f;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < FB; ++a)
#pragma unroll
                for (int b = 0; b < FB; ++b) acc[a][b] = mfma16(ta[a][t], tb[b][t], acc[a][b]);
    };
    load(0, a0, b0);
    load(1, a1, b1);
    for (int j = 0; j < nJ; j += 3) {
        load(j + 2, a2, b2);
        compute(j, a0, b0);
        if (j + 1 >= nJ) break;
        load(j + 3, a0, b0);
        compute(j + 1, a1, b1);
        if (j + 2 >= nJ) break;
        load(j + 4, a1, b1);
        compute(j + 2, a2, b2);
    }

    // Epilogue: item e of lane l of block (a, b) is C[4*(l/16) + e][l%16].  C
    // is a buffer too: every C load is issued before any is used, and lanes
    // outside the M x N result load zeros and have their stores dropped by the
    // buffer unit, so no per-lane branch serialises the loads.
    const Mat mc = make_mat(C, ldc, M, N, false);
    uint32_t co[FB][FB][4];
    float cv[FB][FB][4];
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b) {
            const int64_t i0 = x0a + 16 * a + 4 * q, j = x0b + 16 * b + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = i0 + e;
                co[a][b][e] = (i < M && j < N) ? (uint32_t)((i + j * ldc) * (int64_t)sizeof(float))
                                               : kOob;
                cv[a][b][e] = beta != 0.f
                                  ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                                  mc.r, co[a][b][e], 0, 0))
                                  : 0.f;
            }
        }
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = beta != 0.f ? axpby(alpha, acc[a][b][e], beta, cv[a][b][e])
                                            : alpha * acc[a][b][e];
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), mc.r,
                                                      co[a][b][e], 0, 0);
            }
}

template <int TM>
__device__ __forceinline__ void vb_dispatch(int kmaj, const float* A, int64_t lda, const float* B,
                                            int64_t ldb, float* C, int64_t ldc, int M, int N,
                                            int K, int tm, int tn, float alpha, float beta)
{
    switch (kmaj) {
    case 0: wave_tile<TM, false, false>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta); break;
    case 1: wave_tile<TM, true, false>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta); break;
    case 2: wave_tile<TM, false, true>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta); break;
    default: wave_tile<TM, true, true>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn, alpha, beta); break;
    }
}

#ifndef FIP_VB_WAVES_PER_EU
#define FIP_VB_WAVES_PER_EU 3
#endif
__global__ void __launch_bounds__(VB_NTHR, FIP_VB_WAVES_PER_EU) vbatched_kernel(const VbParams P)
{
    // The planner gives each XCD a list of whole problems (balanced by cost)
    // and orders each list longest tile first.  Workgroup w runs on XCD w % 8
    // as that XCD's wave number w / 8 of W / 8 and takes the list's items
    // local, local + W/8, local + 2W/8, ...: no shared counter, every wave
    // knows its items from its index alone, and a problem's tiles share the
    // one XCD's L2.  W is a multiple of 8.
    const int64_t W8 = gridDim.x >> 3;
    const int x = blockIdx.x & 7;
    const int64_t end = P.xcd_off[x + 1];
    int64_t item = P.xcd_off[x] + (blockIdx.x >> 3);
    if (item >= end) return;
    VbItem it = P.items[item];
    VbProblem pr = P.probs[it.prob];
    VbItem it_n = it;
    if (item + W8 < end) it_n = P.items[item + W8];
    while (true) {
        // descriptors of this wave's next item (and the item after), fetched
        // while this one runs
        const int64_t next = item + W8;
        VbProblem pr_n = pr;
        if (next < end) pr_n = P.probs[it_n.prob];
        VbItem it_nn = it_n;
        if (next + W8 < end) it_nn = P.items[next + W8];
        const bool sw = pr.flags & kVbSwapped;
        // kernel A-side: the caller's A, or op(B)^T for a swapped (row-major) problem
        const float* A = sw ? P.B[it.prob] : P.A[it.prob];
        const float* B = sw ? P.A[it.prob] : P.B[it.prob];
        const int64_t lda = sw ? P.ldb[it.prob] : P.lda[it.prob];
        const int64_t ldb = sw ? P.lda[it.prob] : P.ldb[it.prob];
        const int kmaj = (pr.flags & kVbAKmajor ? 1 : 0) | (pr.flags & kVbBKmajor ? 2 : 0);
        const int K = P.no_ab ? 0 : pr.K;
        const int64_t ldc = P.ldc[it.prob];
        if (!vb_valid(lda, ldb, ldc, pr.M, pr.N, K, kmaj & 1, kmaj & 2)) {
            // leading dimensions come from device arrays the host never sees: a problem
            // that would read or write outside its matrices is skipped and reported
            if ((threadIdx.x & 63) == 0) atomicMax(P.status, (unsigned long long)it.prob + 1);
        } else if (pr.cls == 1)
            vb_dispatch<32>(kmaj, A, lda, B, ldb, P.C[it.prob], ldc, pr.M, pr.N, K, it.tm,
                            it.tn, P.alpha, P.beta);
        else
            vb_dispatch<16>(kmaj, A, lda, B, ldb, P.C[it.prob], ldc, pr.M, pr.N, K, it.tm,
                            it.tn, P.alpha, P.beta);
        if (next >= end) break;
        item = next;
        it = it_n;
        pr = pr_n;
        it_n = it_nn;
    }
}

VbParams make_vb_params(const VbLaunchDesc& d)
{
    VbParams P{};
    P.status = d.status;
    P.probs = d.probs; P.items = d.items; P.total = d.total;
    for (int i = 0; i <= kCopies; ++i) P.xcd_off[i] = d.xcd_off[i];
    P.A = d.A; P.lda = d.lda; P.B = d.B; P.ldb = d.ldb; P.C = d.C; P.ldc = d.ldc;
    P.alpha = d.alpha; P.beta = d.beta;
    P.no_ab = d.alpha == 0.f;
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
        grid = (cus * per_cu) & ~7;
        if (grid < 8) grid = 8;
    }
    return grid;
}

// Workgroups of a batch launch: the resident count, but no more than 8 times
// the longest per-XCD list (a multiple of 8, which the numbering needs).
int64_t vb_launch_grid(const VbLaunchDesc& d)
{
    int64_t longest = 1;
    for (int x = 0; x < kCopies; ++x)
        if (d.xcd_off[x + 1] - d.xcd_off[x] > longest) longest = d.xcd_off[x + 1] - d.xcd_off[x];
    const int64_t g = vbatched_grid();
    return g < 8 * longest ? g : 8 * longest;
}

hipError_t launch_vbatched(const VbLaunchDesc& d)
{
    clear_stale_error();
    if (d.total < 1) return hipSuccess;
    const VbParams P = make_vb_params(d);
    vbatched_kernel<<<dim3((unsigned)vb_launch_grid(d)), dim3(VB_NTHR), 0, d.stream>>>(P);
    return hipGetLastError();
}

// A graph of one kernel node running the batch.
hipError_t build_vbatched_graph(const VbLaunchDesc& d, hipGraphExec_t* exec)
{
    VbParams P = make_vb_params(d);
    const int64_t g = vb_launch_grid(d);
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
