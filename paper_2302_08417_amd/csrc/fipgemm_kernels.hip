// HIP kernels of the fused-pack GEMM for gfx950 (CDNA4).
//
// One tile kernel serves every problem size (paper Sec. 3: a single code path
// from which the unpacked "SUP" algorithm and conventional pack-then-compute
// fall out as special cases).  A workgroup computes one MT x NT tile of C,
// stepping through k in chunks of KT.  For each k-step it stages the A-side
// chunk (MT x KT) and B-side chunk (NT x KT) in LDS, double buffered, and runs
// 16x16x4 MFMAs on them (FP64 or FP32 accumulate).
//
// Fused packing (Sec. 3.2): the first workgroup (per XCD) that touches an
// operand panel claims it and becomes its producer: for every k-step it loads
// the unpacked chunk from HBM (coalesced along whichever stride is 1, masked
// with zero fill at the fringes, Sec. 2.2), and stores the same registers both
// to LDS for its own MFMAs and to the HBM pack buffer at the chunk's canonical
// position.  Once every pack store of the panel has completed, the producer
// publishes the panel's completion flag, stamped with the call's epoch.
// Every other workgroup on that XCD needing the panel checks the flag at its
// tile start and then every few k-steps: once set, it reads the packed,
// contiguous chunks (16-byte vector loads, no masks); until then it reads the
// unpacked operand itself.  Nobody ever waits, so the schedule cannot
// deadlock, and both sources hold identical bits, so the result does not
// depend on timing.
//
// Which panels are packed follows the paper's reuse table (Sec. 3.3), decided
// on the host.  The paper's shared-A, private-B multithreading scheme
// (Sec. 3.5) maps to per-XCD pack copies: each XCD has its own L2, so a copy
// written and read by one XCD needs no cross-L2 cache maintenance.
#include "fip_internal.h"
#include "fip_device.h"
#include "fip_tile.h"

namespace fip {
namespace {

template <typename T>
struct Params {
    const T* A; const T* B; T* C;
    int64_t a_smn, a_sk, b_smn, b_sk, ldc;
    int64_t M, N, K;
    T alpha, beta;
    T* apack; T* bpack;
    int64_t apack_copy, bpack_copy;
    uint64_t* aflag; uint64_t* bflag; uint64_t* aclaim; uint64_t* bclaim;
    unsigned long long* stats;
    uint64_t epoch;
    int tilesM, tilesN, nK, group_m;
    int mode, pack_a, pack_b, no_publish, do_stats;
    int a_pack_from, b_pack_from;  // first tile row / column whose panel is packed
    int shared_copy;  // 1: one pack copy for all XCDs (copy 0), else one per XCD
    int a_vec, b_vec, c_vec;
    int a_fast, b_fast;  // interior chunks may use the 32-bit-offset vector loader
    int order;       // tile order inside an XCD's run: 0 grouped, 1 column-distinct rounds
    int split, slice_ksteps;  // k split into `split` slices of slice_ksteps k-steps
    T* part;                  // split partials: [split][N][M] (kernel view, column-major)
    // Other level-3 operations on the same tile body (see LaunchDesc; the
    // operation itself is the kernel's KIND parameter)
    int tri_upper;            // SYRK: C's triangle is row <= column (else row >= column)
    int tri_side;             // TRMM: 1 = A side triangular, 2 = B side
    int tri_keep_ge;          // TRMM: element (x, p) kept when x >= p (else x <= p)
    int tri_unit;             // TRMM: the diagonal x == p reads as 1
    T alpha_im, beta_im;      // k1m: imaginary parts of alpha and beta
    int conj_a, conj_b;       // k1m: the side reads the conjugated operand
};

// TRMM: workgroup w -> tile, longest k-range first.  A tile's k-range is set
// by its row (triangular A side) or column (triangular B side) of tiles, and
// runs from 1 to all k-steps, so the tiles are issued in order of decreasing
// k-range, consecutive workgroups (which go to different XCDs) taking the
// tiles of one row (column): every XCD gets its share of the long tiles, and
// the short ones fill in at the end.
__device__ __forceinline__ void trmm_tile(int w, int tilesM, int tilesN, bool tri_a, bool keep_ge,
                                          int& tm, int& tn)
{
    if (tri_a) {
        const int r = w / tilesN;
        tn = w - r * tilesN;
        tm = keep_ge ? tilesM - 1 - r : r;
    } else {
        const int c = w / tilesM;
        tm = w - c * tilesM;
        tn = keep_ge ? tilesN - 1 - c : c;
    }
}

// SYRK: workgroup w -> tile (tm, tn) of the stored triangle.  XCD-contiguous
// runs of the triangle's tiles in row order (lower: tn <= tm), so consecutive
// tiles of an XCD share their A-side panel.
__device__ __forceinline__ void tri_tile(int w, int t, bool upper, int& tm, int& tn)
{
    const int T = t * (t + 1) / 2;
    const int xcd = w & 7, local = w >> 3;
    const int q = T >> 3, rr = T & 7;
    const int idx = xcd * q + (xcd < rr ? xcd : rr) + local;
    int r = (int)((__builtin_sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > idx) --r;
    while ((r + 1) * (r + 2) / 2 <= idx) ++r;
    const int c = idx - r * (r + 1) / 2;
    tm = upper ? c : r;
    tn = upper ? r : c;
}

// KIND (kGemm, kSyrk, kTrmm) is a compile-time parameter so that the GEMM
// instantiations carry none of the triangle logic (it costs registers).
template <typename T, int MT, int NT, int KT, int WM, int WN, bool AKC, bool BKC, int KIND>
__global__ void __launch_bounds__(WM * WN * 64, 2) gemm_kernel(const Params<T> P)
{
    constexpr int NTHR = WM * WN * 64;
    typedef Chunk<T, MT, KT, NTHR, AKC> ChA;
    typedef Chunk<T, NT, KT, NTHR, BKC> ChB;
    typedef typename Types<T>::acc Acc;
    constexpr int WTM = MT / WM, WTN = NT / WN;  // per-wave C sub-tile
    constexpr int FM = WTM / 16, FN = WTN / 16;  // MFMA blocks per wave
    static_assert(FM >= 1 && FN >= 1 && KT % 4 == 0, "tile shape");

    __shared__ __attribute__((aligned(16))) T sA[2][ChA::LDS_ELEMS];
    __shared__ __attribute__((aligned(16))) T sB[2][ChB::LDS_ELEMS];
    __shared__ int s_role;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    // Split k: workgroup w computes k-slice w / tiles of tile w % tiles
    // (chunks [slice * slice_ksteps, +slice_ksteps)); the slices of one tile
    // are `tiles` workgroups apart, so they fall on the same XCD whenever the
    // tile count is a multiple of 8.
    const int S = P.split;
    const int ntiles = P.tilesM * P.tilesN;
    const int slice = S > 1 ? (int)(blockIdx.x / (unsigned)ntiles) : 0;
    const int wt = (int)blockIdx.x - slice * ntiles;
    int tm, tn;
    if constexpr (KIND == kSyrk) tri_tile(wt, P.tilesM, P.tri_upper, tm, tn);
    else if constexpr (KIND == kTrmm) trmm_tile(wt, P.tilesM, P.tilesN, P.tri_side == 1, P.tri_keep_ge, tm, tn);
    else tile_coords(wt, P.tilesM, P.tilesN, P.group_m, P.order, tm, tn);
    const int64_t x0a = (int64_t)tm * MT, x0b = (int64_t)tn * NT;
    const int nK = P.nK;
    int q0 = slice * P.slice_ksteps;
    int q1 = q0 + P.slice_ksteps < nK ? q0 + P.slice_ksteps : nK;
    // TRMM: the k-steps whose chunk of the triangular operand is not all
    // structural zeros (rows x of the tile's panel keep p <= x, or p >= x)
    const bool tri_a = KIND == kTrmm && P.tri_side == 1;
    const bool tri_b = KIND == kTrmm && P.tri_side == 2;
    if (tri_a || tri_b) {
        const int64_t tx0 = tri_a ? x0a : x0b, tmn = tri_a ? MT : NT;
        if (P.tri_keep_ge) {
            const int64_t last = (tx0 + tmn + KT - 1) / KT;   // chunks holding p < tx0 + tmn
            if (last < q1) q1 = (int)last;
        } else {
            const int64_t first = tx0 / KT;
            if (first > q0) q0 = (int)first;
        }
    }
    const int nKfull = (int)(P.K / KT);  // chunks with all KT k-values present
    const uint64_t epoch = P.epoch;

    // Unpacked operands: leading dimension, chunk origin and per-lane byte
    // offsets of interior chunks (loop-invariant; the host guarantees they fit
    // in 32 bits).  A tile is interior along MN when it lies fully inside.
    const int64_t lda = AKC ? P.a_smn : P.a_sk, ldb = BKC ? P.b_smn : P.b_sk;
    const bool a_in = P.a_fast && x0a + MT <= P.M, b_in = P.b_fast && x0b + NT <= P.N;
    // chunk origin and bytes per chunk; k1m: in complex elements of 2 T (the
    // A side's real row x0a is complex row x0a/2, a chunk spans KT/2 complex k)
    constexpr bool CX = KIND == k1m;
    constexpr int64_t ES = CX ? 2 * (int64_t)sizeof(T) : (int64_t)sizeof(T);
    const int64_t ra0 = CX ? x0a / 2 : x0a, kstep = CX ? KT / 2 : KT;
    const char* a_org = reinterpret_cast<const char*>(P.A) + (AKC ? ra0 * lda : ra0) * ES;
    const char* b_org = reinterpret_cast<const char*>(P.B) + (BKC ? x0b * ldb : x0b) * ES;
    const int64_t a_step = (AKC ? kstep : kstep * lda) * ES;
    const int64_t b_step = (BKC ? kstep : kstep * ldb) * ES;
    uint32_t a_off[ChA::NV], b_off[ChB::NV];
    // A fringe tile (overhanging M or N) may read its full-k chunks the same
    // way when no vector straddles the edge: a vector outside the operand
    // reads the chunk origin instead (a valid element).  Rows of the A side
    // beyond M (columns of the B side beyond N) only ever reach C entries
    // outside the matrix, which the epilogue does not store, so their values
    // do not matter; only a packed copy must hold zeros there, so the
    // producer of a fringe panel keeps the zero-filling loads.
    constexpr int VEC = Types<T>::VEC;
    const bool a_ff = P.a_fast && !a_in && (AKC || P.M % VEC == 0);
    const bool b_ff = P.b_fast && !b_in && (BKC || P.N % VEC == 0);
    uint32_t apar = 0, bpar = 0;   // k1m: per-vector arrangement bits
#pragma unroll
    for (int i = 0; i < ChA::NV; ++i) {
        const uint32_t o = CX ? ChA::template cx_offset<0>(i, tid, lda) : ChA::fast_offset(i, tid, lda);
        a_off[i] = a_ff && !ChA::vec_inside(i, tid, x0a, P.M) ? 0u : o;
        if (CX && ChA::template cx_par<0>(i, tid)) apar |= 1u << i;
    }
#pragma unroll
    for (int i = 0; i < ChB::NV; ++i) {
        const uint32_t o = CX ? ChB::template cx_offset<1>(i, tid, ldb) : ChB::fast_offset(i, tid, ldb);
        b_off[i] = b_ff && !ChB::vec_inside(i, tid, x0b, P.N) ? 0u : o;
        if (CX && ChB::template cx_par<1>(i, tid)) bpar |= 1u << i;
    }

    const bool consume = P.mode == kModeConsumePacked;
    bool fused = P.mode == kModeFused;
    int copy = 0;
    if (fused) {
        const unsigned x = xcc_id();
        if (P.shared_copy) copy = 0;
        else if (x < (unsigned)kCopies) copy = (int)x;
        else fused = false;  // unknown XCD id: this workgroup stays unpacked
    }
    const bool useA = fused && P.pack_a && tm >= P.a_pack_from;
    const bool useB = fused && P.pack_b && tn >= P.b_pack_from;

    T* apanel = nullptr;
    T* bpanel = nullptr;
    // a copy holds the packed panels from a_pack_from / b_pack_from on
    if (useA || consume)
        apanel = P.apack + (int64_t)copy * P.apack_copy + (int64_t)(tm - P.a_pack_from) * nK * KT * MT;
    if (useB || consume)
        bpanel = P.bpack + (int64_t)copy * P.bpack_copy + (int64_t)(tn - P.b_pack_from) * nK * KT * NT;
    // (SYRK: the host points the B side's pack, flags and claims at the A
    // side's, so a panel is claimed, packed and read once for both roles; the
    // diagonal tile's B-side claim then finds its own A-side claim.)
    // One completion flag and one claim per (copy, panel, k-slice): a slice's
    // chunks of a panel are packed by the first workgroup of that slice.
    const int64_t aslot = ((int64_t)copy * P.tilesM + tm) * S + slice;
    const int64_t bslot = ((int64_t)copy * P.tilesN + tn) * S + slice;
    uint64_t* adone = useA ? P.aflag + aslot : nullptr;
    uint64_t* bdone = useB ? P.bflag + bslot : nullptr;

    // First touch claims a panel (Sec. 3.2: the first pass packs it).  The role
    // must be workgroup-uniform because every thread stores its share of each
    // packed chunk, so thread 0 claims and broadcasts.
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
    const bool wantA = useA && !prodA, wantB = useB && !prodB;  // would read a packed copy
    // unpacked full-k chunks through the offset loader (interior tiles, and
    // fringe tiles that do not produce a pack)
    const bool a_fastpath = a_in || (a_ff && !prodA), b_fastpath = b_in || (b_ff && !prodB);

    // Later passes (Sec. 3.1) read the packed copy once its producer has
    // published the whole panel.  Packed and unpacked sources stage the same
    // elements into the same LDS places (same thread-to-element mapping), so
    // each wave decides for itself from its own flag reads: at the tile start,
    // then again every REPOLL k-steps while still unpacked.  Nobody waits.
    constexpr int REPOLL = 16;
    bool apk = consume, bpk = consume;
    {
        const uint64_t fa = wantA ? peek_flag(adone) : 0, fb = wantB ? peek_flag(bdone) : 0;
        apk = apk || (wantA && __builtin_amdgcn_readfirstlane((int)(fa == epoch)) != 0);
        bpk = bpk || (wantB && __builtin_amdgcn_readfirstlane((int)(fb == epoch)) != 0);
        if ((wantA && apk) || (wantB && bpk)) acquire_packed();
    }

    unsigned long long n_prod = 0, n_pk = 0, n_unpk = 0, n_polls = 0;
    ChA ra;
    ChB rb;
    // Whether chunk c of a triangular operand's panel (rows [tx0, tx0 + tmn))
    // holds both kept and dropped entries, or diagonal ones: not entirely
    // strictly inside the kept triangle.
    auto tri_meets = [&](int64_t tx0, int64_t tmn, int c) -> bool {
        const int64_t p0 = (int64_t)c * KT;
        return P.tri_keep_ge ? p0 + KT - 1 >= tx0 : p0 <= tx0 + tmn - 1;
    };
    // k1m: whether the chunk in registers still awaits its 1m arrangement
    bool a_cxraw = false, b_cxraw = false;
    auto cx_settle = [&]() {
        if constexpr (CX) {
            if (a_cxraw) ra.template cx_fix<0>(apar, P.conj_a);
            if (b_cxraw) rb.template cx_fix<1>(bpar, P.conj_b);
        }
    };
    // Packed chunks and interior unpacked chunks are read by one and the same
    // vector-load sequence: only the base pointer and the per-lane offsets
    // differ (packed element o sits o*sizeof(T) bytes into its chunk).
    auto load_chunks = [&](int c) {
        const bool kin = c < nKfull;
        if constexpr (CX) {
            // complex operands: the packed copy holds the expanded real chunk;
            // interior chunks that arrange in place are loaded raw and
            // arranged by cx_settle once the step's MFMAs have been issued
            a_cxraw = b_cxraw = false;
            if (apk) {
                ra.load_packed(apanel + (int64_t)c * KT * MT, tid);
            } else if (a_fastpath && kin) {
                if constexpr (ChA::template cx_in_place<0>()) {
                    ra.load_at(a_org + (int64_t)c * a_step, a_off);
                    a_cxraw = true;
                } else {
                    ra.template load_cx_at<0>(a_org + (int64_t)c * a_step, a_off, apar, P.conj_a);
                }
            } else {
                ra.template load_cx_edge<0>(P.A, lda, P.M / 2, P.K / 2, x0a, (int64_t)c * KT, P.conj_a, tid);
            }
            if (bpk) {
                rb.load_packed(bpanel + (int64_t)c * KT * NT, tid);
            } else if (b_fastpath && kin) {
                if constexpr (ChB::template cx_in_place<1>()) {
                    rb.load_at(b_org + (int64_t)c * b_step, b_off);
                    b_cxraw = true;
                } else {
                    rb.template load_cx_at<1>(b_org + (int64_t)c * b_step, b_off, bpar, P.conj_b);
                }
            } else {
                rb.template load_cx_edge<1>(P.B, ldb, P.N, P.K / 2, x0b, (int64_t)c * KT, P.conj_b, tid);
            }
        } else {
        if (apk || (a_fastpath && kin)) {
            const char* base = apk ? reinterpret_cast<const char*>(apanel + (int64_t)c * KT * MT)
                                   : a_org + (int64_t)c * a_step;
            uint32_t off[ChA::NV];
#pragma unroll
            for (int i = 0; i < ChA::NV; ++i)
                off[i] = apk ? (uint32_t)(ChA::elem_o(i, tid) * sizeof(T)) : a_off[i];
            ra.load_at(base, off);
        } else {
            ra.load_edge(P.A, lda, P.M, P.K, x0a, (int64_t)c * KT, P.a_vec, tid);
        }
        if (bpk || (b_fastpath && kin)) {
            const char* base = bpk ? reinterpret_cast<const char*>(bpanel + (int64_t)c * KT * NT)
                                   : b_org + (int64_t)c * b_step;
            uint32_t off[ChB::NV];
#pragma unroll
            for (int i = 0; i < ChB::NV; ++i)
                off[i] = bpk ? (uint32_t)(ChB::elem_o(i, tid) * sizeof(T)) : b_off[i];
            rb.load_at(base, off);
        } else {
            rb.load_edge(P.B, ldb, P.N, P.K, x0b, (int64_t)c * KT, P.b_vec, tid);
        }
        }
        // TRMM: an unpacked chunk that meets the diagonal gets the triangle
        // applied in registers (zeros outside it, ones on a unit diagonal)
        // before it reaches LDS or the pack; a packed chunk already holds it.
        if (tri_a && !apk && tri_meets(x0a, MT, c))
            ra.mask_tri(x0a, (int64_t)c * KT, P.tri_keep_ge, P.tri_unit, P.M, P.K, tid);
        if (tri_b && !bpk && tri_meets(x0b, NT, c))
            rb.mask_tri(x0b, (int64_t)c * KT, P.tri_keep_ge, P.tri_unit, P.N, P.K, tid);
        if (P.do_stats && tid == 0) {
            n_prod += (int)prodA + (int)prodB;
            n_pk += (int)(wantA && apk) + (int)(wantB && bpk) + (consume ? 2 : 0);
            n_unpk += (int)(wantA && !apk) + (int)(wantB && !bpk);
        }
    };

    Acc acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = Acc{};

    // MFMAs on the chunk in LDS buffer cur.  Fragment element (row x, k-row
    // kr) of either orientation: lane l supplies x = base + l%16, kr = 4s + l/16.
    auto mfma_step = [&](int cur) {
        const T* la = sA[cur] + ChA::lds_at(wm * WTM + (lane & 15), lane >> 4);
        const T* lb = sB[cur] + ChB::lds_at(wn * WTN + (lane & 15), lane >> 4);
#pragma unroll
        for (int s = 0; s < KT / 4; ++s) {
            T af[FM], bf[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) af[a] = la[ChA::lds_at(a * 16, 4 * s)];
#pragma unroll
            for (int b = 0; b < FN; ++b) bf[b] = lb[ChB::lds_at(b * 16, 4 * s)];
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) acc[a][b] = mfma16(af[a], bf[b], acc[a][b]);
        }
    };
    if constexpr (KIND == kGemmDma) {
        // Direct global -> LDS loads (the paper's footnote to Sec. 5: on a GPU
        // whose L1-level store is a DMA-fed scratchpad, packing through DMA is
        // expected to pay).  The host launches this variant only when no tile
        // produces a pack and every chunk can be fetched whole: all chunks
        // packed (pack-then-compute), or unpacked with k a multiple of KT and
        // the operands readable through the offset loaders.  Each wave fetches
        // its share of a chunk straight into the LDS buffer: no staging
        // registers, no LDS stores; every element lands where the register
        // path stores it, so C is the same bit for bit.
        auto stage = [&](int c, int buf) {
            if (apk) ChA::dma_issue(sA[buf], reinterpret_cast<const char*>(apanel + (int64_t)c * KT * MT), -1, 0, 0, wave, lane);
            else ChA::dma_issue(sA[buf], a_org + (int64_t)c * a_step, lda, x0a, P.M, wave, lane);
            if (bpk) ChB::dma_issue(sB[buf], reinterpret_cast<const char*>(bpanel + (int64_t)c * KT * NT), -1, 0, 0, wave, lane);
            else ChB::dma_issue(sB[buf], b_org + (int64_t)c * b_step, ldb, x0b, P.N, wave, lane);
            if (P.do_stats && tid == 0) n_pk += consume ? 2 : 0;
        };
        stage(q0, 0);
        wait_all_memory();
        __syncthreads();
        for (int q = q0; q < q1; ++q) {
            const int cur = (q - q0) & 1;
            // the other buffer was last read before the previous barrier
            if (q + 1 < q1) stage(q + 1, cur ^ 1);
            mfma_step(cur);
            wait_all_memory();   // this wave's loads into LDS have landed
            __syncthreads();
        }
    } else {
    // Prologue: stage the slice's first chunk.
    load_chunks(q0);
    cx_settle();
    ra.store_lds(sA[0], tid);
    rb.store_lds(sB[0], tid);
    if (prodA) ra.store_pack(apanel + (int64_t)q0 * KT * MT, tid);
    if (prodB) rb.store_pack(bpanel + (int64_t)q0 * KT * NT, tid);
    __syncthreads();

    for (int q = q0; q < q1; ++q) {
        const int cur = (q - q0) & 1;
        const bool more = q + 1 < q1;
        // Re-poll while an operand is still read unpacked.  The flag load is
        // issued before this step's chunk loads and read after them, when the
        // loads have been waited for anyway.
        const bool poll = ((wantA && !apk) || (wantB && !bpk)) && q % REPOLL == REPOLL - 1;
        uint64_t fa = 0, fb = 0;
        if (poll) {
            if (wantA && !apk) fa = peek_flag(adone);
            if (wantB && !bpk) fb = peek_flag(bdone);
        }
        if (more) load_chunks(q + 1);
        mfma_step(cur);
        if (more) {
            cx_settle();
            ra.store_lds(sA[cur ^ 1], tid);
            rb.store_lds(sB[cur ^ 1], tid);
            if (prodA) ra.store_pack(apanel + (int64_t)(q + 1) * KT * MT, tid);
            if (prodB) rb.store_pack(bpanel + (int64_t)(q + 1) * KT * NT, tid);
        }
        if (poll) {  // takes effect from chunk q+2 on
            const bool na = !apk && wantA && __builtin_amdgcn_readfirstlane((int)(fa == epoch)) != 0;
            const bool nb = !bpk && wantB && __builtin_amdgcn_readfirstlane((int)(fb == epoch)) != 0;
            if (na || nb) acquire_packed();
            apk = apk || na;
            bpk = bpk || nb;
            if (P.do_stats && tid == 0) ++n_polls;
        }
        __syncthreads();
    }
    }

    // The producer publishes its panel once every pack store of it has
    // completed (see publish_flag).
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

    // Split k: each slice stores its raw partial product (no alpha, beta or
    // C) into its own column-major M x N plane of the workspace; a second
    // kernel sums the planes in slice order and applies the epilogue.
    if (S > 1) {
        T* pp = P.part + (int64_t)slice * P.M * P.N;
        auto di_ = [&](int r) -> int { return sizeof(T) == 8 ? (lane & 15) : 4 * (lane >> 4) + r; };
        auto dj_ = [&](int r) -> int { return sizeof(T) == 8 ? 4 * r + (lane >> 4) : (lane & 15); };
        const int64_t r0 = x0a + wm * WTM, c0 = x0b + wn * WTN;
        const bool vec = sizeof(T) == 4 && x0a + MT <= P.M && x0b + NT <= P.N && P.M % 4 == 0;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                if (vec) {
                    // four consecutive rows of one column: one 16-byte store
                    typedef typename Types<T>::uvec U;
                    U u;
#pragma unroll
                    for (int r = 0; r < 4; ++r) u[r] = acc[a][b][r];
                    *reinterpret_cast<U*>(pp + (r0 + a * 16 + di_(0)) + (c0 + b * 16 + dj_(0)) * P.M) = u;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t i = r0 + a * 16 + di_(r), j = c0 + b * 16 + dj_(r);
                        if (i < P.M && j < P.N) pp[i + j * P.M] = acc[a][b][r];
                    }
                }
            }
        return;
    }

    if constexpr (CX) {
        // Complex epilogue on the real view of C (a pair array with real
        // leading dimension 2 ldc): kernel rows 2i and 2i + 1 hold re and im of
        // complex row i.  C = alpha * acc + beta * C in complex arithmetic; C
        // is not read when beta == 0.  A lane needs the other component of each
        // of its entries: FP64 keeps one row per lane, so it comes from the
        // neighbouring lane (the other parity); FP32 keeps row pairs (items
        // r, r ^ 1) in the lane.  Each lane reads both components of C before
        // any store of the pair.
        const T ar = P.alpha, ai = P.alpha_im, br = P.beta, bi = P.beta_im;
        const bool has_beta = br != T(0) || bi != T(0);
        const int64_t ldr = 2 * P.ldc;
        const int64_t r0c = x0a + wm * WTM, c0c = x0b + wn * WTN;
        auto dic = [&](int r) -> int { return sizeof(T) == 8 ? (lane & 15) : 4 * (lane >> 4) + r; };
        auto djc = [&](int r) -> int { return sizeof(T) == 8 ? 4 * r + (lane >> 4) : (lane & 15); };
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                T v[4], w[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = acc[a][b][r];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if constexpr (sizeof(T) == 8) w[r] = __shfl_xor(v[r], 1);
                    else w[r] = v[r ^ 1];
                }
                // both components of every entry are read before any store
                // (with FP32 one lane stores both of them)
                T o[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = r0c + a * 16 + dic(r), j = c0c + b * 16 + djc(r);
                    const bool imr = i & 1;
                    const T sre = imr ? w[r] : v[r], sim = imr ? v[r] : w[r];
                    o[r] = imr ? ar * sim + ai * sre : ar * sre - ai * sim;
                    if (has_beta && i < P.M && j < P.N) {
                        const T cre = P.C[(i & ~(int64_t)1) + j * ldr];
                        const T cim = P.C[(i | 1) + j * ldr];
                        o[r] = o[r] + (imr ? br * cim + bi * cre : br * cre - bi * cim);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = r0c + a * 16 + dic(r), j = c0c + b * 16 + djc(r);
                    if (i < P.M && j < P.N) P.C[i + j * ldr] = o[r];
                }
            }
        return;
    }

    // Epilogue: C = alpha*acc + beta*C (C not read when beta == 0).  Lane l of
    // block (a, b) holds C elements (row r0 + di(l, r), column c0 + dj(l, r)),
    // r = 0..3 (see mfma16).  Interior tiles read all of their C first, then
    // write it back, with no masks.
    const T alpha = P.alpha, beta = P.beta;
    const bool diag_tile = KIND == kSyrk && tm == tn;
    const bool c_in = x0a + MT <= P.M && x0b + NT <= P.N && !diag_tile;
    auto di = [&](int r) -> int { return sizeof(T) == 8 ? (lane & 15) : 4 * (lane >> 4) + r; };
    auto dj = [&](int r) -> int { return sizeof(T) == 8 ? 4 * r + (lane >> 4) : (lane & 15); };
    const int64_t r0w = x0a + wm * WTM, c0w = x0b + wn * WTN;
    if (c_in) {
        // one block row at a time: all of its C loads are issued before any
        // use, without holding a second full accumulator's worth of registers
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            T cv[FN][4];
            if (beta != T(0)) {
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    const T* cb = P.C + (r0w + a * 16) + (c0w + b * 16) * P.ldc;
                    if constexpr (sizeof(T) == 8) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) cv[b][r] = cb[di(r) + (int64_t)dj(r) * P.ldc];
                    } else {
                        typedef typename Types<T>::uvec U;
                        const U u = *reinterpret_cast<const U*>(cb + di(0) + (int64_t)dj(0) * P.ldc);
#pragma unroll
                        for (int r = 0; r < 4; ++r) cv[b][r] = u[r];
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                T* cb = P.C + (r0w + a * 16) + (c0w + b * 16) * P.ldc;
                T out[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    out[r] = beta != T(0) ? axpby(alpha, acc[a][b][r], beta, cv[b][r])
                                          : alpha * acc[a][b][r];
                }
                if constexpr (sizeof(T) == 8) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) cb[di(r) + (int64_t)dj(r) * P.ldc] = out[r];
                } else {
                    typedef typename Types<T>::uvec U;
                    U u;
#pragma unroll
                    for (int r = 0; r < 4; ++r) u[r] = out[r];
                    *reinterpret_cast<U*>(cb + di(0) + (int64_t)dj(0) * P.ldc) = u;
                }
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = r0w + a * 16 + di(r), j = c0w + b * 16 + dj(r);
                    const bool in_tri = !diag_tile || (P.tri_upper ? i <= j : i >= j);
                    if (i < P.M && j < P.N && in_tri) {
                        T* cp = P.C + i + j * P.ldc;
                        *cp = beta != T(0) ? axpby(alpha, acc[a][b][r], beta, *cp)
                                           : alpha * acc[a][b][r];
                    }
                }
    }
}

// Second half of a split-k call: C = alpha * (sum of the slice planes, in
// slice order 0, 1, ...) + beta * C, with the tile kernel's epilogue rounding
// (C not read when beta == 0).  One thread per C element, column by column.
template <typename T>
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const T* __restrict__ part, int S,
                                                            int64_t M, int64_t N, T* C,
                                                            int64_t ldc, T alpha, T beta)
{
    const int64_t MN = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < MN;
         idx += (int64_t)gridDim.x * 256) {
        T v = part[idx];
        for (int sl = 1; sl < S; ++sl) v = v + part[(int64_t)sl * MN + idx];
        const int64_t i = idx % M, j = idx / M;
        T* cp = C + i + j * ldc;
        *cp = beta != T(0) ? axpby(alpha, v, beta, *cp) : alpha * v;
    }
}

// Standalone pack of both operands into copy 0 (the first half of the
// conventional pack-then-compute baseline).  Same register mapping and
// stores as a producer of the tile kernel, one chunk per workgroup.
// CX: complex operands, packed as their 1m expansions (real chunks).
template <typename T, int MT, int NT, int KT, int NTHR, bool AKC, bool BKC, bool CX>
__global__ void __launch_bounds__(NTHR) pack_kernel(const Params<T> P)
{
    const int tid = threadIdx.x;
    const int nK = P.nK;
    const int64_t nA = (int64_t)P.tilesM * nK;
    const int64_t b = blockIdx.x;
    if (b < nA) {
        const int64_t t = b / nK, q = b % nK;
        Chunk<T, MT, KT, NTHR, AKC> r;
        const int64_t ld = AKC ? P.a_smn : P.a_sk;
        if constexpr (CX) r.template load_cx_edge<0>(P.A, ld, P.M / 2, P.K / 2, t * MT, q * KT, P.conj_a, tid);
        else r.load_edge(P.A, ld, P.M, P.K, t * MT, q * KT, P.a_vec, tid);
        r.store_pack(P.apack + (t * nK + q) * KT * MT, tid);
    } else {
        const int64_t bb = b - nA;
        const int64_t t = bb / nK, q = bb % nK;
        Chunk<T, NT, KT, NTHR, BKC> r;
        const int64_t ld = BKC ? P.b_smn : P.b_sk;
        if constexpr (CX) r.template load_cx_edge<1>(P.B, ld, P.N, P.K / 2, t * NT, q * KT, P.conj_b, tid);
        else r.load_edge(P.B, ld, P.N, P.K, t * NT, q * KT, P.b_vec, tid);
        r.store_pack(P.bpack + (t * nK + q) * KT * NT, tid);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) scale_kernel(T* C, int64_t M, int64_t N, int64_t ldc, T beta)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx % M, j = idx / M;
        T* p = C + i + j * ldc;
        *p = beta == T(0) ? T(0) : beta * *p;
    }
}

__global__ void __launch_bounds__(64) xcc_map_kernel(uint32_t* out)
{
    if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <typename T>
Params<T> make_params(const LaunchDesc& d, int MT, int NT, int KT)
{
    constexpr int VEC = Types<T>::VEC;
    Params<T> P{};
    P.A = static_cast<const T*>(d.A);
    P.B = static_cast<const T*>(d.B);
    P.C = static_cast<T*>(d.C);
    P.a_smn = d.a_smn; P.a_sk = d.a_sk; P.b_smn = d.b_smn; P.b_sk = d.b_sk; P.ldc = d.ldc;
    P.M = d.M; P.N = d.N; P.K = d.K;
    P.alpha = (T)d.alpha; P.beta = (T)d.beta;
    P.apack = static_cast<T*>(d.apack); P.bpack = static_cast<T*>(d.bpack);
    P.apack_copy = d.apack_copy_elems; P.bpack_copy = d.bpack_copy_elems;
    P.aflag = d.aflag; P.bflag = d.bflag; P.aclaim = d.aclaim; P.bclaim = d.bclaim;
    P.stats = d.stats_ptr;
    P.epoch = d.epoch;
    P.tilesM = (int)((d.M + MT - 1) / MT);
    P.tilesN = (int)((d.N + NT - 1) / NT);
    P.nK = (int)((d.K + KT - 1) / KT);
    P.group_m = kGroupM;
    P.mode = d.mode; P.pack_a = d.pack_a; P.pack_b = d.pack_b;
    P.a_pack_from = d.a_pack_from; P.b_pack_from = d.b_pack_from;
    P.shared_copy = d.shared_copy;
    P.no_publish = d.no_publish; P.do_stats = d.stats && d.stats_ptr != nullptr;
    const int64_t a_far = d.a_kmajor ? d.a_smn : d.a_sk;  // the leading dimension
    const int64_t b_far = d.b_kmajor ? d.b_smn : d.b_sk;
    // unpacked vector loads need only element alignment (see Types::uvec)
    P.a_vec = ((uintptr_t)d.A % sizeof(T)) == 0;
    P.b_vec = ((uintptr_t)d.B % sizeof(T)) == 0;
    (void)a_far; (void)b_far;
    P.c_vec = aligned16(d.C) && d.ldc % VEC == 0;
    // byte offsets inside one chunk must fit in 32 bits: (MT + KT*ld) elements
    // for an MN-contiguous operand, (MT*ld + KT) for a k-contiguous one
    const int64_t a_span = (d.a_kmajor ? MT * a_far + KT : MT + KT * a_far) * (int64_t)sizeof(T);
    const int64_t b_span = (d.b_kmajor ? NT * b_far + KT : NT + KT * b_far) * (int64_t)sizeof(T);
    P.a_fast = P.a_vec && a_span < ((int64_t)1 << 31);
    P.b_fast = P.b_vec && b_span < ((int64_t)1 << 31);
    P.order = d.order;
    // split k (the host sizes slice_ksteps so that no slice is empty)
    P.split = d.split > 1 ? d.split : 1;
    P.slice_ksteps = d.split > 1 ? d.slice_ksteps : P.nK;
    P.part = static_cast<T*>(d.part);
    P.tri_upper = d.tri_upper;
    P.tri_side = d.tri_side;
    P.tri_keep_ge = d.tri_keep_ge;
    P.tri_unit = d.tri_unit;
    P.alpha_im = (T)d.alpha_im;
    P.beta_im = (T)d.beta_im;
    P.conj_a = d.conj_a;
    P.conj_b = d.conj_b;
    if (d.kind == k1m) {
        // complex operands: a chunk spans MT/2 (A side) or NT complex elements
        // along MN and KT/2 along k, each of 2 T; the spans above counted real
        // elements of the expanded extents, so twice them bounds the bytes
        P.a_fast = P.a_vec && 2 * a_span < ((int64_t)1 << 31);
        P.b_fast = P.b_vec && 2 * b_span < ((int64_t)1 << 31);
    }
    return P;
}

template <typename T, int MT, int NT, int KT, int WM, int WN, int KIND>
void launch_oriented(bool akc, bool bkc, dim3 grid, dim3 block, hipStream_t st, const Params<T>& P)
{
    if (!akc && !bkc) gemm_kernel<T, MT, NT, KT, WM, WN, false, false, KIND><<<grid, block, 0, st>>>(P);
    else if (!akc && bkc) gemm_kernel<T, MT, NT, KT, WM, WN, false, true, KIND><<<grid, block, 0, st>>>(P);
    else if (akc && !bkc) gemm_kernel<T, MT, NT, KT, WM, WN, true, false, KIND><<<grid, block, 0, st>>>(P);
    else gemm_kernel<T, MT, NT, KT, WM, WN, true, true, KIND><<<grid, block, 0, st>>>(P);
}

template <typename T, int MT, int NT, int WM, int WN>
hipError_t launch_tile(const LaunchDesc& d)
{
    constexpr int KT = sizeof(T) == 8 ? 16 : 32;
    const Params<T> P = make_params<T>(d, MT, NT, KT);
    const bool akc = d.a_kmajor, bkc = d.b_kmajor;
    const int64_t tiles = d.kind == kSyrk ? (int64_t)P.tilesM * (P.tilesM + 1) / 2
                                          : (int64_t)P.tilesM * P.tilesN;
    const dim3 grid((unsigned)(tiles * P.split)), block(WM * WN * 64);
    // GEMM through direct global -> LDS loads: only when no tile produces a
    // pack and every chunk can be fetched whole (see kGemmDma in the kernel)
    constexpr int VEC = Types<T>::VEC;
    const bool no_producer = d.mode == kModeConsumePacked || d.mode == kModeUnpacked ||
                             (d.mode == kModeFused && !d.pack_a && !d.pack_b);
    const bool whole = d.mode == kModeConsumePacked ||
                       (d.K % KT == 0 && P.a_fast && P.b_fast && (akc || d.M % VEC == 0) &&
                        (bkc || d.N % VEC == 0));
    // FIP_ATTR_DMA: 1 always, 0 never, -1 (default) where it measured faster:
    // binary64 launches that read their operands unpacked (binary32 ran 3-5 %
    // slower through it, binary64 pack-then-compute up to 2.6 % slower)
    const bool want = d.dma == 1 || (d.dma == -1 && sizeof(T) == 8 && d.mode != kModeConsumePacked);
    const bool dma = d.kind == kGemm && want && no_producer && whole;
    if (d.used_dma) *d.used_dma = dma;
    if (dma)
        launch_oriented<T, MT, NT, KT, WM, WN, kGemmDma>(akc, bkc, grid, block, d.stream, P);
    else if (d.kind == k1m) launch_oriented<T, MT, NT, KT, WM, WN, k1m>(akc, bkc, grid, block, d.stream, P);
    else if (d.kind == kSyrk) launch_oriented<T, MT, NT, KT, WM, WN, kSyrk>(akc, bkc, grid, block, d.stream, P);
    else if (d.kind == kTrmm) launch_oriented<T, MT, NT, KT, WM, WN, kTrmm>(akc, bkc, grid, block, d.stream, P);
    else launch_oriented<T, MT, NT, KT, WM, WN, kGemm>(akc, bkc, grid, block, d.stream, P);
    if (P.split > 1) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        int64_t blocks = (d.M * d.N + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        splitk_reduce_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, d.stream>>>(
            P.part, P.split, d.M, d.N, P.C, d.ldc, P.alpha, P.beta);
    }
    return hipGetLastError();
}

template <typename T, int MT, int NT, int WM, int WN>
hipError_t launch_pack_t(const LaunchDesc& d)
{
    constexpr int KT = sizeof(T) == 8 ? 16 : 32;
    constexpr int NTHR = WM * WN * 64;
    const Params<T> P = make_params<T>(d, MT, NT, KT);
    const bool akc = d.a_kmajor, bkc = d.b_kmajor;
    const int64_t blocks = ((int64_t)P.tilesM + P.tilesN) * P.nK;
    const dim3 grid((unsigned)blocks), block(NTHR);
    if (d.kind == k1m) {
        if (!akc && !bkc) pack_kernel<T, MT, NT, KT, NTHR, false, false, true><<<grid, block, 0, d.stream>>>(P);
        else if (!akc && bkc) pack_kernel<T, MT, NT, KT, NTHR, false, true, true><<<grid, block, 0, d.stream>>>(P);
        else if (akc && !bkc) pack_kernel<T, MT, NT, KT, NTHR, true, false, true><<<grid, block, 0, d.stream>>>(P);
        else pack_kernel<T, MT, NT, KT, NTHR, true, true, true><<<grid, block, 0, d.stream>>>(P);
    } else {
        if (!akc && !bkc) pack_kernel<T, MT, NT, KT, NTHR, false, false, false><<<grid, block, 0, d.stream>>>(P);
        else if (!akc && bkc) pack_kernel<T, MT, NT, KT, NTHR, false, true, false><<<grid, block, 0, d.stream>>>(P);
        else if (akc && !bkc) pack_kernel<T, MT, NT, KT, NTHR, true, false, false><<<grid, block, 0, d.stream>>>(P);
        else pack_kernel<T, MT, NT, KT, NTHR, true, true, false><<<grid, block, 0, d.stream>>>(P);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_gemm(const LaunchDesc& d)
{
    switch (d.tile_class) {
    case 0: return launch_tile<T, 128, 128, 2, 2>(d);
    case 1: return launch_tile<T, 64, 64, 2, 2>(d);
    case 2: return launch_tile<T, 32, 32, 2, 2>(d);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t dispatch_pack(const LaunchDesc& d)
{
    switch (d.tile_class) {
    case 0: return launch_pack_t<T, 128, 128, 2, 2>(d);
    case 1: return launch_pack_t<T, 64, 64, 2, 2>(d);
    case 2: return launch_pack_t<T, 32, 32, 2, 2>(d);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_gemm(const LaunchDesc& d)
{
    clear_stale_error();
    return d.elem == 8 ? dispatch_gemm<double>(d) : dispatch_gemm<float>(d);
}

hipError_t launch_pack(const LaunchDesc& d)
{
    clear_stale_error();
    return d.elem == 8 ? dispatch_pack<double>(d) : dispatch_pack<float>(d);
}

hipError_t launch_xcc_map(uint32_t* out, int64_t nblocks, hipStream_t stream)
{
    clear_stale_error();
    xcc_map_kernel<<<dim3((unsigned)nblocks), dim3(64), 0, stream>>>(out);
    return hipGetLastError();
}

hipError_t launch_scale(int elem, int64_t M, int64_t N, void* C, int64_t ldc, double beta,
                        hipStream_t stream)
{
    clear_stale_error();
    const int64_t total = M * N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    if (elem == 8)
        scale_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(
            static_cast<double*>(C), M, N, ldc, beta);
    else
        scale_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(
            static_cast<float*>(C), M, N, ldc, (float)beta);
    return hipGetLastError();
}

}  // namespace fip
