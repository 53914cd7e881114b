// C-ABI host layer: argument validation (before any HIP call), the planner
// (operand normalisation, tile class, the paper's pack-option table, workspace
// layout) and kernel launches.  See include/fipgemm.h for the contract.
#include "fipgemm.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <map>
#include <stdio.h>
#include <new>
#include <random>
#include <string.h>
#include <unordered_map>
#include <vector>

#include "fip_internal.h"
#include "fip_device.h"

namespace {

constexpr uint32_t kMagic = 0xF1F6E77u;
constexpr int64_t kMinSliceKsteps = 16;  // split k: at least this many k-steps per slice
constexpr int kMaxSplit = 32;            // split k: at most this many slices
// split k, mixed forms: at least this many k per slice (bfloat16 / E4M3, whose first
// pass only copies, and the bfloat16 split forms of binary32)
constexpr int64_t kMinSliceKCopy = 1024, kMinSliceKSplit = 256;
// AUTO packs nothing when a panel has fewer k-steps than this: a k-loop that
// short is over before a later pass could read the pack, and its reads are
// all first touches (each chunk is read once per tile either way).
constexpr int64_t kMinPackKsteps = 4;
// FIP_ATTR_DMA's default: the launch decides (see the attribute)
constexpr int kDefaultDma = -1;

// Epoch stamps of fused calls.  Claims and publish flags in a workspace are
// compared for equality with the current call's stamp, so a stamp must never
// repeat for the same memory: not across calls, handles, workspaces that
// reuse freed memory, nor lines a cache still holds from earlier calls.  A
// process-wide 64-bit counter started at a random point gives that without
// ever clearing the workspace.
uint64_t next_epoch()
{
    static std::atomic<uint64_t> counter([] {
        std::random_device rd;
        uint64_t r = ((uint64_t)rd() << 32) ^ (uint64_t)rd() ^
                     (uint64_t)std::chrono::high_resolution_clock::now().time_since_epoch().count();
        return (r & 0x0000FFFFFFFFFFFFull) | 0x0001000000000000ull;  // nonzero, far from ~0
    }());
    return counter.fetch_add(1, std::memory_order_relaxed);
}

}  // namespace

// Batched calls: the plan uploaded to the workspace, the tile-size threshold
// the autotuner chose per batch signature, and the graph of the last
// repeated call.
struct VbState {
    uint64_t sig = 0;
    int split = -1;
    void* ws = nullptr;
    int64_t total = 0;
    int64_t xcd_off[fip::kCopies + 1] = {};
    int64_t off_probs = 0, off_items = 0;
    std::vector<fip::VbProblem> probs;
    std::vector<fip::VbItem> items;
    std::unordered_map<uint64_t, int> tuned;
    hipGraphExec_t exec = nullptr;
    uint64_t gkey[12] = {};
    ~VbState()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// Tile class and k split that fip_gemm_tune measured fastest for a call
// shape (dtype, layout, m, n, k, transA, transB).
typedef std::array<int64_t, 7> GemmKey;
struct GemmChoice {
    int tile;    // tile class 0, 1, 2
    int split;   // FIP_ATTR_SPLIT_K semantics: -1 planner's, 1 none, >= 2 slices
};

struct fip_handle_s {
    uint32_t magic;
    hipStream_t stream;
    int policy;
    int tile_override;
    int no_publish;
    int stats;
    int order;
    void* ws;
    size_t ws_bytes;
    uint64_t epoch;   // stamp of the most recent fused call
    fip_plan_t last;
    int has_last;
    int vb_split;     // FIP_ATTR_VB_SPLIT (-1: tuned or default)
    int mx_tile;      // FIP_ATTR_MX_TILE (-1: planner's choice, 128, 256)
    int split_k;      // FIP_ATTR_SPLIT_K (-1: planner's choice, 1: off, 2..64: forced)
    int copies;       // FIP_ATTR_COPIES (-1: planner's choice, 1 or 8)
    int dma;          // FIP_ATTR_DMA (-1, 0 or 1)
    int last_dma;     // FIP_ATTR_LAST_DMA
    int last_hip_error;  // FIP_ATTR_LAST_HIP_ERROR
    VbState* vb;
    std::map<GemmKey, GemmChoice>* tuned;   // fip_gemm_tune results (null: none)
};

namespace {

bool valid_handle(fip_handle_t h) { return h != nullptr && h->magic == kMagic; }
bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}
// A failed launch: keep the HIP status for FIP_ATTR_LAST_HIP_ERROR.
int launch_failed(fip_handle_t h, hipError_t e)
{
    h->last_hip_error = (int)e;
    return FIP_ERR_LAUNCH;
}
bool valid_trans(char t)
{
    return t == 'N' || t == 'n' || t == 'T' || t == 't' || t == 'C' || t == 'c';
}
bool is_trans(char t) { return t != 'N' && t != 'n'; }
int64_t max1(int64_t v) { return v > 1 ? v : 1; }
int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Kernel view of one call: C is always column-major; for row-major storage
// the kernel computes C^T = op(B)^T op(A)^T, i.e. the operands swap sides.
struct KernelShape {
    int64_t M, N;     // kernel C rows / columns
    bool swapped;     // kernel A-side is the caller's op(B)
};

KernelShape kernel_shape(int layout, int64_t m, int64_t n)
{
    if (layout == FIP_ROW_MAJOR) return {n, m, true};
    return {m, n, false};
}

// Workgroups of one tile class that fit on the device at once (256 CUs times
// the per-CU residency the kernels' LDS and register use allow: about 2, 4 and
// 6 for the 128, 64 and 32 tiles).
int64_t resident_tiles(int cls)
{
    return 256 * (cls == 0 ? 2 : cls == 1 ? 4 : 6);
}

// Tile class: the largest C tile that still gives the 256 CUs about one tile
// each.  The class only changes blocking parameters, never the algorithm.
int choose_tile_class(int64_t M, int64_t N)
{
    const int64_t t128 = cdiv(M, 128) * cdiv(N, 128);
    if (t128 >= 256) return 0;
    const int64_t t64 = cdiv(M, 64) * cdiv(N, 64);
    if (t64 >= 128) return 1;
    return 2;
}

// Which panels does a later round read again?  Replays the launch order:
// workgroup w runs on XCD w % 8 and computes tile tile_coords(w); an XCD runs
// about per_xcd workgroups at a time, in dispatch order, so its local index
// divided by per_xcd is the round.  A panel (tile row of A, tile column of B)
// that an XCD touches in two different rounds is re-read by a pass that
// starts after an earlier pass over it could have finished: the reuse the
// paper's Sec. 3.3 table is about, as it happens on this schedule.  Returns
// the fraction of (XCD, panel) pairs that are reused, per operand.
void later_round_reuse(int64_t tilesM, int64_t tilesN, int order, int64_t per_xcd, int split,
                       double* fracA, double* fracB)
{
    const int64_t T = tilesM * tilesN;
    *fracA = *fracB = 0.0;
    if (T <= 0 || per_xcd <= 0 || T * split > ((int64_t)1 << 24)) return;
    // a claim unit is (XCD, panel, k-slice); workgroup w runs slice w / T of tile w % T
    const int64_t nA = 8 * tilesM * split, nB = 8 * tilesN * split;
    std::vector<int32_t> firstA(nA, -1), firstB(nB, -1);
    std::vector<char> reA(nA, 0), reB(nB, 0);
    for (int64_t w = 0; w < T * split; ++w) {
        const int64_t sl = w / T, wt = w - sl * T;
        int tm, tn;
        fip::tile_coords((int)wt, (int)tilesM, (int)tilesN, fip::kGroupM, order, tm, tn);
        const int64_t x = w & 7;
        const int32_t r = (int32_t)((w >> 3) / per_xcd);
        const int64_t ia = (x * tilesM + tm) * split + sl, ib = (x * tilesN + tn) * split + sl;
        int32_t& fa = firstA[ia];
        if (fa < 0) fa = r; else if (fa != r) reA[ia] = 1;
        int32_t& fb = firstB[ib];
        if (fb < 0) fb = r; else if (fb != r) reB[ib] = 1;
    }
    int64_t tA = 0, uA = 0, tB = 0, uB = 0;
    for (int64_t i = 0; i < nA; ++i) { tA += firstA[i] >= 0; uA += reA[i]; }
    for (int64_t i = 0; i < nB; ++i) { tB += firstB[i] >= 0; uB += reB[i]; }
    *fracA = tA ? (double)uA / tA : 0.0;
    *fracB = tB ? (double)uB / tB : 0.0;
}

// Internal plan: kernel-side quantities plus the caller-facing fip_plan_t.
struct Plan {
    fip_plan_t pub;
    KernelShape ks;
    int elem;
    int mode;
    int kpack_a, kpack_b;           // packing in kernel terms
    int kfrom_a, kfrom_b;           // first packed tile row / column (kernel terms)
    int shared_copy;                // one pack copy for all XCDs
    int64_t tilesKM, tilesKN, nK;
    int64_t off_stats, off_aflag, off_bflag, off_aclaim, off_bclaim, off_apack, off_bpack;
    int64_t apack_copy_elems, bpack_copy_elems;
    int split, slice_ksteps;        // k split (1 = none; not on the 256 tile)
    int order;                      // tile order in effect (FIP_ATTR_ORDER or the planner's)
    int64_t off_part;
};

bool mn_major(bool is_b, int layout, char trans);

// Mixed-precision form of a dtype code, or -1 for FIP_F64 / FIP_F32.
int mx_form_of(int dtype)
{
    switch (dtype) {
    case FIP_BF16: return fip::kMxBF16;
    case FIP_E4M3: return fip::kMxFP8;
    case FIP_BF16X3: return fip::kMxX3;
    case FIP_BF16X3_FAST: return fip::kMxX3Fast;
    default: return -1;
    }
}

bool is_complex(int dtype) { return dtype == FIP_C128 || dtype == FIP_C64; }
bool valid_dtype(int dtype)
{
    return dtype == FIP_F64 || dtype == FIP_F32 || is_complex(dtype) || mx_form_of(dtype) >= 0;
}

// The one exception to packing only fringe panels (binary64 measurements at
// m = n = k = 8192, 8 rounds of 512 resident workgroups): when both operands
// reach the kernel in the same orientation (both K-major or both MN-major),
// the unpacked reads of the two run 1.8-3.2 % slower than packed ones, and
// packing every reused panel on first touch beats both the unpacked launch
// and pack-then-compute; with one operand of each orientation the unpacked
// launch (direct global-to-LDS loads) stays ahead by about 1 %.  At 4096 (2
// rounds) and in binary32 packing gained nothing.  So: binary64, at least
// kWholePackRounds rounds of workgroups, k-loops of at least
// kWholePackKsteps k-steps, operands of one orientation.
constexpr int64_t kWholePackRounds = 8;
constexpr int64_t kWholePackKsteps = 64;

bool whole_panels(const Plan* pl, int layout, char tA, char tB, int64_t resident)
{
    if (pl->elem != 8 || pl->nK < kWholePackKsteps || !pl->shared_copy) return false;
    if (pl->tilesKM * pl->tilesKN * pl->split < kWholePackRounds * resident) return false;
    const bool ka_mn = pl->ks.swapped ? mn_major(true, layout, tB) : mn_major(false, layout, tA);
    const bool kb_mn = pl->ks.swapped ? mn_major(false, layout, tA) : mn_major(true, layout, tB);
    return ka_mn == kb_mn;
}

GemmKey gemm_key(int dtype, int layout, int64_t m, int64_t n, int64_t k, char tA, char tB)
{
    return GemmKey{dtype, layout, m, n, k, is_trans(tA) ? 1 : 0, is_trans(tB) ? 1 : 0};
}

void make_plan(const fip_handle_s* h, int dtype, int layout, int64_t m, int64_t n, int64_t k,
               char tA, char tB, bool standalone_pack, Plan* pl, int policy_override = -1)
{
    memset(pl, 0, sizeof(*pl));
    const int form = mx_form_of(dtype);
    // Tile order: the attribute's, or by default 0 (GROUP_M tiles of a column
    // together), except for the split forms: there an unpacked read redoes the
    // split, and order 1 (the first round touches every column panel of a
    // band once, so later rounds find them packed) measured 20-35 % faster.
    pl->order = h->order >= 0 ? h->order : (form == fip::kMxX3 || form == fip::kMxX3Fast ? 1 : 0);
    pl->ks = kernel_shape(layout, m, n);
    int split_attr = h->split_k;   // FIP_ATTR_SPLIT_K, or a tuned choice below
    // Complex calls (1m method): the kernel multiplies the 2M x 2K expansion of
    // its A side by the 2K x N expansion of its B side, all in real terms.
    const bool cx = is_complex(dtype);
    if (cx) pl->ks.M *= 2;
    const int64_t kr = cx ? 2 * k : k;
    int cls, MT, KT;
    int64_t resident;
    if (form >= 0) {
        // 128 x 128 tiles, or 256 x 256 (bfloat16, E4M3); a packed element is
        // PLANES values of the packed type.  Default: 256 for bfloat16 once
        // the launch fills the device with 256-tiles (one workgroup per CU,
        // 256 tiles): measured ahead of 128 at m = n = k = 4096, 8192 and
        // 16384.  E4M3 takes 256 only when asked: its 128 tile, two per CU,
        // measured faster at 4096 and 16384.
        cls = 0;
        const int64_t big_tiles = cdiv(pl->ks.M, fip::kMxTileBig) * cdiv(pl->ks.N, fip::kMxTileBig);
        const bool big = fip::mx_has_big(form) &&
                         (h->mx_tile == 256 ||
                          (h->mx_tile == -1 && fip::mx_big_default(form) && big_tiles >= 256));
        MT = big ? fip::kMxTileBig : fip::kMxTile;
        KT = fip::mx_kt(form);
        pl->elem = fip::mx_planes(form) * fip::mx_pack_bytes(form);
        resident = 256 * fip::mx_per_cu(form, MT);
    } else {
        pl->elem = dtype == FIP_F64 || dtype == FIP_C128 ? 8 : 4;
        cls = h->tile_override >= 0 ? h->tile_override : choose_tile_class(pl->ks.M, pl->ks.N);
        // a tuned choice for this call shape, unless the attributes force one
        if (h->tuned != nullptr && h->tile_override < 0 && h->split_k == -1) {
            const auto it = h->tuned->find(gemm_key(dtype, layout, m, n, k, tA, tB));
            if (it != h->tuned->end()) {
                cls = it->second.tile;
                split_attr = it->second.split;
            }
        }
        MT = fip::tile_mt(cls);
        KT = fip::tile_kt(cls, pl->elem);
        resident = resident_tiles(cls);
    }
    const int NT = MT;
    pl->tilesKM = cdiv(pl->ks.M, MT);
    pl->tilesKN = cdiv(pl->ks.N, NT);
    pl->nK = cdiv(kr, KT);

    // Split k: when the tiles leave most of the device idle, k is cut into
    // slices, one workgroup per (tile, slice), up to the resident count; a
    // second kernel sums the slices' partial products.  FP64/FP32: at most
    // half the resident workgroups busy, slices of at least kMinSliceKsteps
    // k-steps.  Mixed forms (128 tile only): at most a quarter busy (their
    // MFMA time per slice is short against the partial planes' traffic).
    // The split forms take slices of >= 256 k: their first pass splits every
    // binary32 operand element, and `split` times as many CUs share that work
    // (measured 2.7x at m = n = k = 1024).  bfloat16 and E4M3 only copy, so
    // short slices bring them nothing (E4M3 at 1024 with 256-k slices was
    // 30 % slower): >= 1024 k.  The choice depends on the shape only (not on
    // the pack policy), so every policy runs the same arithmetic.
    pl->split = 1;
    pl->slice_ksteps = (int)pl->nK;
    if ((form < 0 || MT == fip::kMxTile) && pl->nK > 1 && !cx) {
        const int64_t tiles = pl->tilesKM * pl->tilesKN;
        const int64_t busy = form < 0 ? 2 : 4;
        const bool splits = form == fip::kMxX3 || form == fip::kMxX3Fast;
        const int64_t min_slice = form < 0 ? kMinSliceKsteps
                                           : std::max<int64_t>(1, (splits ? kMinSliceKSplit : kMinSliceKCopy) / KT);
        int64_t sp = 1;
        if (split_attr > 0) {
            sp = split_attr;
        } else if (split_attr == -1 && tiles > 0 && busy * tiles <= resident) {
            sp = resident / tiles;
            if (sp > pl->nK / min_slice) sp = pl->nK / min_slice;
            if (sp > kMaxSplit) sp = kMaxSplit;
        }
        if (sp > pl->nK) sp = pl->nK;
        if (sp >= 2) {
            const int64_t per = cdiv(pl->nK, sp);
            pl->slice_ksteps = (int)per;
            pl->split = (int)cdiv(pl->nK, per);   // no empty slice
        }
    }

    int policy = standalone_pack ? FIP_PACK_CONSUME_ONLY
                 : policy_override >= 0 ? policy_override : h->policy;
    // Under stream capture a fused call runs unpacked: its claims and flags are
    // stamped with an epoch chosen on the host per call, and every replay of a
    // captured launch would carry the same one, so a replay would take the
    // previous replay's flags for its own and read packs of old data.
    if ((policy == FIP_PACK_AUTO || policy == FIP_PACK_ALL) && stream_capturing(h->stream))
        policy = FIP_PACK_NONE;
    int copies = 0;
    if (policy == FIP_PACK_CONSUME_ONLY) {
        pl->mode = fip::kModeConsumePacked;
        pl->kpack_a = pl->kpack_b = 1;
        copies = 1;
    } else if (policy == FIP_PACK_NONE) {
        pl->mode = fip::kModeUnpacked;
    } else {
        pl->mode = fip::kModeFused;
        if (policy == FIP_PACK_ALL) {
            pl->kpack_a = pl->kpack_b = 1;
        } else {
            // Paper Sec. 3.3: pack A's panel only if several tile columns of C
            // reuse it (n > n_R), B's panel only if several tile rows do (m > m_R).
            // On the GPU the tiles of one launch run concurrently: a later pass
            // can read a packed panel without waiting only if it starts after
            // the first pass finished, i.e. in a later round of workgroups on
            // the same XCD (each XCD keeps its own copy).  The planner replays
            // the launch order and packs an operand when most of its panels are
            // read again in a later round; with a single round nobody could
            // reuse a pack.
            // The split forms need more than 4 rounds: each XCD produces its own
            // copy of every panel it reads, a producer costs about three packed
            // tiles, and with few rounds that is not repaid (2-term split at
            // 4096^3, 4 rounds: 932 us packed, 773 unpacked; 8192^3, 16 rounds:
            // 6.5 ms packed, 7.4 unpacked).
            const bool split_form = form == fip::kMxX3 || form == fip::kMxX3Fast;
            // One pack copy shared by all XCDs unless the attribute asks for one
            // per XCD.  Per-XCD copies make every XCD produce its own copy of
            // each panel it reads; for the split forms a producer costs about
            // three packed tiles, which fewer than 5 rounds do not repay.
            pl->shared_copy = h->copies != fip::kCopies;
            const bool later_passes =
                pl->tilesKM * pl->tilesKN * pl->split >
                    (split_form && !pl->shared_copy ? 4 : 1) * resident &&
                pl->nK >= kMinPackKsteps;
            double fa = 0.0, fb = 0.0;
            if (later_passes)
                later_round_reuse(pl->tilesKM, pl->tilesKN, pl->order, resident / fip::kCopies,
                                  pl->split, &fa, &fb);
            const bool reuse_a = pl->tilesKN > 1 && fa >= 0.5;
            const bool reuse_b = pl->tilesKM > 1 && fb >= 0.5;
            // Sec. 3.3's stride conditions, read for this GPU: a reused
            // panel is packed only where its unpacked read is slower than a
            // packed one would be.
            //  - The split forms: an unpacked read redoes the binary32 split,
            //    a packed one reads the terms: every reused panel is packed.
            //  - Otherwise the unpacked read of an interior chunk is as
            //    coalesced as the packed one, whatever the transposes: each
            //    of its rows (the k-rows of an MN-major operand, the MN-rows of
            //    a K-major one) is one contiguous run of at least a 128-byte
            //    line (MT or NT times the element size is 256 bytes or more;
            //    KT times it is 128 bytes in every form), and a panel's runs
            //    span as many lines as the packed copy, plus at most one per
            //    row that the next k-step reads from the XCD's L2.  So only a
            //    fringe panel (the operand's M or N extent not a multiple of
            //    the tile) is packed: its unpacked chunks take the masked,
            //    zero-filling loads, its packed chunks are zero padded and
            //    read with the same unmasked loads as any other.  Measured
            //    exception: binary64 launches of many rounds whose operands
            //    share one orientation pack every reused panel (whole_panels).
            //  - Complex operands (1m): a chunk that keeps whole complex
            //    elements in its vectors (the A side, a K-major B side) is
            //    loaded raw and arranged after the step's MFMAs, as fast as a
            //    packed read (binary64 at 4096^3: 9.74 ms unpacked, 9.78 ms
            //    packing the A side); an MN-major B side takes one component
            //    of two loads per vector and is arranged before its MFMAs, so
            //    its reused panels are packed.  Fringe panels as below.
            if (split_form) {
                pl->kpack_a = reuse_a;
                pl->kpack_b = reuse_b;
            } else if (cx) {
                const bool kb_mn = pl->ks.swapped ? mn_major(false, layout, tA) : mn_major(true, layout, tB);
                pl->kpack_a = reuse_a && pl->ks.M % MT != 0;
                pl->kpack_b = reuse_b && (pl->ks.N % NT != 0 || kb_mn);
                pl->kfrom_a = (int)pl->tilesKM - 1;
                pl->kfrom_b = kb_mn ? 0 : (int)pl->tilesKN - 1;
            } else if (whole_panels(pl, layout, tA, tB, resident)) {
                // the reuse table itself (n > n_R, m > m_R): with one copy for
                // the device and 8 or more rounds, every panel of an operand
                // that several tiles read is read again in a later round
                pl->kpack_a = pl->tilesKN > 1;
                pl->kpack_b = pl->tilesKM > 1;
                pl->kfrom_a = pl->kfrom_b = 0;
            } else {
                pl->kpack_a = reuse_a && pl->ks.M % MT != 0;
                pl->kpack_b = reuse_b && pl->ks.N % NT != 0;
                pl->kfrom_a = (int)pl->tilesKM - 1;
                pl->kfrom_b = (int)pl->tilesKN - 1;
            }
        }
        if (policy == FIP_PACK_ALL) pl->shared_copy = h->copies != fip::kCopies;
        if (pl->kpack_a || pl->kpack_b) copies = pl->shared_copy ? 1 : fip::kCopies;
        else pl->shared_copy = 0;
    }
    if (k == 0 || m == 0 || n == 0) { pl->kpack_a = pl->kpack_b = 0; copies = 0; }
    if (!pl->kpack_a) pl->kfrom_a = 0;
    if (!pl->kpack_b) pl->kfrom_b = 0;

    if (k == 0 || m == 0 || n == 0) { pl->split = 1; pl->slice_ksteps = (int)pl->nK; }
    const bool fz = pl->mode == fip::kModeFused;
    const int64_t sp = pl->split;
    int64_t off = 0;
    pl->off_stats = off; off = align256(off + 4 * 8);
    pl->off_aflag = off; off = align256(off + (pl->kpack_a && fz ? copies * pl->tilesKM * sp * 8 : 0));
    pl->off_bflag = off; off = align256(off + (pl->kpack_b && fz ? copies * pl->tilesKN * sp * 8 : 0));
    pl->off_aclaim = off; off = align256(off + (pl->kpack_a && fz ? copies * pl->tilesKM * sp * 8 : 0));
    pl->off_bclaim = off; off = align256(off + (pl->kpack_b && fz ? copies * pl->tilesKN * sp * 8 : 0));
    pl->apack_copy_elems = pl->kpack_a ? (pl->tilesKM - pl->kfrom_a) * pl->nK * KT * MT : 0;
    pl->bpack_copy_elems = pl->kpack_b ? (pl->tilesKN - pl->kfrom_b) * pl->nK * KT * NT : 0;
    pl->off_apack = off; off = align256(off + copies * pl->apack_copy_elems * pl->elem);
    pl->off_bpack = off; off = align256(off + copies * pl->bpack_copy_elems * pl->elem);
    // slice partials: the output type's accumulator (binary32 for the mixed forms)
    const int64_t part_elem = form >= 0 ? 4 : pl->elem;
    pl->off_part = off; off = align256(off + (sp > 1 ? sp * pl->ks.M * pl->ks.N * part_elem : 0));

    fip_plan_t& p = pl->pub;
    p.dtype = dtype; p.layout = layout; p.m = m; p.n = n; p.k = k;
    p.tile_class = cls;
    p.MT = MT; p.NT = NT; p.KT = KT;
    p.ksteps = (int32_t)pl->nK;
    p.copies = copies;
    p.policy = policy;
    p.stats_offset = pl->off_stats;
    // packed block orientation: the operand's own (every form)
    p.a_kmajor = !mn_major(false, layout, tA);
    p.b_kmajor = !mn_major(true, layout, tB);
    const bool fl = pl->mode == fip::kModeFused;
    p.workspace_bytes = (pl->kpack_a || pl->kpack_b || pl->split > 1) ? off : 0;
    p.split_k = pl->split;
    p.slice_ksteps = pl->slice_ksteps;
    p.partial_offset = pl->split > 1 ? pl->off_part : -1;
    // Report in the caller's terms: op(A) is the kernel's B-side when swapped.
    if (!pl->ks.swapped) {
        p.tiles_m = (int32_t)pl->tilesKM; p.tiles_n = (int32_t)pl->tilesKN;
        p.pack_a = pl->kpack_a; p.pack_b = pl->kpack_b;
        p.a_pack_first = pl->kfrom_a; p.b_pack_first = pl->kfrom_b;
        p.a_pack_offset = pl->off_apack; p.a_copy_bytes = pl->apack_copy_elems * pl->elem;
        p.b_pack_offset = pl->off_bpack; p.b_copy_bytes = pl->bpack_copy_elems * pl->elem;
        p.a_flag_offset = fl ? pl->off_aflag : -1; p.b_flag_offset = fl ? pl->off_bflag : -1;
        p.a_claim_offset = fl ? pl->off_aclaim : -1; p.b_claim_offset = fl ? pl->off_bclaim : -1;
    } else {
        p.tiles_m = (int32_t)pl->tilesKN; p.tiles_n = (int32_t)pl->tilesKM;
        p.pack_a = pl->kpack_b; p.pack_b = pl->kpack_a;
        p.a_pack_first = pl->kfrom_b; p.b_pack_first = pl->kfrom_a;
        p.a_pack_offset = pl->off_bpack; p.a_copy_bytes = pl->bpack_copy_elems * pl->elem;
        p.b_pack_offset = pl->off_apack; p.b_copy_bytes = pl->apack_copy_elems * pl->elem;
        p.a_flag_offset = fl ? pl->off_bflag : -1; p.b_flag_offset = fl ? pl->off_aflag : -1;
        p.a_claim_offset = fl ? pl->off_bclaim : -1; p.b_claim_offset = fl ? pl->off_aclaim : -1;
        int32_t t = p.MT; p.MT = p.NT; p.NT = t;
    }
}

// Validation of the BLAS-style argument list; returns the 1-based position of
// the first invalid argument (handle = 1, layout = pos0) or 0.  Leading
// dimensions are only judged once the transposes they depend on are valid.
int check_args(int pos0, int layout, int64_t m, int64_t n, int64_t k, bool alpha_nonzero,
               const void* A, int64_t lda, char tA, const void* B, int64_t ldb, char tB,
               bool check_c, bool beta_one, const void* C, int64_t ldc)
{
    // positions relative to layout: m+1, n+2, k+3, alpha+4, A+5, lda+6, tA+7,
    // B+8, ldb+9, tB+10, beta+11, C+12, ldc+13
    if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return pos0;
    if (m < 0) return pos0 + 1;
    if (n < 0) return pos0 + 2;
    if (k < 0) return pos0 + 3;
    const bool tA_ok = valid_trans(tA), tB_ok = valid_trans(tB);
    const bool col = layout == FIP_COL_MAJOR;
    const bool reads_ab = m > 0 && n > 0 && k > 0 && alpha_nonzero;
    const bool writes_c = check_c && m > 0 && n > 0 && !(beta_one && !reads_ab);
    if (reads_ab && A == nullptr) return pos0 + 5;
    if (tA_ok) {
        const int64_t need = col ? (is_trans(tA) ? k : m) : (is_trans(tA) ? m : k);
        if (lda < max1(need)) return pos0 + 6;
    }
    if (!tA_ok) return pos0 + 7;
    if (reads_ab && B == nullptr) return pos0 + 8;
    if (tB_ok) {
        const int64_t need = col ? (is_trans(tB) ? n : k) : (is_trans(tB) ? k : n);
        if (ldb < max1(need)) return pos0 + 9;
    }
    if (!tB_ok) return pos0 + 10;
    if (check_c) {
        if (writes_c && C == nullptr) return pos0 + 12;
        if (ldc < max1(col ? m : n)) return pos0 + 13;
    }
    return 0;
}

// Whether op(X)'s storage runs along its MN index (M for op(A), N for op(B)).
// op(X)[r, c] is stored element (r, c) for 'N' and (c, r) for 'T'/'C'; column-
// major storage runs along the stored row index, row-major along the column.
bool mn_major(bool is_b, int layout, char trans)
{
    const int runs_along = (layout == FIP_ROW_MAJOR) ^ (int)is_trans(trans);  // 0 = r, 1 = c
    return runs_along == (is_b ? 1 : 0);
}

// Fill the kernel descriptor's operand fields (kernel A-side/B-side).  An
// MN-major operand has element (x, p) at X[x + p*ld], a K-major one at
// X[x*ld + p].
void fill_operands(const Plan& pl, int layout, const void* A, int64_t lda, char tA, const void* B,
                   int64_t ldb, char tB, fip::LaunchDesc* d)
{
    const bool a_mn = mn_major(false, layout, tA), b_mn = mn_major(true, layout, tB);
    auto set = [](bool mn, const void* X, int64_t ld, const void** P, int64_t* smn, int64_t* sk,
                  int* kmajor) {
        *P = X;
        *smn = mn ? 1 : ld;
        *sk = mn ? ld : 1;
        *kmajor = !mn;
    };
    if (!pl.ks.swapped) {
        set(a_mn, A, lda, &d->A, &d->a_smn, &d->a_sk, &d->a_kmajor);
        set(b_mn, B, ldb, &d->B, &d->b_smn, &d->b_sk, &d->b_kmajor);
    } else {
        set(b_mn, B, ldb, &d->A, &d->a_smn, &d->a_sk, &d->a_kmajor);
        set(a_mn, A, lda, &d->B, &d->b_smn, &d->b_sk, &d->b_kmajor);
    }
}

void fill_workspace(void* base, const Plan& pl, fip::LaunchDesc* d)
{
    char* ws = static_cast<char*>(base);
    d->stats_ptr = reinterpret_cast<unsigned long long*>(ws + pl.off_stats);
    d->aflag = reinterpret_cast<uint64_t*>(ws + pl.off_aflag);
    d->bflag = reinterpret_cast<uint64_t*>(ws + pl.off_bflag);
    d->aclaim = reinterpret_cast<uint64_t*>(ws + pl.off_aclaim);
    d->bclaim = reinterpret_cast<uint64_t*>(ws + pl.off_bclaim);
    d->apack = ws + pl.off_apack;
    d->bpack = ws + pl.off_bpack;
    d->apack_copy_elems = pl.apack_copy_elems;
    d->bpack_copy_elems = pl.bpack_copy_elems;
    if (pl.split > 1) d->part = ws + pl.off_part;
}

int prepare_workspace(fip_handle_s* h, const Plan& pl)
{
    if (pl.pub.workspace_bytes == 0) return 0;
    if (h->ws == nullptr || (int64_t)h->ws_bytes < pl.pub.workspace_bytes) return FIP_ERR_WORKSPACE;
    return 0;
}

// noalloc: run on the library's scratch array (fip_dgemm_noalloc) instead of
// the handle's workspace.
template <typename T>
int gemm_impl(fip_handle_t h, int dtype, int layout, int64_t m, int64_t n, int64_t k, T alpha,
              const T* A, int64_t lda, char tA, const T* B, int64_t ldb, char tB, T beta, T* C,
              int64_t ldc, bool noalloc = false)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        const int bad = check_args(2, layout, m, n, k, alpha != T(0), A, lda, tA, B, ldb, tB, true,
                                   beta == T(1), C, ldc);
        if (bad) return bad;
        if (m == 0 || n == 0) return 0;
        if ((alpha == T(0) || k == 0) && beta == T(1)) return 0;
        const KernelShape ks = kernel_shape(layout, m, n);
        if (alpha == T(0) || k == 0) {
            if (const hipError_t e = fip::launch_scale(sizeof(T), ks.M, ks.N, C, ldc, (double)beta,
                                                       h->stream); e != hipSuccess)
                return launch_failed(h, e);
            return 0;
        }
        Plan pl;
        make_plan(h, dtype, layout, m, n, k, tA, tB, false, &pl);
        void* ws_base = h->ws;
        if (noalloc) {
            // The scratch array replaces the workspace.  A plan whose packed
            // panels would not fit runs unpacked (the same kernel and k order,
            // so the same C bit for bit); one whose split-k partials alone
            // exceed the array is rejected before anything is launched.
            if (pl.pub.workspace_bytes > fip::kScratchBytes && pl.mode == fip::kModeFused)
                make_plan(h, dtype, layout, m, n, k, tA, tB, false, &pl, FIP_PACK_NONE);
            if (pl.pub.workspace_bytes > fip::kScratchBytes) return FIP_ERR_WORKSPACE;
            if (pl.pub.workspace_bytes > 0) {
                if (const hipError_t e = fip::scratch_buffer(&ws_base); e != hipSuccess)
                    return launch_failed(h, e);
            }
        } else if (const int ws = prepare_workspace(h, pl); ws) {
            return ws;
        }
        fip::LaunchDesc d;
        memset(&d, 0, sizeof(d));
        d.elem = sizeof(T);
        d.tile_class = pl.pub.tile_class;
        d.mode = pl.mode;
        d.pack_a = pl.kpack_a; d.pack_b = pl.kpack_b;
        d.a_pack_from = pl.kfrom_a; d.b_pack_from = pl.kfrom_b;
        d.shared_copy = pl.shared_copy;
        d.no_publish = h->no_publish;
        d.stats = noalloc ? 0 : h->stats;   // the scratch array's counters are never cleared
        d.order = pl.order;
        d.dma = h->dma;
        d.used_dma = &h->last_dma;
        d.M = ks.M; d.N = ks.N; d.K = k;
        fill_operands(pl, layout, A, lda, tA, B, ldb, tB, &d);
        d.C = C; d.ldc = ldc;
        d.alpha = (double)alpha; d.beta = (double)beta;
        d.split = pl.split;
        d.slice_ksteps = pl.slice_ksteps;
        if (pl.pub.workspace_bytes > 0) {
            fill_workspace(ws_base, pl, &d);
            if (pl.mode == fip::kModeFused) d.epoch = h->epoch = next_epoch();
        } else {
            d.stats = 0;
        }
        d.stream = h->stream;
        if (const hipError_t e = fip::launch_gemm(d); e != hipSuccess) return launch_failed(h, e);
        h->last = pl.pub;
        h->has_last = 1;
        return 0;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

// Complex GEMM through the 1m method (paper Sec. 5: complex multiplication
// encoded in the packing, the real microkernel unchanged).  The tile kernel's
// A side is the 2M x 2K real expansion of op(A) (each element a 2 x 2 block
// [[re, -im], [im, re]]), its B side the 2K x N expansion of op(B) (each
// element its (re, im) pair along k), and their real product is the real view
// of column-major complex C (rows 2i, 2i + 1: re, im of row i).  Row-major C
// is handled as C^T = op(B)^T op(A)^T like the real path: op(X)^T of a
// conjugate transpose is conj(X), so each side carries a conjugation flag.
// The expansion happens in the loads; a packed panel holds it.  alpha and
// beta are (re, im) pairs on the host.
template <typename T>
int zgemm_impl(fip_handle_t h, int dtype, int layout, int64_t m, int64_t n, int64_t k,
               const T* alpha, const T* A, int64_t lda, char tA, const T* B, int64_t ldb,
               char tB, const T* beta, T* C, int64_t ldc)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        // positions: layout 2, m 3, n 4, k 5, alpha 6, A 7, lda 8, transA 9, B 10, ldb 11,
        // transB 12, beta 13, C 14, ldc 15
        if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
        if (alpha == nullptr) return 6;
        if (beta == nullptr) return 13;
        const bool a_nz = alpha[0] != T(0) || alpha[1] != T(0);
        const bool b_one = beta[0] == T(1) && beta[1] == T(0);
        const int bad = check_args(2, layout, m, n, k, a_nz, A, lda, tA, B, ldb, tB, true, b_one,
                                   C, ldc);
        if (bad) return bad;
        if (m == 0 || n == 0) return 0;
        if ((!a_nz || k == 0) && b_one) return 0;
        const bool no_ab = !a_nz || k == 0;   // C := beta C, A and B not read
        Plan pl;
        make_plan(h, dtype, layout, m, n, no_ab ? 0 : k, tA, tB, false, &pl);
        if (const int ws = prepare_workspace(h, pl); ws) return ws;
        fip::LaunchDesc d;
        memset(&d, 0, sizeof(d));
        d.elem = sizeof(T);
        d.kind = fip::k1m;
        d.tile_class = pl.pub.tile_class;
        d.mode = pl.mode;
        d.pack_a = pl.kpack_a; d.pack_b = pl.kpack_b;
        d.a_pack_from = pl.kfrom_a; d.b_pack_from = pl.kfrom_b;
        d.shared_copy = pl.shared_copy;
        d.no_publish = h->no_publish;
        d.stats = h->stats;
        d.order = pl.order;
        d.M = pl.ks.M;                 // 2 x the kernel's complex rows
        d.N = pl.ks.N;
        d.K = no_ab ? 0 : 2 * k;
        // operand strides in complex elements, as the real path sets them
        fill_operands(pl, layout, A, lda, tA, B, ldb, tB, &d);
        // conjugation per kernel side: op 'C' conjugates; on the swapped
        // (row-major) path the side holds op(X)^T, conjugated for 'C' as well
        const bool ca = tA == 'C' || tA == 'c', cb = tB == 'C' || tB == 'c';
        d.conj_a = pl.ks.swapped ? cb : ca;
        d.conj_b = pl.ks.swapped ? ca : cb;
        d.C = C; d.ldc = ldc;
        d.alpha = no_ab ? 0.0 : (double)alpha[0];
        d.alpha_im = no_ab ? 0.0 : (double)alpha[1];
        d.beta = (double)beta[0]; d.beta_im = (double)beta[1];
        d.split = 1;
        d.slice_ksteps = (int)pl.nK;
        if (pl.pub.workspace_bytes > 0) {
            fill_workspace(h->ws, pl, &d);
            if (pl.mode == fip::kModeFused) d.epoch = h->epoch = next_epoch();
        } else {
            d.stats = 0;
        }
        d.stream = h->stream;
        if (const hipError_t e = fip::launch_gemm(d); e != hipSuccess) return launch_failed(h, e);
        h->last = pl.pub;
        h->has_last = 1;
        return 0;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

// Kernel descriptor of a mixed-precision call (operands, workspace, stream);
// the caller fills C, alpha, beta, scales and the epoch.
void fill_mx_desc(const fip_handle_s* h, const Plan& pl, int form, int layout, int64_t k,
                  const void* A, int64_t lda, char tA, const void* B, int64_t ldb, char tB,
                  fip::MxLaunchDesc* d)
{
    memset(d, 0, sizeof(*d));
    d->form = form;
    d->mt = pl.pub.MT;
    d->mode = pl.mode;
    d->pack_a = pl.kpack_a; d->pack_b = pl.kpack_b;
    d->a_pack_from = pl.kfrom_a; d->b_pack_from = pl.kfrom_b;
    d->shared_copy = pl.shared_copy;
    d->no_publish = h->no_publish;
    d->stats = h->stats;
    d->order = pl.order;
    d->M = pl.ks.M; d->N = pl.ks.N; d->K = k;
    const bool a_mn = mn_major(false, layout, tA), b_mn = mn_major(true, layout, tB);
    if (!pl.ks.swapped) {
        d->A = A; d->a_ld = lda; d->a_kmajor = !a_mn;
        d->B = B; d->b_ld = ldb; d->b_kmajor = !b_mn;
    } else {
        d->A = B; d->a_ld = ldb; d->a_kmajor = !b_mn;
        d->B = A; d->b_ld = lda; d->b_kmajor = !a_mn;
    }
    if (pl.pub.workspace_bytes > 0) {
        char* ws = static_cast<char*>(h->ws);
        d->stats_ptr = reinterpret_cast<unsigned long long*>(ws + pl.off_stats);
        d->aflag = reinterpret_cast<uint64_t*>(ws + pl.off_aflag);
        d->bflag = reinterpret_cast<uint64_t*>(ws + pl.off_bflag);
        d->aclaim = reinterpret_cast<uint64_t*>(ws + pl.off_aclaim);
        d->bclaim = reinterpret_cast<uint64_t*>(ws + pl.off_bclaim);
        d->apack = ws + pl.off_apack;
        d->bpack = ws + pl.off_bpack;
        d->apack_copy_bytes = pl.apack_copy_elems * pl.elem;
        d->bpack_copy_bytes = pl.bpack_copy_elems * pl.elem;
        if (pl.split > 1) d->part = ws + pl.off_part;
    } else {
        d->stats = 0;
    }
    d->split = pl.split;
    d->slice_ksteps = pl.slice_ksteps;
    d->stream = h->stream;
}

int gemm_mx_impl(fip_handle_t h, int dtype, int layout, int64_t m, int64_t n, int64_t k,
                 float alpha, const void* A, int64_t lda, char tA, const void* B, int64_t ldb,
                 char tB, float beta, void* C, int64_t ldc, int c_type, const float* a_scale,
                 const float* b_scale)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        const int form = mx_form_of(dtype);
        if (form < 0) return 2;
        // positions: layout 3, m 4, n 5, k 6, alpha 7, A 8, lda 9, transA 10, B 11, ldb 12,
        // transB 13, beta 14, C 15, ldc 16, c_type 17, a_scale 18, b_scale 19
        const int bad = check_args(3, layout, m, n, k, alpha != 0.f, A, lda, tA, B, ldb, tB, true,
                                   beta == 1.f, C, ldc);
        if (bad) return bad;
        if (c_type != FIP_F32 && c_type != FIP_BF16) return 17;
        if (form != fip::kMxFP8 && a_scale != nullptr) return 18;
        if (form != fip::kMxFP8 && b_scale != nullptr) return 19;
        if (m == 0 || n == 0) return 0;
        if ((alpha == 0.f || k == 0) && beta == 1.f) return 0;
        const KernelShape ks = kernel_shape(layout, m, n);
        const int c_bf16 = c_type == FIP_BF16;
        if (alpha == 0.f || k == 0) {
            if (const hipError_t e = fip::launch_scale_mx(c_bf16, ks.M, ks.N, C, ldc, beta, h->stream);
                e != hipSuccess)
                return launch_failed(h, e);
            return 0;
        }
        Plan pl;
        make_plan(h, dtype, layout, m, n, k, tA, tB, false, &pl);
        const int ws = prepare_workspace(h, pl);
        if (ws) return ws;
        fip::MxLaunchDesc d;
        fill_mx_desc(h, pl, form, layout, k, A, lda, tA, B, ldb, tB, &d);
        d.C = C; d.ldc = ldc; d.c_bf16 = c_bf16;
        d.alpha = alpha; d.beta = beta;
        // per row of op(A) / column of op(B); the kernel's A-side is op(B)^T
        // when the operands are swapped for row-major storage
        d.a_scale = ks.swapped ? b_scale : a_scale;
        d.b_scale = ks.swapped ? a_scale : b_scale;
        if (pl.pub.workspace_bytes > 0 && pl.mode == fip::kModeFused) d.epoch = h->epoch = next_epoch();
        if (const hipError_t e = fip::launch_gemm_mx(d); e != hipSuccess) return launch_failed(h, e);
        h->last = pl.pub;
        h->has_last = 1;
        return 0;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

// ---- other level-3 operations: SYRK and TRMM -------------------------------------

bool valid_uplo(char u) { return u == 'L' || u == 'l' || u == 'U' || u == 'u'; }
bool valid_side(char c) { return c == 'L' || c == 'l' || c == 'R' || c == 'r'; }
bool valid_diag(char c) { return c == 'N' || c == 'n' || c == 'U' || c == 'u'; }
bool is_lower(char u) { return u == 'L' || u == 'l'; }
bool is_left(char c) { return c == 'L' || c == 'l'; }
bool is_unit(char c) { return c == 'U' || c == 'u'; }

// One SYRK or TRMM call in kernel terms (column-major kernel C, see the
// operation's entry point for how the caller's storage maps onto it).
struct L3Shape {
    int kind;
    int64_t M, N, K;
    int tri_side;       // TRMM: 1 = kernel A side triangular, 2 = B side
    int tri_keep_ge, tri_unit, tri_upper;
    bool a_mn, b_mn;    // kernel operands MN-major
};

// Plan of a SYRK / TRMM call: the GEMM planner's tile class, no split k, and
// Sec. 3.3's rule for the one operand that may be packed (SYRK: the single
// operand, whose pack both sides read; TRMM: the triangular one, whose chunks
// the pack holds with the triangle applied; the dense TRMM operand is never
// packed, because tiles with different k-ranges read different parts of its
// panels).  pub reports the caller's A as op(A) (SYRK) or the triangular matrix.
void make_plan_l3(const fip_handle_s* h, int dtype, const L3Shape& ls, Plan* pl)
{
    memset(pl, 0, sizeof(*pl));
    pl->elem = dtype == FIP_F64 ? 8 : 4;
    const int cls = h->tile_override >= 0 ? h->tile_override : choose_tile_class(ls.M, ls.N);
    const int MT = fip::tile_mt(cls), KT = fip::tile_kt(cls, pl->elem);
    const int64_t resident = resident_tiles(cls);
    pl->ks = KernelShape{ls.M, ls.N, false};
    pl->tilesKM = cdiv(ls.M, MT);
    pl->tilesKN = cdiv(ls.N, MT);
    pl->nK = cdiv(ls.K, KT);
    pl->split = 1;
    pl->slice_ksteps = (int)pl->nK;
    pl->order = 0;
    const int64_t tiles = ls.kind == fip::kSyrk ? pl->tilesKM * (pl->tilesKM + 1) / 2
                                                : pl->tilesKM * pl->tilesKN;
    int policy = h->policy;
    if ((policy == FIP_PACK_AUTO || policy == FIP_PACK_ALL) && stream_capturing(h->stream))
        policy = FIP_PACK_NONE;
    // the packable operand in kernel terms: SYRK and side-L TRMM the A side
    const bool on_a = ls.kind == fip::kSyrk || ls.tri_side == 1;
    const int64_t ext = on_a ? ls.M : ls.N, ptiles = on_a ? pl->tilesKM : pl->tilesKN;
    int pk = 0, from = 0;
    if (ls.K > 0 && ls.M > 0 && ls.N > 0) {
        if (policy == FIP_PACK_ALL) {
            pk = 1;
        } else if (policy == FIP_PACK_AUTO) {
            // reused by later rounds, a k-loop of at least kMinPackKsteps, and
            // (the stride rule) only the fringe panel, whose unpacked chunks
            // take the masked loads
            pk = tiles > resident && pl->nK >= kMinPackKsteps && ptiles > 1 && ext % MT != 0;
            from = (int)ptiles - 1;
        }
    }
    if (!pk) from = 0;
    pl->mode = policy == FIP_PACK_NONE ? fip::kModeUnpacked : fip::kModeFused;
    pl->shared_copy = h->copies != fip::kCopies;
    const int copies = pk ? (pl->shared_copy ? 1 : fip::kCopies) : 0;
    pl->kpack_a = on_a && pk;
    pl->kpack_b = (!on_a || ls.kind == fip::kSyrk) && pk;
    pl->kfrom_a = pl->kfrom_b = from;
    int64_t off = 0;
    pl->off_stats = off; off = align256(off + 4 * 8);
    const int64_t flags = pk ? copies * ptiles * 8 : 0;
    pl->off_aflag = off; off = align256(off + flags);
    pl->off_aclaim = off; off = align256(off + flags);
    const int64_t copy_elems = pk ? (ptiles - from) * pl->nK * KT * MT : 0;
    pl->off_apack = off; off = align256(off + copies * copy_elems * pl->elem);
    // one set of flags, claims and pack serves whichever side is packed
    pl->off_bflag = pl->off_aflag; pl->off_bclaim = pl->off_aclaim; pl->off_bpack = pl->off_apack;
    pl->apack_copy_elems = pl->kpack_a ? copy_elems : 0;
    pl->bpack_copy_elems = pl->kpack_b ? copy_elems : 0;
    pl->off_part = off;

    fip_plan_t& p = pl->pub;
    p.dtype = dtype;
    p.m = ls.kind == fip::kSyrk ? ls.M : 0;
    p.k = ls.K;
    p.MT = p.NT = MT; p.KT = KT;
    p.tiles_m = (int32_t)pl->tilesKM; p.tiles_n = (int32_t)pl->tilesKN;
    p.ksteps = (int32_t)pl->nK;
    p.tile_class = cls;
    p.pack_a = pk; p.pack_b = ls.kind == fip::kSyrk ? pk : 0;
    p.a_pack_first = from; p.b_pack_first = ls.kind == fip::kSyrk ? from : 0;
    p.copies = copies;
    p.policy = policy;
    p.a_kmajor = on_a ? !ls.a_mn : !ls.b_mn;
    p.b_kmajor = ls.kind == fip::kSyrk ? !ls.a_mn : (on_a ? !ls.b_mn : !ls.a_mn);
    p.a_pack_offset = pl->off_apack; p.a_copy_bytes = copy_elems * pl->elem;
    p.b_pack_offset = pl->off_apack; p.b_copy_bytes = ls.kind == fip::kSyrk ? copy_elems * pl->elem : 0;
    const bool fl = pk && pl->mode == fip::kModeFused;
    p.a_flag_offset = fl ? pl->off_aflag : -1; p.b_flag_offset = p.a_flag_offset;
    p.a_claim_offset = fl ? pl->off_aclaim : -1; p.b_claim_offset = p.a_claim_offset;
    p.stats_offset = pl->off_stats;
    p.workspace_bytes = pk ? off : 0;
    p.split_k = 1;
    p.slice_ksteps = (int32_t)pl->nK;
    p.partial_offset = -1;
}

// SYRK in kernel terms.  Row-major storage is the column-major view of the
// transposed matrices: op(A) keeps its strides and C's view holds the other
// triangle (the product is symmetric).
L3Shape syrk_shape(int layout, char uplo, char trans, int64_t n, int64_t k)
{
    L3Shape ls{};
    ls.kind = fip::kSyrk;
    ls.M = ls.N = n;
    ls.K = k;
    const bool lower = is_lower(uplo) != (layout == FIP_ROW_MAJOR);
    ls.tri_upper = !lower;
    ls.a_mn = ls.b_mn = mn_major(false, layout, trans);
    return ls;
}

// TRMM in kernel terms.  Row-major storage is the column-major view of the
// transposed matrices: the side and the triangle swap and m, n exchange.  On
// the column-major views, side L computes op(T) B (T on the kernel A side,
// element (x, p) = op(T)[x, p]) and side R computes B op(T) (T on the B side,
// element (p, x) = op(T)[p, x]); T's stored (row, col) is (x, p) or (p, x)
// depending on the transpose, so the kept triangle is x >= p exactly when
// lower XOR transposed (side L), or its negation (side R).
L3Shape trmm_shape(int layout, char side, char uplo, char transA, char diag, int64_t m, int64_t n)
{
    L3Shape ls{};
    ls.kind = fip::kTrmm;
    const bool row = layout == FIP_ROW_MAJOR;
    const bool left = is_left(side) != row, lower = is_lower(uplo) != row;
    const bool tr = is_trans(transA);
    ls.M = row ? n : m;
    ls.N = row ? m : n;
    ls.K = left ? ls.M : ls.N;
    ls.tri_side = left ? 1 : 2;
    ls.tri_keep_ge = left ? (lower != tr) : !(lower != tr);
    ls.tri_unit = is_unit(diag);
    // kernel operands: T (column-major view, element (r, c) at A[r + c*lda]) and
    // B's column-major view (element (r, c) at B[r + c*ldb])
    if (left) {
        ls.a_mn = !tr;   // op(T)[x, p]: A[x + p*lda] ('N'), A[p + x*lda] ('T')
        ls.b_mn = false; // B[p + x*ldb]: K-major
    } else {
        ls.a_mn = true;  // B[x + p*ldb]: MN-major
        ls.b_mn = tr;    // op(T)[p, x]: A[p + x*lda] ('N', K-major), A[x + p*lda] ('T')
    }
    return ls;
}

template <typename T>
int run_l3(fip_handle_t h, int dtype, const L3Shape& ls, T alpha, const T* A, int64_t lda,
           const T* B, int64_t ldb, T beta, T* C, int64_t ldc)
{
    const bool no_ab = alpha == T(0) || ls.K == 0;
    L3Shape run = ls;
    if (no_ab) run.K = 0;   // C := beta*C on the computed entries, A and B not read
    Plan pl;
    make_plan_l3(h, dtype, run, &pl);
    if (const int ws = prepare_workspace(h, pl); ws) return ws;
    fip::LaunchDesc d;
    memset(&d, 0, sizeof(d));
    d.elem = sizeof(T);
    d.tile_class = pl.pub.tile_class;
    d.mode = pl.mode;
    d.pack_a = pl.kpack_a; d.pack_b = pl.kpack_b;
    d.a_pack_from = pl.kfrom_a; d.b_pack_from = pl.kfrom_b;
    d.shared_copy = pl.shared_copy;
    d.no_publish = h->no_publish;
    d.stats = h->stats;
    d.order = 0;
    d.M = run.M; d.N = run.N; d.K = run.K;
    auto set = [](bool mn, const void* X, int64_t ld, const void** P, int64_t* smn, int64_t* sk,
                  int* kmajor) {
        *P = X; *smn = mn ? 1 : ld; *sk = mn ? ld : 1; *kmajor = !mn;
    };
    if (ls.kind == fip::kSyrk) {
        set(ls.a_mn, A, lda, &d.A, &d.a_smn, &d.a_sk, &d.a_kmajor);
        set(ls.b_mn, A, lda, &d.B, &d.b_smn, &d.b_sk, &d.b_kmajor);
    } else if (ls.tri_side == 1) {
        set(ls.a_mn, A, lda, &d.A, &d.a_smn, &d.a_sk, &d.a_kmajor);
        set(ls.b_mn, B, ldb, &d.B, &d.b_smn, &d.b_sk, &d.b_kmajor);
    } else {
        set(ls.a_mn, B, ldb, &d.A, &d.a_smn, &d.a_sk, &d.a_kmajor);
        set(ls.b_mn, A, lda, &d.B, &d.b_smn, &d.b_sk, &d.b_kmajor);
    }
    d.C = C; d.ldc = ldc;
    d.alpha = (double)alpha; d.beta = (double)beta;
    d.split = 1;
    d.slice_ksteps = (int)pl.nK;
    d.kind = ls.kind;
    d.tri_upper = ls.tri_upper;
    d.tri_side = ls.tri_side;
    d.tri_keep_ge = ls.tri_keep_ge;
    d.tri_unit = ls.tri_unit;
    if (pl.pub.workspace_bytes > 0) {
        fill_workspace(h->ws, pl, &d);
        if (pl.mode == fip::kModeFused) d.epoch = h->epoch = next_epoch();
    } else {
        d.stats = 0;
    }
    d.stream = h->stream;
    if (const hipError_t e = fip::launch_gemm(d); e != hipSuccess) return launch_failed(h, e);
    h->last = pl.pub;
    h->has_last = 1;
    return 0;
}

template <typename T>
int syrk_impl(fip_handle_t h, int dtype, int layout, char uplo, char trans, int64_t n, int64_t k,
              T alpha, const T* A, int64_t lda, T beta, T* C, int64_t ldc)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        // positions: layout 2, uplo 3, trans 4, n 5, k 6, alpha 7, A 8, lda 9, beta 10,
        // C 11, ldc 12
        if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
        if (!valid_uplo(uplo)) return 3;
        if (!valid_trans(trans)) return 4;
        if (n < 0) return 5;
        if (k < 0) return 6;
        const bool reads_a = n > 0 && k > 0 && alpha != T(0);
        if (reads_a && A == nullptr) return 8;
        const bool col = layout == FIP_COL_MAJOR;
        if (lda < max1(col != is_trans(trans) ? n : k)) return 9;
        if (n > 0 && !(beta == T(1) && !reads_a) && C == nullptr) return 11;
        if (ldc < max1(n)) return 12;
        if (n == 0) return 0;
        if (!reads_a && beta == T(1)) return 0;
        return run_l3<T>(h, dtype, syrk_shape(layout, uplo, trans, n, k), alpha, A, lda, nullptr,
                         1, beta, C, ldc);
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

template <typename T>
int trmm_impl(fip_handle_t h, int dtype, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, T alpha, const T* A, int64_t lda, const T* B, int64_t ldb,
              T beta, T* C, int64_t ldc)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        // positions: layout 2, side 3, uplo 4, transA 5, diag 6, m 7, n 8, alpha 9, A 10,
        // lda 11, B 12, ldb 13, beta 14, C 15, ldc 16
        if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
        if (!valid_side(side)) return 3;
        if (!valid_uplo(uplo)) return 4;
        if (!valid_trans(transA)) return 5;
        if (!valid_diag(diag)) return 6;
        if (m < 0) return 7;
        if (n < 0) return 8;
        const int64_t ka = is_left(side) ? m : n;
        const bool reads_ab = m > 0 && n > 0 && alpha != T(0);
        if (reads_ab && A == nullptr) return 10;
        if (lda < max1(ka)) return 11;
        if (reads_ab && B == nullptr) return 12;
        const bool col = layout == FIP_COL_MAJOR;
        if (ldb < max1(col ? m : n)) return 13;
        if (m > 0 && n > 0 && !(beta == T(1) && !reads_ab) && C == nullptr) return 15;
        if (ldc < max1(col ? m : n)) return 16;
        if (m == 0 || n == 0) return 0;
        if (!reads_ab && beta == T(1)) return 0;
        if (!reads_ab) {
            const KernelShape ks = kernel_shape(layout, m, n);
            if (const hipError_t e = fip::launch_scale(sizeof(T), ks.M, ks.N, C, ldc, (double)beta,
                                                       h->stream); e != hipSuccess)
                return launch_failed(h, e);
            return 0;
        }
        return run_l3<T>(h, dtype, trmm_shape(layout, side, uplo, transA, diag, m, n), alpha, A,
                         lda, B, ldb, beta, C, ldc);
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

// ---- TRSM: recursive blocking onto the fused-pack GEMM --------------------------
//
// op(T) X = alpha B (side L) or X op(T) = alpha B (side R), in place in B.  On
// the column-major view, op(T) is split into [T11 0; T21 T22] (lower) or
// [T11 T12; 0 T22] (upper) at a multiple of the diagonal-block size; the block
// solved first takes alpha, the other part of B becomes alpha B - (its
// coupling block) times the solved X through a GEMM of the fused-pack tile
// kernel (C := -1 * op(X) op(Y) + alpha * C), and the remaining solve runs with
// alpha = 1.  Blocks of at most kTrsmBlock rows go to the diagonal-block
// kernel.  A dry run walks the same recursion to size the workspace the GEMM
// updates need, so nothing is launched unless all of them fit.
struct TrsmCtx {
    fip_handle_t h;
    int dtype;
    bool dry;
    int64_t ws_need;
    fip_plan_t first;   // plan of the top-level update (dry run)
    bool have_first;
};

template <typename T>
int trsm_rec(TrsmCtx& c, bool left, bool op_lower, bool trans, bool unit, int64_t m, int64_t n,
             T alpha, const T* A, int64_t lda, T* B, int64_t ldb)
{
    const int64_t k = left ? m : n;
    if (k <= fip::kTrsmBlock) {
        if (c.dry) return 0;
        fip::TrsmBlockDesc d{};
        d.elem = sizeof(T);
        d.A = A; d.lda = lda;
        // the matrix acting on one right-hand side: op(T) (a column of B), or
        // op(T)^T (a row of B)
        d.s_trans = left ? trans : !trans;
        d.s_lower = left ? op_lower : !op_lower;
        d.unit = unit;
        d.nb = (int)k;
        d.B = B;
        d.s_e = left ? 1 : ldb;
        d.s_v = left ? ldb : 1;
        d.nrhs = left ? n : m;
        d.alpha = (double)alpha;
        d.stream = c.h->stream;
        if (const hipError_t e = fip::launch_trsm_block(d); e != hipSuccess) return launch_failed(c.h, e);
        return 0;
    }
    const int64_t k1 = cdiv(k / 2, fip::kTrsmBlock) * fip::kTrsmBlock, k2 = k - k1;
    const T* A11 = A;
    const T* A22 = A + k1 + k1 * lda;
    // op(T)[k1:, :k1] and op(T)[:k1, k1:] as stored blocks with their op
    const char top = trans ? 'T' : 'N';
    const T* Tlo = trans ? A + k1 * lda : A + k1;
    const T* Tup = trans ? A + k1 : A + k1 * lda;
    auto update = [&](int64_t gm, int64_t gn, int64_t gk, const T* X, int64_t ldx, char tx,
                      const T* Y, int64_t ldy, char ty, T* C, int64_t ldc) -> int {
        if (c.dry) {
            Plan pl;
            make_plan(c.h, c.dtype, FIP_COL_MAJOR, gm, gn, gk, tx, ty, false, &pl);
            c.ws_need = std::max<int64_t>(c.ws_need, pl.pub.workspace_bytes);
            if (!c.have_first) { c.first = pl.pub; c.have_first = true; }
            return 0;
        }
        return gemm_impl<T>(c.h, c.dtype, FIP_COL_MAJOR, gm, gn, gk, T(-1), X, ldx, tx, Y, ldy,
                            ty, alpha, C, ldc);
    };
    int rc;
    if (left) {
        T* B1 = B;
        T* B2 = B + k1;
        if (op_lower) {
            if ((rc = trsm_rec<T>(c, left, op_lower, trans, unit, k1, n, alpha, A11, lda, B1, ldb))) return rc;
            if ((rc = update(k2, n, k1, Tlo, lda, top, B1, ldb, 'N', B2, ldb))) return rc;
            return trsm_rec<T>(c, left, op_lower, trans, unit, k2, n, T(1), A22, lda, B2, ldb);
        }
        if ((rc = trsm_rec<T>(c, left, op_lower, trans, unit, k2, n, alpha, A22, lda, B2, ldb))) return rc;
        if ((rc = update(k1, n, k2, Tup, lda, top, B2, ldb, 'N', B1, ldb))) return rc;
        return trsm_rec<T>(c, left, op_lower, trans, unit, k1, n, T(1), A11, lda, B1, ldb);
    }
    T* B1 = B;
    T* B2 = B + k1 * ldb;
    if (op_lower) {
        if ((rc = trsm_rec<T>(c, left, op_lower, trans, unit, m, k2, alpha, A22, lda, B2, ldb))) return rc;
        if ((rc = update(m, k1, k2, B2, ldb, 'N', Tlo, lda, top, B1, ldb))) return rc;
        return trsm_rec<T>(c, left, op_lower, trans, unit, m, k1, T(1), A11, lda, B1, ldb);
    }
    if ((rc = trsm_rec<T>(c, left, op_lower, trans, unit, m, k1, alpha, A11, lda, B1, ldb))) return rc;
    if ((rc = update(m, k2, k1, B1, ldb, 'N', Tup, lda, top, B2, ldb))) return rc;
    return trsm_rec<T>(c, left, op_lower, trans, unit, m, k2, T(1), A22, lda, B2, ldb);
}

// Column-major view of a TRSM call: row-major storage is the transposed view
// of the same memory, so the side and the stored triangle swap and m, n
// exchange (op's transpose stays).
struct TrsmShape {
    bool left, op_lower, trans, unit;
    int64_t m, n;
};
TrsmShape trsm_shape(int layout, char side, char uplo, char transA, char diag, int64_t m, int64_t n)
{
    const bool row = layout == FIP_ROW_MAJOR;
    TrsmShape t;
    t.left = is_left(side) != row;
    const bool lower = is_lower(uplo) != row;
    t.trans = is_trans(transA);
    t.op_lower = lower != t.trans;
    t.unit = is_unit(diag);
    t.m = row ? n : m;
    t.n = row ? m : n;
    return t;
}

template <typename T>
int trsm_impl(fip_handle_t h, int dtype, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, T alpha, const T* A, int64_t lda, T* B, int64_t ldb)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        // positions: layout 2, side 3, uplo 4, transA 5, diag 6, m 7, n 8, alpha 9, A 10,
        // lda 11, B 12, ldb 13
        if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
        if (!valid_side(side)) return 3;
        if (!valid_uplo(uplo)) return 4;
        if (!valid_trans(transA)) return 5;
        if (!valid_diag(diag)) return 6;
        if (m < 0) return 7;
        if (n < 0) return 8;
        const int64_t ka = is_left(side) ? m : n;
        const bool reads = m > 0 && n > 0 && alpha != T(0);
        if (reads && A == nullptr) return 10;
        if (lda < max1(ka)) return 11;
        if (m > 0 && n > 0 && B == nullptr) return 12;
        const bool col = layout == FIP_COL_MAJOR;
        if (ldb < max1(col ? m : n)) return 13;
        if (m == 0 || n == 0) return 0;
        const TrsmShape t = trsm_shape(layout, side, uplo, transA, diag, m, n);
        if (alpha == T(0)) {   // X = 0; neither A nor B is read
            if (const hipError_t e = fip::launch_scale(sizeof(T), t.m, t.n, B, ldb, 0.0, h->stream);
                e != hipSuccess)
                return launch_failed(h, e);
            return 0;
        }
        TrsmCtx c{h, dtype, true, 0, {}, false};
        trsm_rec<T>(c, t.left, t.op_lower, t.trans, t.unit, t.m, t.n, alpha, A, lda, B, ldb);
        if (c.ws_need > 0 && (h->ws == nullptr || (int64_t)h->ws_bytes < c.ws_need))
            return FIP_ERR_WORKSPACE;
        c.dry = false;
        return trsm_rec<T>(c, t.left, t.op_lower, t.trans, t.unit, t.m, t.n, alpha, A, lda, B,
                           ldb);
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

// Workspace plan of a TRSM: the dry run of the recursion (the largest need of
// its GEMM updates, and the top-level update's plan for the other fields).
int trsm_plan(fip_handle_t h, int dtype, int layout, char side, char uplo, char trans, char diag,
              int64_t m, int64_t n, fip_plan_t* out)
{
    const TrsmShape t = trsm_shape(layout, side, uplo, trans, diag, m, n);
    TrsmCtx c{h, dtype, true, 0, {}, false};
    if (dtype == FIP_F64)
        trsm_rec<double>(c, t.left, t.op_lower, t.trans, t.unit, t.m, t.n, 1.0, nullptr, 1,
                         nullptr, 1);
    else
        trsm_rec<float>(c, t.left, t.op_lower, t.trans, t.unit, t.m, t.n, 1.0f, nullptr, 1,
                        nullptr, 1);
    fip_plan_t p{};
    if (c.have_first) p = c.first;
    p.dtype = dtype;
    p.layout = layout;
    p.m = m;
    p.n = n;
    p.k = 0;
    p.workspace_bytes = c.ws_need;
    *out = p;
    return 0;
}

// ---- batched binary32 GEMM ----------------------------------------------------

constexpr int kVbDefaultSplit = 16;   // untuned: max(m, n) <= 16 -> 16 x 16 tiles
constexpr int kVbMaxTiles = 65535;    // tile indices are 16-bit

uint64_t fnv(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

uint64_t vb_signature(int layout, int64_t count, const int32_t* m, const int32_t* n,
                      const int32_t* k, const char* tA, const char* tB)
{
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &layout, sizeof layout);
    h = fnv(h, &count, sizeof count);
    h = fnv(h, m, count * sizeof(int32_t));
    h = fnv(h, n, count * sizeof(int32_t));
    h = fnv(h, k, count * sizeof(int32_t));
    for (int64_t i = 0; i < count; ++i) {
        const char t[2] = {(char)is_trans(tA[i]), (char)is_trans(tB[i])};
        h = fnv(h, t, 2);
    }
    return h;
}

int64_t vb_tiles(int64_t M, int64_t N, int mt) { return cdiv(M, mt) * cdiv(N, mt); }

// Workspace bytes: a 256-byte header (its first 8 bytes: the skipped-problem
// status word, see FIP_ATTR_VB_STATUS), the problem table, and the
// item list of the smallest tile class for every problem (the most items any
// split yields).
int64_t vb_workspace_bytes(int layout, int64_t count, const int32_t* m, const int32_t* n,
                           int64_t* off_probs, int64_t* off_items)
{
    int64_t items = 0;
    for (int64_t i = 0; i < count; ++i) {
        const KernelShape ks = kernel_shape(layout, m[i], n[i]);
        items += vb_tiles(ks.M, ks.N, 16);
    }
    int64_t off = 256;
    *off_probs = off; off = align256(off + count * (int64_t)sizeof(fip::VbProblem));
    *off_items = off; off = align256(off + items * (int64_t)sizeof(fip::VbItem));
    return off;
}

int vb_check(int layout, int64_t count, const int32_t* m, const int32_t* n, const int32_t* k,
             const char* tA, const char* tB)
{
    if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
    if (count < 0 || count > ((int64_t)1 << 31)) return 3;
    if (count == 0) return 0;
    if (m == nullptr) return 4;
    if (n == nullptr) return 5;
    if (k == nullptr) return 6;
    if (tA == nullptr) return 7;
    if (tB == nullptr) return 8;
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] < 0 || m[i] > 16 * kVbMaxTiles) return 4;
        if (n[i] < 0 || n[i] > 16 * kVbMaxTiles) return 5;
        if (k[i] < 0) return 6;
        if (!valid_trans(tA[i])) return 7;
        if (!valid_trans(tB[i])) return 8;
    }
    return 0;
}

// Build the problem table and the LPT-ordered item list for a split, and copy
// them into the workspace (after the stream has drained: an earlier batch may
// still be reading the previous plan).
int vb_upload(fip_handle_s* h, int layout, int64_t count, const int32_t* m, const int32_t* n,
              const int32_t* k, const char* tA, const char* tB, uint64_t sig, int split)
{
    VbState& v = *h->vb;
    int64_t off_probs, off_items;
    vb_workspace_bytes(layout, count, m, n, &off_probs, &off_items);
    v.probs.assign(count, fip::VbProblem{});
    std::vector<int64_t> order(count);
    std::vector<int64_t> cost(count);
    for (int64_t i = 0; i < count; ++i) {
        const KernelShape ks = kernel_shape(layout, m[i], n[i]);
        fip::VbProblem& p = v.probs[i];
        p.M = (int32_t)ks.M; p.N = (int32_t)ks.N; p.K = k[i];
        const bool a_mn = mn_major(false, layout, tA[i]), b_mn = mn_major(true, layout, tB[i]);
        const bool akm = ks.swapped ? !b_mn : !a_mn, bkm = ks.swapped ? !a_mn : !b_mn;
        p.flags = (akm ? fip::kVbAKmajor : 0) | (bkm ? fip::kVbBKmajor : 0) |
                  (ks.swapped ? fip::kVbSwapped : 0);
        p.cls = std::max(ks.M, ks.N) <= split ? 2 : 1;
        const int mt = p.cls == 1 ? 32 : 16;
        cost[i] = (cdiv(k[i], 16) + 1) * mt * mt;   // one tile's k-blocks plus its epilogue
        order[i] = i;
    }
    // Whole problems to XCDs, longest problem first to the least loaded XCD
    // (a problem's tiles then share one L2), then each XCD's problems longest
    // tile first, a problem's tiles together.
    std::vector<int64_t> total_cost(count);
    for (int64_t i = 0; i < count; ++i) {
        const fip::VbProblem& p = v.probs[i];
        const int mt = p.cls == 1 ? 32 : 16;
        total_cost[i] = cost[i] * cdiv(p.M, mt) * cdiv(p.N, mt);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return total_cost[a] > total_cost[b]; });
    std::vector<std::vector<int64_t>> bins(fip::kCopies);
    int64_t load[fip::kCopies] = {};
    for (int64_t oi = 0; oi < count; ++oi) {
        const int64_t i = order[oi];
        if (total_cost[i] == 0) continue;
        int best = 0;
        for (int x = 1; x < fip::kCopies; ++x)
            if (load[x] < load[best]) best = x;
        load[best] += total_cost[i];
        bins[best].push_back(i);
    }
    v.items.clear();
    for (int x = 0; x < fip::kCopies; ++x) {
        std::vector<int64_t>& b = bins[x];
        std::stable_sort(b.begin(), b.end(), [&](int64_t p, int64_t q) { return cost[p] > cost[q]; });
        v.xcd_off[x] = (int64_t)v.items.size();
        for (int64_t i : b) {
            const fip::VbProblem& p = v.probs[i];
            const int mt = p.cls == 1 ? 32 : 16;
            const int64_t tm_n = cdiv(p.M, mt), tn_n = cdiv(p.N, mt);
            for (int64_t tn = 0; tn < tn_n; ++tn)
                for (int64_t tm = 0; tm < tm_n; ++tm)
                    v.items.push_back(fip::VbItem{(int32_t)i, (uint16_t)tm, (uint16_t)tn});
        }
    }
    v.xcd_off[fip::kCopies] = (int64_t)v.items.size();
    if (hipStreamSynchronize(h->stream) != hipSuccess) return FIP_ERR_LAUNCH;
    char* ws = static_cast<char*>(h->ws);
    const unsigned long long zero = 0;   // the header's skipped-problem status word
    if (hipMemcpy(ws, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
        return FIP_ERR_LAUNCH;
    if (count > 0 &&
        hipMemcpy(ws + off_probs, v.probs.data(), count * sizeof(fip::VbProblem),
                  hipMemcpyHostToDevice) != hipSuccess)
        return FIP_ERR_LAUNCH;
    if (!v.items.empty() &&
        hipMemcpy(ws + off_items, v.items.data(), v.items.size() * sizeof(fip::VbItem),
                  hipMemcpyHostToDevice) != hipSuccess)
        return FIP_ERR_LAUNCH;
    v.sig = sig;
    v.split = split;
    v.ws = h->ws;
    v.total = (int64_t)v.items.size();
    v.off_probs = off_probs;
    v.off_items = off_items;
    if (v.exec) { (void)hipGraphExecDestroy(v.exec); v.exec = nullptr; }
    return 0;
}

fip::VbLaunchDesc vb_desc(const fip_handle_s* h, float alpha, const float* const* A,
                          const int64_t* lda, const float* const* B, const int64_t* ldb,
                          float beta, float* const* C, const int64_t* ldc)
{
    const VbState& v = *h->vb;
    char* ws = static_cast<char*>(h->ws);
    fip::VbLaunchDesc d{};
    d.status = reinterpret_cast<unsigned long long*>(ws);
    d.probs = reinterpret_cast<const fip::VbProblem*>(ws + v.off_probs);
    d.items = reinterpret_cast<const fip::VbItem*>(ws + v.off_items);
    d.total = v.total;
    for (int x = 0; x <= fip::kCopies; ++x) d.xcd_off[x] = v.xcd_off[x];
    d.A = A; d.lda = lda; d.B = B; d.ldb = ldb; d.C = C; d.ldc = ldc;
    d.alpha = alpha; d.beta = beta;
    d.stream = h->stream;
    return d;
}

// Validate, make sure the plan for (signature, split) is in the workspace.
int vb_prepare(fip_handle_s* h, int layout, int64_t count, const int32_t* m, const int32_t* n,
               const int32_t* k, const char* tA, const char* tB, int forced_split,
               uint64_t* sig_out)
{
    if (h->vb == nullptr) {
        h->vb = new (std::nothrow) VbState;
        if (h->vb == nullptr) return FIP_ERR_ALLOC;
    }
    const uint64_t sig = vb_signature(layout, count, m, n, k, tA, tB);
    *sig_out = sig;
    int split = forced_split;
    if (split < 0) split = h->vb_split;
    if (split < 0) {
        auto it = h->vb->tuned.find(sig);
        split = it != h->vb->tuned.end() ? it->second : kVbDefaultSplit;
    }
    int64_t op, oi;
    const int64_t need = vb_workspace_bytes(layout, count, m, n, &op, &oi);
    if (h->ws == nullptr || (int64_t)h->ws_bytes < need) return FIP_ERR_WORKSPACE;
    VbState& v = *h->vb;
    if (v.sig != sig || v.split != split || v.ws != h->ws || v.total == 0)
        return vb_upload(h, layout, count, m, n, k, tA, tB, sig, split);
    return 0;
}

}  // namespace

extern "C" {

int fip_create(fip_handle_t* handle)
{
    if (handle == nullptr) return 1;
    fip_handle_s* h = new (std::nothrow) fip_handle_s;
    if (h == nullptr) return FIP_ERR_ALLOC;
    memset(h, 0, sizeof(*h));
    h->magic = kMagic;
    h->stream = nullptr;
    h->policy = FIP_PACK_AUTO;
    h->tile_override = -1;
    h->order = -1;
    h->vb_split = -1;
    h->mx_tile = -1;
    h->split_k = -1;
    h->copies = -1;
    h->dma = kDefaultDma;
    h->vb = nullptr;
    h->tuned = nullptr;
    *handle = h;
    return 0;
}

int fip_destroy(fip_handle_t handle)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    handle->magic = 0;
    delete handle->vb;
    delete handle->tuned;
    delete handle;
    return 0;
}

int fip_set_stream(fip_handle_t handle, void* hip_stream)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    handle->stream = static_cast<hipStream_t>(hip_stream);
    return 0;
}

int fip_set_attr(fip_handle_t handle, int attr, int64_t value)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    switch (attr) {
    case FIP_ATTR_PACK_POLICY:
        if (value < FIP_PACK_AUTO || value > FIP_PACK_CONSUME_ONLY) return 3;
        handle->policy = (int)value;
        return 0;
    case FIP_ATTR_TILE:
        if (value < -1 || value >= fip::kNumTileClasses) return 3;
        handle->tile_override = (int)value;
        return 0;
    case FIP_ATTR_NO_PUBLISH:
        if (value != 0 && value != 1) return 3;
        handle->no_publish = (int)value;
        return 0;
    case FIP_ATTR_STATS:
        if (value != 0 && value != 1) return 3;
        handle->stats = (int)value;
        return 0;
    case FIP_ATTR_ORDER:
        if (value != -1 && value != 0 && value != 1) return 3;
        handle->order = (int)value;
        return 0;
    case FIP_ATTR_VB_SPLIT:
        if (value < -1 || value > (int64_t)1 << 30) return 3;
        handle->vb_split = (int)value;
        return 0;
    case FIP_ATTR_MX_TILE:
        if (value != -1 && value != 128 && value != 256) return 3;
        handle->mx_tile = (int)value;
        return 0;
    case FIP_ATTR_SPLIT_K:
        if (value != -1 && (value < 1 || value > kMaxSplit)) return 3;
        handle->split_k = (int)value;
        return 0;
    case FIP_ATTR_COPIES:
        if (value != -1 && value != 1 && value != fip::kCopies) return 3;
        handle->copies = (int)value;
        return 0;
    case FIP_ATTR_DMA:
        if (value != 0 && value != 1 && value != -1) return 3;
        handle->dma = (int)value;
        return 0;
    default:
        return 2;
    }
}

int fip_get_attr(fip_handle_t handle, int attr, int64_t* value)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (value == nullptr) return 3;
    switch (attr) {
    case FIP_ATTR_PACK_POLICY: *value = handle->policy; return 0;
    case FIP_ATTR_TILE: *value = handle->tile_override; return 0;
    case FIP_ATTR_NO_PUBLISH: *value = handle->no_publish; return 0;
    case FIP_ATTR_STATS: *value = handle->stats; return 0;
    case FIP_ATTR_ORDER: *value = handle->order; return 0;
    case FIP_ATTR_EPOCH: *value = (int64_t)handle->epoch; return 0;
    case FIP_ATTR_LAST_HIP_ERROR: *value = handle->last_hip_error; return 0;
    case FIP_ATTR_VB_SPLIT: *value = handle->vb_split; return 0;
    case FIP_ATTR_VB_GRID: *value = fip::vbatched_grid(); return 0;
    case FIP_ATTR_MX_TILE: *value = handle->mx_tile; return 0;
    case FIP_ATTR_SPLIT_K: *value = handle->split_k; return 0;
    case FIP_ATTR_COPIES: *value = handle->copies; return 0;
    case FIP_ATTR_DMA: *value = handle->dma; return 0;
    case FIP_ATTR_LAST_DMA: *value = handle->last_dma; return 0;
    case FIP_ATTR_VB_STATUS: {
        *value = 0;
        VbState* v = handle->vb;
        if (v == nullptr || v->ws == nullptr || v->ws != handle->ws) return 0;
        unsigned long long st = 0;
        const unsigned long long zero = 0;
        if (hipStreamSynchronize(handle->stream) != hipSuccess ||
            hipMemcpy(&st, v->ws, sizeof st, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(v->ws, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
            return FIP_ERR_LAUNCH;
        *value = (int64_t)st;
        return 0;
    }
    default: return 2;
    }
}

int fip_set_workspace(fip_handle_t handle, void* dptr, size_t bytes)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (dptr == nullptr && bytes != 0) return 2;
    if (dptr != nullptr && ((uintptr_t)dptr & 255) != 0) return 2;  // 256-byte aligned
    handle->ws = dptr;
    handle->ws_bytes = dptr ? bytes : 0;

    return 0;
}

int fip_plan(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
             char transA, char transB, fip_plan_t* plan)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (!valid_dtype(dtype)) return 2;
    if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 3;
    if (m < 0) return 4;
    if (n < 0) return 5;
    if (k < 0) return 6;
    if (!valid_trans(transA)) return 7;
    if (!valid_trans(transB)) return 8;
    if (plan == nullptr) return 9;
    Plan pl;
    make_plan(handle, dtype, layout, m, n, k, transA, transB, false, &pl);
    *plan = pl.pub;
    return 0;
}

int fip_last_plan(fip_handle_t handle, fip_plan_t* plan)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (plan == nullptr) return 2;
    if (!handle->has_last) return FIP_ERR_UNSUPPORTED;
    *plan = handle->last;
    return 0;
}

int fip_dgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, char transA, const double* B, int64_t ldb,
              char transB, double beta, double* C, int64_t ldc)
{
    return gemm_impl<double>(handle, FIP_F64, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                             transB, beta, C, ldc);
}

int fip_dgemm_noalloc(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, char transA, const double* B,
                      int64_t ldb, char transB, double beta, double* C, int64_t ldc)
{
    return gemm_impl<double>(handle, FIP_F64, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                             transB, beta, C, ldc, true);
}

int fip_sgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, float alpha,
              const float* A, int64_t lda, char transA, const float* B, int64_t ldb, char transB,
              float beta, float* C, int64_t ldc)
{
    return gemm_impl<float>(handle, FIP_F32, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                            transB, beta, C, ldc);
}

int fip_zgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
              const double* alpha, const double* A, int64_t lda, char transA, const double* B,
              int64_t ldb, char transB, const double* beta, double* C, int64_t ldc)
{
    return zgemm_impl<double>(handle, FIP_C128, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                              transB, beta, C, ldc);
}

int fip_cgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
              const float* alpha, const float* A, int64_t lda, char transA, const float* B,
              int64_t ldb, char transB, const float* beta, float* C, int64_t ldc)
{
    return zgemm_impl<float>(handle, FIP_C64, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                             transB, beta, C, ldc);
}

int fip_dsyrk(fip_handle_t handle, int layout, char uplo, char trans, int64_t n, int64_t k,
              double alpha, const double* A, int64_t lda, double beta, double* C, int64_t ldc)
{
    return syrk_impl<double>(handle, FIP_F64, layout, uplo, trans, n, k, alpha, A, lda, beta, C,
                             ldc);
}

int fip_ssyrk(fip_handle_t handle, int layout, char uplo, char trans, int64_t n, int64_t k,
              float alpha, const float* A, int64_t lda, float beta, float* C, int64_t ldc)
{
    return syrk_impl<float>(handle, FIP_F32, layout, uplo, trans, n, k, alpha, A, lda, beta, C,
                            ldc);
}

int fip_dtrmm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, double alpha, const double* A, int64_t lda, const double* B,
              int64_t ldb, double beta, double* C, int64_t ldc)
{
    return trmm_impl<double>(handle, FIP_F64, layout, side, uplo, transA, diag, m, n, alpha, A,
                             lda, B, ldb, beta, C, ldc);
}

int fip_strmm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, float alpha, const float* A, int64_t lda, const float* B,
              int64_t ldb, float beta, float* C, int64_t ldc)
{
    return trmm_impl<float>(handle, FIP_F32, layout, side, uplo, transA, diag, m, n, alpha, A,
                            lda, B, ldb, beta, C, ldc);
}

int fip_dtrsm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, double alpha, const double* A, int64_t lda, double* B,
              int64_t ldb)
{
    return trsm_impl<double>(handle, FIP_F64, layout, side, uplo, transA, diag, m, n, alpha, A,
                             lda, B, ldb);
}

int fip_strsm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, float alpha, const float* A, int64_t lda, float* B,
              int64_t ldb)
{
    return trsm_impl<float>(handle, FIP_F32, layout, side, uplo, transA, diag, m, n, alpha, A,
                            lda, B, ldb);
}

int fip_plan_l3(fip_handle_t handle, int op, int dtype, int layout, char side, char uplo,
                char trans, char diag, int64_t m, int64_t n, int64_t k, fip_plan_t* plan)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (op != FIP_OP_SYRK && op != FIP_OP_TRMM && op != FIP_OP_TRSM) return 2;
    if (dtype != FIP_F64 && dtype != FIP_F32) return 3;
    if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 4;
    if (op != FIP_OP_SYRK && !valid_side(side)) return 5;
    if (!valid_uplo(uplo)) return 6;
    if (!valid_trans(trans)) return 7;
    if (op != FIP_OP_SYRK && !valid_diag(diag)) return 8;
    if (m < 0) return 9;
    if (n < 0) return 10;
    if (k < 0) return 11;
    if (plan == nullptr) return 12;
    if (op == FIP_OP_TRSM) return trsm_plan(handle, dtype, layout, side, uplo, trans, diag, m, n, plan);
    Plan pl;
    const L3Shape ls = op == FIP_OP_SYRK ? syrk_shape(layout, uplo, trans, n, k)
                                         : trmm_shape(layout, side, uplo, trans, diag, m, n);
    make_plan_l3(handle, dtype, ls, &pl);
    pl.pub.layout = layout;
    pl.pub.m = op == FIP_OP_SYRK ? n : m;
    pl.pub.n = n;
    *plan = pl.pub;
    return 0;
}

int fip_pack(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
             const void* A, int64_t lda, char transA, const void* B, int64_t ldb, char transB)
{
    try {
        if (!valid_handle(handle)) return FIP_ERR_HANDLE;
        if (!valid_dtype(dtype)) return 2;
        // positions: layout 3, m 4, n 5, k 6, A 7, lda 8, transA 9, B 10, ldb 11, transB 12
        const int bad = check_args(3, layout, m, n, k, true, A, lda, transA, B, ldb, transB, false,
                                   false, nullptr, 1);
        if (bad) {
            // check_args numbers alpha as an argument; fip_pack has none, so
            // positions after k shift down by one.
            return bad > 6 ? bad - 1 : bad;
        }
        Plan pl;
        make_plan(handle, dtype, layout, m, n, k, transA, transB, true, &pl);
        if (pl.pub.workspace_bytes == 0) { handle->last = pl.pub; handle->has_last = 1; return 0; }
        const int ws = prepare_workspace(handle, pl);
        if (ws) return ws;
        if (mx_form_of(dtype) >= 0) {
            fip::MxLaunchDesc d;
            fill_mx_desc(handle, pl, mx_form_of(dtype), layout, k, A, lda, transA, B, ldb, transB,
                         &d);
            if (const hipError_t e = fip::launch_pack_mx(d); e != hipSuccess) return launch_failed(handle, e);
            handle->last = pl.pub;
            handle->has_last = 1;
            return 0;
        }
        fip::LaunchDesc d;
        memset(&d, 0, sizeof(d));
        d.elem = pl.elem;
        d.tile_class = pl.pub.tile_class;
        d.mode = pl.mode;
        d.M = pl.ks.M; d.N = pl.ks.N; d.K = k;
        fill_operands(pl, layout, A, lda, transA, B, ldb, transB, &d);
        if (is_complex(dtype)) {   // the 1m expansions (see zgemm_impl)
            d.kind = fip::k1m;
            d.K = 2 * k;
            const bool ca = transA == 'C' || transA == 'c', cb = transB == 'C' || transB == 'c';
            d.conj_a = pl.ks.swapped ? cb : ca;
            d.conj_b = pl.ks.swapped ? ca : cb;
        }
        fill_workspace(handle->ws, pl, &d);
        d.stream = handle->stream;
        if (const hipError_t e = fip::launch_pack(d); e != hipSuccess) return launch_failed(handle, e);
        handle->last = pl.pub;
        handle->has_last = 1;
        return 0;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

int fip_gemm_mx(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
                float alpha, const void* A, int64_t lda, char transA, const void* B, int64_t ldb,
                char transB, float beta, void* C, int64_t ldc, int c_type, const float* a_scale,
                const float* b_scale)
{
    return gemm_mx_impl(handle, dtype, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB,
                        beta, C, ldc, c_type, a_scale, b_scale);
}

int fip_quantize_fp8(fip_handle_t handle, int layout, int64_t rows, int64_t cols, const float* X,
                     int64_t ldx, int axis, uint8_t* Q, int64_t ldq, float* scales)
{
    try {
        if (!valid_handle(handle)) return FIP_ERR_HANDLE;
        if (layout != FIP_COL_MAJOR && layout != FIP_ROW_MAJOR) return 2;
        if (rows < 0) return 3;
        if (cols < 0) return 4;
        const bool col = layout == FIP_COL_MAJOR;
        const bool any = rows > 0 && cols > 0;
        if (any && X == nullptr) return 5;
        if (ldx < max1(col ? rows : cols)) return 6;
        if (axis != 0 && axis != 1) return 7;
        if (any && Q == nullptr) return 8;
        if (ldq < max1(col ? rows : cols)) return 9;
        if (any && scales == nullptr) return 10;
        if (!any) return 0;
        return fip::launch_quantize_fp8(col, rows, cols, X, ldx, axis, Q, ldq, scales,
                                        handle->stream) == hipSuccess ? 0 : FIP_ERR_LAUNCH;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

int fip_vbatched_workspace(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                           const int32_t* n, const int32_t* k, const char* transA,
                           const char* transB, size_t* bytes)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    const int bad = vb_check(layout, count, m, n, k, transA, transB);
    if (bad) return bad;
    if (bytes == nullptr) return 9;
    int64_t op, oi;
    *bytes = (size_t)vb_workspace_bytes(layout, count, m, n, &op, &oi);
    return 0;
}

int fip_sgemm_vbatched(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                       const int32_t* n, const int32_t* k, const char* transA, const char* transB,
                       float alpha, const float* const* A, const int64_t* lda,
                       const float* const* B, const int64_t* ldb, float beta, float* const* C,
                       const int64_t* ldc, int flags)
{
    try {
        if (!valid_handle(handle)) return FIP_ERR_HANDLE;
        const int bad = vb_check(layout, count, m, n, k, transA, transB);
        if (bad) return bad;
        if (count > 0) {
            if (A == nullptr) return 10;
            if (lda == nullptr) return 11;
            if (B == nullptr) return 12;
            if (ldb == nullptr) return 13;
            if (C == nullptr) return 15;
            if (ldc == nullptr) return 16;
        }
        if (flags & ~FIP_VB_GRAPH) return 17;
        if (count == 0 || (alpha == 0.f && beta == 1.f)) return 0;
        uint64_t sig;
        const int rc = vb_prepare(handle, layout, count, m, n, k, transA, transB, -1, &sig);
        if (rc) return rc;
        VbState& v = *handle->vb;
        if (v.total == 0) return 0;
        const fip::VbLaunchDesc d = vb_desc(handle, alpha, A, lda, B, ldb, beta, C, ldc);
        if (!(flags & FIP_VB_GRAPH))
            return fip::launch_vbatched(d) == hipSuccess ? 0 : FIP_ERR_LAUNCH;
        // graph replay: one kernel node, rebuilt only when the call changes
        uint64_t key[12];
        float ab[2] = {alpha, beta};
        uint64_t abits;
        memcpy(&abits, ab, 8);
        const void* ptrs[] = {A, lda, B, ldb, C, ldc, handle->ws, handle->stream};
        key[0] = v.sig; key[1] = (uint64_t)v.split; key[2] = abits;
        for (int i = 0; i < 8; ++i) key[3 + i] = (uint64_t)(uintptr_t)ptrs[i];
        key[11] = (uint64_t)v.total;
        if (v.exec == nullptr || memcmp(key, v.gkey, sizeof key) != 0) {
            if (v.exec) { (void)hipGraphExecDestroy(v.exec); v.exec = nullptr; }
            if (fip::build_vbatched_graph(d, &v.exec) != hipSuccess) { v.exec = nullptr; return FIP_ERR_LAUNCH; }
            memcpy(v.gkey, key, sizeof key);
        }
        return hipGraphLaunch(v.exec, handle->stream) == hipSuccess ? 0 : FIP_ERR_LAUNCH;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

int fip_vbatched_tune(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                      const int32_t* n, const int32_t* k, const char* transA, const char* transB,
                      float alpha, const float* const* A, const int64_t* lda,
                      const float* const* B, const int64_t* ldb, float beta, float* const* C,
                      const int64_t* ldc, int* split_out)
{
    try {
        if (!valid_handle(handle)) return FIP_ERR_HANDLE;
        const int bad = vb_check(layout, count, m, n, k, transA, transB);
        if (bad) return bad;
        if (count > 0 && (A == nullptr || lda == nullptr || B == nullptr || ldb == nullptr ||
                          C == nullptr || ldc == nullptr))
            return A == nullptr ? 10 : lda == nullptr ? 11 : B == nullptr ? 12
                 : ldb == nullptr ? 13 : C == nullptr ? 15 : 16;
        if (split_out == nullptr) return 17;
        *split_out = kVbDefaultSplit;
        if (count == 0) return 0;
        // candidate thresholds on max(m, n) for 32 x 32 tiles
        const int cands[] = {0, 8, 16, 24, 32, 48, 64, 1 << 30};
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return FIP_ERR_LAUNCH;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FIP_ERR_LAUNCH; }
        float best_t = 1e30f;
        int best = kVbDefaultSplit;
        uint64_t sig = 0;
        int rc = 0;
        for (int c : cands) {
            rc = vb_prepare(handle, layout, count, m, n, k, transA, transB, c, &sig);
            if (rc) break;
            const fip::VbLaunchDesc d = vb_desc(handle, alpha, A, lda, B, ldb, beta, C, ldc);
            if (d.total == 0) { best = c; break; }
            float t[3];
            bool ok = fip::launch_vbatched(d) == hipSuccess;  // warm-up
            for (int r = 0; r < 3 && ok; ++r) {
                ok = hipEventRecord(e0, handle->stream) == hipSuccess &&
                     fip::launch_vbatched(d) == hipSuccess &&
                     hipEventRecord(e1, handle->stream) == hipSuccess &&
                     hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
            }
            if (!ok) { rc = FIP_ERR_LAUNCH; break; }
            std::sort(t, t + 3);
            if (t[1] < best_t) { best_t = t[1]; best = c; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        handle->vb->tuned[sig] = best;
        *split_out = best;
        return vb_prepare(handle, layout, count, m, n, k, transA, transB, -1, &sig);
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

extern "C++" {
namespace {

// Time one configuration of a GEMM call: a warm-up, then the median of three
// launches (HIP events on the handle's stream), in milliseconds.
template <typename T>
int time_gemm(fip_handle_t h, int dtype, int layout, int64_t m, int64_t n, int64_t k, T alpha,
              const T* A, int64_t lda, char tA, const T* B, int64_t ldb, char tB, T beta, T* C,
              int64_t ldc, hipEvent_t e0, hipEvent_t e1, float* ms)
{
    float t[3];
    int rc = gemm_impl<T>(h, dtype, layout, m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc);
    for (int r = 0; r < 3 && rc == 0; ++r) {
        if (hipEventRecord(e0, h->stream) != hipSuccess) return FIP_ERR_LAUNCH;
        rc = gemm_impl<T>(h, dtype, layout, m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc);
        if (rc) break;
        if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            return FIP_ERR_LAUNCH;
    }
    if (rc) return rc;
    std::sort(t, t + 3);
    *ms = t[1];
    return 0;
}

template <typename T>
int gemm_tune_impl(fip_handle_t h, int dtype, int layout, int64_t m, int64_t n, int64_t k,
                   T alpha, const T* A, int64_t lda, char tA, const T* B, int64_t ldb, char tB,
                   T beta, T* C, int64_t ldc, int* tile_out, int* split_out)
{
    try {
        if (!valid_handle(h)) return FIP_ERR_HANDLE;
        const int bad = check_args(2, layout, m, n, k, alpha != T(0), A, lda, tA, B, ldb, tB, true,
                                   beta == T(1), C, ldc);
        if (bad) return bad;
        if (tile_out == nullptr) return 16;
        if (split_out == nullptr) return 17;
        // the planner's choice, reported when there is nothing to time
        Plan pl0;
        make_plan(h, dtype, layout, m, n, k, tA, tB, false, &pl0);
        *tile_out = pl0.pub.tile_class;
        *split_out = -1;
        if (m == 0 || n == 0 || k == 0 || alpha == T(0)) return 0;
        const int keep_tile = h->tile_override, keep_split = h->split_k;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return FIP_ERR_LAUNCH;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FIP_ERR_LAUNCH; }
        // candidates: every tile class, with the planner's k split and with none
        // (configurations that plan the same tile class and split are timed once)
        std::vector<std::pair<int, int>> seen;
        float best_t = 1e30f;
        GemmChoice best{pl0.pub.tile_class, -1};
        int rc = 0;
        for (int cls = 0; cls < fip::kNumTileClasses && rc == 0; ++cls) {
            for (int sp : {-1, 1}) {
                h->tile_override = cls;
                h->split_k = sp;
                Plan pl;
                make_plan(h, dtype, layout, m, n, k, tA, tB, false, &pl);
                if (std::find(seen.begin(), seen.end(), std::make_pair(cls, pl.split)) != seen.end())
                    continue;
                seen.emplace_back(cls, pl.split);
                float ms = 0.f;
                rc = time_gemm<T>(h, dtype, layout, m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C,
                                  ldc, e0, e1, &ms);
                if (rc) break;
                if (ms < best_t) {
                    best_t = ms;
                    best = GemmChoice{cls, sp};
                }
            }
        }
        h->tile_override = keep_tile;
        h->split_k = keep_split;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        if (h->tuned == nullptr) {
            h->tuned = new (std::nothrow) std::map<GemmKey, GemmChoice>;
            if (h->tuned == nullptr) return FIP_ERR_ALLOC;
        }
        (*h->tuned)[gemm_key(dtype, layout, m, n, k, tA, tB)] = best;
        *tile_out = best.tile;
        *split_out = best.split;
        return 0;
    } catch (...) {
        return FIP_ERR_LAUNCH;
    }
}

constexpr const char* kTuneHeader = "fipgemm-tune 1";

}  // namespace
}  // extern "C++"

int fip_dgemm_tune(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, double alpha,
                   const double* A, int64_t lda, char transA, const double* B, int64_t ldb,
                   char transB, double beta, double* C, int64_t ldc, int* tile_out,
                   int* split_out)
{
    return gemm_tune_impl<double>(handle, FIP_F64, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                                  transB, beta, C, ldc, tile_out, split_out);
}

int fip_sgemm_tune(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, float alpha,
                   const float* A, int64_t lda, char transA, const float* B, int64_t ldb,
                   char transB, float beta, float* C, int64_t ldc, int* tile_out, int* split_out)
{
    return gemm_tune_impl<float>(handle, FIP_F32, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                                 transB, beta, C, ldc, tile_out, split_out);
}

int fip_tune_save(fip_handle_t handle, const char* path)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (path == nullptr) return 1;
    FILE* f = fopen(path, "w");
    if (f == nullptr) return 1;
    bool ok = fprintf(f, "%s\n", kTuneHeader) > 0;
    if (handle->tuned != nullptr)
        for (const auto& e : *handle->tuned)
            ok = ok && fprintf(f, "gemm %lld %lld %lld %lld %lld %lld %lld %d %d\n",
                               (long long)e.first[0], (long long)e.first[1], (long long)e.first[2],
                               (long long)e.first[3], (long long)e.first[4], (long long)e.first[5],
                               (long long)e.first[6], e.second.tile, e.second.split) > 0;
    if (handle->vb != nullptr)
        for (const auto& e : handle->vb->tuned)
            ok = ok && fprintf(f, "vb %llu %d\n", (unsigned long long)e.first, e.second) > 0;
    ok = (fclose(f) == 0) && ok;
    return ok ? 0 : 1;
}

int fip_tune_load(fip_handle_t handle, const char* path)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (path == nullptr) return 1;
    FILE* f = fopen(path, "r");
    if (f == nullptr) return 1;
    // parse the whole file first: a malformed file changes nothing
    std::vector<std::pair<GemmKey, GemmChoice>> g;
    std::vector<std::pair<uint64_t, int>> v;
    char line[512];
    bool ok = fgets(line, sizeof line, f) != nullptr && strncmp(line, kTuneHeader, strlen(kTuneHeader)) == 0;
    while (ok && fgets(line, sizeof line, f) != nullptr) {
        long long a[7];
        int tile, split;
        unsigned long long sig;
        char tail;
        if (sscanf(line, "gemm %lld %lld %lld %lld %lld %lld %lld %d %d %c", &a[0], &a[1], &a[2],
                   &a[3], &a[4], &a[5], &a[6], &tile, &split, &tail) == 9) {
            ok = valid_dtype((int)a[0]) && mx_form_of((int)a[0]) < 0 &&
                 (a[1] == FIP_COL_MAJOR || a[1] == FIP_ROW_MAJOR) && a[2] >= 0 && a[3] >= 0 &&
                 a[4] >= 0 && (a[5] == 0 || a[5] == 1) && (a[6] == 0 || a[6] == 1) && tile >= 0 &&
                 tile < fip::kNumTileClasses && (split == -1 || (split >= 1 && split <= kMaxSplit));
            g.emplace_back(GemmKey{a[0], a[1], a[2], a[3], a[4], a[5], a[6]}, GemmChoice{tile, split});
        } else if (sscanf(line, "vb %llu %d %c", &sig, &split, &tail) == 2) {
            ok = split >= 0;
            v.emplace_back((uint64_t)sig, split);
        } else {
            ok = line[0] == '\n' || line[0] == '#';
        }
    }
    fclose(f);
    if (!ok) return 2;
    try {
        if (!g.empty() && handle->tuned == nullptr) {
            handle->tuned = new (std::nothrow) std::map<GemmKey, GemmChoice>;
            if (handle->tuned == nullptr) return FIP_ERR_ALLOC;
        }
        if (!v.empty() && handle->vb == nullptr) {
            handle->vb = new (std::nothrow) VbState;
            if (handle->vb == nullptr) return FIP_ERR_ALLOC;
        }
        for (const auto& e : g) (*handle->tuned)[e.first] = e.second;
        for (const auto& e : v) handle->vb->tuned[e.first] = e.second;
    } catch (...) {
        return FIP_ERR_ALLOC;
    }
    return 0;
}

int fip_tile_map(int64_t tiles_m, int64_t tiles_n, int order, int32_t* tm, int32_t* tn)
{
    if (tiles_m < 0 || tiles_m * tiles_n > ((int64_t)1 << 30)) return 1;
    if (tiles_n < 0) return 2;
    if (order != 0 && order != 1) return 3;
    const int64_t T = tiles_m * tiles_n;
    if (T > 0 && tm == nullptr) return 4;
    if (T > 0 && tn == nullptr) return 5;
    for (int64_t w = 0; w < T; ++w) {
        int a, b;
        fip::tile_coords((int)w, (int)tiles_m, (int)tiles_n, fip::kGroupM, order, a, b);
        tm[w] = a;
        tn[w] = b;
    }
    return 0;
}

int fip_xcc_map(fip_handle_t handle, uint32_t* d_out, int64_t nblocks)
{
    if (!valid_handle(handle)) return FIP_ERR_HANDLE;
    if (d_out == nullptr) return 2;
    if (nblocks < 0 || nblocks > (int64_t)1 << 30) return 3;
    if (nblocks == 0) return 0;
    return fip::launch_xcc_map(d_out, nblocks, handle->stream) == hipSuccess ? 0 : FIP_ERR_LAUNCH;
}

}  // extern "C"
