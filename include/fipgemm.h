/*
 * fipgemm -- GEMM with packing fused into the first computational pass, for
 * AMD Instinct MI355X (gfx950).
 *
 * Operation (paper Sec. 2.1: the prototypical product C := A B + C, extended
 * with the BLAS gemm statement's alpha, beta and op()):
 *
 *     C := alpha * op(A) * op(B) + beta * C,     op(A) m x k, op(B) k x n, C m x n
 *
 * Method (paper Sec. 3.1-3.3): operand panels are packed into a contiguous,
 * zero-padded tile layout *during* the first pass that computes with them; a
 * panel's later passes read only the packed copy.  Which operand is packed
 * follows the paper's reuse table (Sec. 3.3): A's row panel is packed only
 * when more than one tile column of C reuses it, B's column panel only when
 * more than one tile row does.  Four variants of the tile body exist (A and B
 * each read packed or unpacked, Sec. 3.2); the choice is made per tile and per
 * k-step at run time.
 *
 * Conventions shared by every entry point:
 *   - All matrix pointers are DEVICE pointers owned by the caller.  alpha and
 *     beta are host values passed by value.
 *   - layout is FIP_COL_MAJOR or FIP_ROW_MAJOR.  Stored element (r, c) of a
 *     matrix with leading dimension ld sits at X[r + c*ld] (column-major) or
 *     X[r*ld + c] (row-major).
 *   - trans is one of 'N','n','T','t','C','c'; 'C' equals 'T' for real data.
 *   - Calls enqueue work on the handle's stream and return before it
 *     finishes.  A handle is not thread-safe; use one handle per stream.
 *   - Nothing is allocated on the GEMM path: scratch memory (pack buffers,
 *     flags) is the caller's workspace, see fip_set_workspace.
 *
 * Return codes:
 *    0   success
 *   >0   the 1-based position, in the entry point's own signature (handle
 *        = 1), of the first invalid argument (LAPACK "info" style).  Checked
 *        before any HIP call.
 *   <0   FIP_ERR_* below.
 * No entry point prints, throws or aborts.
 */
#ifndef FIPGEMM_H
#define FIPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fip_handle_s* fip_handle_t;

enum { FIP_COL_MAJOR = 0, FIP_ROW_MAJOR = 1 };
/* Element types / compute forms ("dtype" arguments).  FIP_F64 and FIP_F32 are
   the plain GEMMs; the others are the mixed-precision forms of fip_gemm_mx
   (binary32 accumulation); FIP_F32 and FIP_BF16 also name the C storage type
   of fip_gemm_mx. */
enum {
    FIP_F64 = 0,          /* binary64 operands and C */
    FIP_F32 = 1,          /* binary32 operands and C */
    FIP_BF16 = 2,         /* bfloat16 operands */
    FIP_E4M3 = 3,         /* OCP FP8 E4M3 operands (codes), optional power-of-two scales */
    FIP_BF16X3 = 4,       /* binary32 operands split into 3 bfloat16 terms, 6 products */
    FIP_BF16X3_FAST = 5,  /* binary32 operands split into 2 bfloat16 terms, 3 products */
    FIP_C128 = 6,         /* complex binary64 (re, im pairs): fip_zgemm, the 1m method */
    FIP_C64 = 7,          /* complex binary32 (re, im pairs): fip_cgemm, the 1m method */
};

/* Error codes (negative). */
#define FIP_ERR_HANDLE (-1)      /* null or destroyed handle */
#define FIP_ERR_WORKSPACE (-2)   /* packing needed but workspace unset or too small */
#define FIP_ERR_LAUNCH (-3)      /* a HIP call failed (launch, memset) */
#define FIP_ERR_UNSUPPORTED (-4) /* unsupported dtype / attribute / value */
#define FIP_ERR_ALLOC (-5)       /* host allocation of the handle failed */

/* Attributes (fip_set_attr / fip_get_attr). */
enum {
    /* Which operands are packed.  Value: one of FIP_PACK_*.  Default AUTO. */
    FIP_ATTR_PACK_POLICY = 1,
    /* Force a tile class: -1 = planner's choice (default); 0, 1, 2 = the
       128x128, 64x64, 32x32 C tile classes. */
    FIP_ATTR_TILE = 2,
    /* 1: producers pack but never publish, so every consumer takes the
       unpacked fallback (a test knob; the result must not change). */
    FIP_ATTR_NO_PUBLISH = 3,
    /* 1: count per-chunk events (packed, read packed, read unpacked, polls)
       into the workspace's statistics block (a diagnostic; costs atomics). */
    FIP_ATTR_STATS = 4,
    /* Tile order inside an XCD's run: 0 = GROUP_M tiles of a column
       consecutive, 1 = consecutive tiles in distinct columns; -1 (default):
       1 for the split forms (FIP_BF16X3, FIP_BF16X3_FAST), else 0. */
    FIP_ATTR_ORDER = 7,
    /* Batched calls: problems with max(m, n) <= value use 16 x 16 C tiles,
       the others 32 x 32.  -1 (default): the value fip_vbatched_tune chose for
       the batch's shapes, else 16. */
    FIP_ATTR_VB_SPLIT = 8,
    /* Read only: workgroups (one wave each) a batched launch keeps resident
       on the device; the batch's tiles are dealt round-robin over them. */
    FIP_ATTR_VB_GRID = 9,
    /* Mixed-precision calls: C tile extent.  128: 128 x 128; 256: 256 x 256
       (128 x 128 per wave), bfloat16 and E4M3 only (the split forms always
       use 128); -1 (default): 256 for bfloat16 when the call has at least
       256 tiles of 256 x 256, else 128 (E4M3 runs faster on 128 tiles, two
       per CU, so it takes 256 only when asked). */
    FIP_ATTR_MX_TILE = 10,
    /* Split k into slices computed by separate workgroups; each slice
       writes its partial product to the workspace and a second kernel sums
       the slices in slice order and applies alpha and beta.  FP64/FP32 calls
       and mixed-precision calls on the 128 tile (a 256 tile never splits).
       -1 (default): the planner splits when the tiles would occupy at most
       half (FP64/FP32) or a quarter (mixed forms) of the resident workgroups,
       with slices of >= 16 k-steps (FP64/FP32), >= 256 k (split forms) or
       >= 1024 k (bfloat16, E4M3), at most 32 slices; 1: never; 2..32: slices of ceil(ksteps / value) k-steps
       (fewer slices if that leaves some empty).  The split depends on the
       shape and this attribute only, so every pack policy gives bit-identical
       C for a given split. */
    FIP_ATTR_SPLIT_K = 11,
    /* Read only: the 64-bit epoch stamp of the most recent fused call
       (claims and publish flags of that call hold this value; stamps are
       unique within the process). */
    FIP_ATTR_EPOCH = 5,
    /* Read only: the hipError_t of the last launch that failed on this handle
       (a call returning FIP_ERR_LAUNCH), 0 if none. */
    FIP_ATTR_LAST_HIP_ERROR = 12,
    /* Read only, batched calls: 1 + the largest index of a problem that the
       batched calls since the last read skipped because a device leading
       dimension was too small or a matrix spans 2 GiB or more (0: none).
       Reading it waits for the handle's stream and resets it to 0. */
    FIP_ATTR_VB_STATUS = 13,
    /* Pack copies of a fused call: 1 (one copy shared by all XCDs: a panel
       is packed once on the device, and the publish protocol's agent-scope
       release and acquire make it visible across XCDs) or 8 (one per XCD,
       indexed by the hardware XCC id: every XCD packs its own copy of each
       panel it reads); -1 (default): 1. */
    FIP_ATTR_COPIES = 14,
    /* Direct global-to-LDS loads.  An FP64/FP32 GEMM launch in which no
       workgroup produces a pack (pack-then-compute's CONSUME_ONLY call, an
       unpacked call, or a fused call whose plan packs nothing) and every chunk
       can be fetched whole (all chunks packed; or unpacked with k a multiple
       of the plan's KT, element-aligned operands, and m (n) a multiple of the
       16-byte vector width when op(A) (op(B)) is stored along it) may run the
       kernel variant that fetches each operand chunk with
       global_load_lds_dwordx4 (no staging registers, no LDS stores; the
       paper's Sec. 5 footnote expects DMA-fed packing to pay on GPUs).
       1: every eligible launch; 0: none (every chunk goes through registers);
       -1 (default): eligible binary64 launches that read their operands
       unpacked (measured faster there; binary32 and pack-then-compute
       consumers measured slower).  Same C bit for bit either way. */
    FIP_ATTR_DMA = 15,
    /* Read only: 1 if the most recent FP64/FP32 GEMM launch on the handle ran
       the direct global-to-LDS variant (FIP_ATTR_DMA), else 0. */
    FIP_ATTR_LAST_DMA = 16,
};

enum {
    FIP_PACK_AUTO = 0,         /* paper Sec. 3.3 reuse table and stride
                                  conditions: a panel is packed only if a later
                                  round of workgroups re-reads it (the launch
                                  has more tiles than fit on the device at
                                  once, more than 4 such rounds for the bfloat16
                                  split forms of binary32, and at least 4
                                  k-steps) and its unpacked read is slower than a
                                  packed one: every reused panel of the split
                                  forms (an unpacked read redoes the split), and
                                  for the other forms only the fringe panel of an
                                  operand whose extent is not a multiple of the
                                  tile (interior chunks read coalesced either
                                  way; see fip_plan_t.a_pack_first) */
    FIP_PACK_ALL = 1,          /* pack both operands whatever the shape */
    FIP_PACK_NONE = 2,         /* never pack (the unpacked "SUP" path, Sec. 2.3) */
    FIP_PACK_CONSUME_ONLY = 3, /* read only packed panels written beforehand by
                                  fip_pack (the pack-then-compute baseline) */
};
/* Stream capture: while the handle's stream is being captured into a graph,
   AUTO and ALL calls are planned as NONE (fip_plan reports it), so a captured
   GEMM replays correctly however its inputs change between replays: a fused
   pack's claims and flags carry an epoch chosen per call on the host, which a
   replay would reuse.  Split k and CONSUME_ONLY need no epoch and are kept. */

/*
 * The plan of one call, in the caller's terms (op(A) is m x k, op(B) k x n).
 * Packed layout (the contract): the pack of op(A) is ceil(m/MT)*ceil(k/KT)
 * contiguous blocks of KT*MT elements; block (t, q) (tile row t, k-step q) is
 * block number t*ceil(k/KT) + q (a copy that starts at tile row
 * a_pack_first holds block number (t - a_pack_first)*ceil(k/KT) + q).  Inside a block the tile keeps the
 * orientation op(A) has in storage: if A's storage runs along m (column-major
 * 'N', row-major 'T'), element (i, p) sits at (p % KT)*MT + (i % MT), each
 * k-slice contiguous; otherwise (column-major 'T', row-major 'N') at
 * (i % MT)*KT + (p % KT), each row's k-run contiguous.  The pack of op(B) is
 * the same with (MT, i) replaced by (NT, j): its storage runs along n for
 * column-major 'T' and row-major 'N'.  Entries outside the matrix are +0.0.
 * Element bits are copied unchanged; alpha is not folded in.
 * The fused path keeps one copy shared by all XCDs (copies = 1) or, with
 * FIP_ATTR_COPIES = 8, one per XCD (copies = 8), indexed by the hardware XCC
 * id of the workgroup that packs it; copy c of op(A)'s pack starts at
 * workspace + a_pack_offset + c * a_copy_bytes.  The standalone pack
 * (fip_pack) and CONSUME_ONLY use copy 0.
 * Mixed-precision forms (dtype FIP_BF16 .. FIP_BF16X3_FAST): MT = NT = 128
 * (256 for bfloat16 and E4M3, see FIP_ATTR_MX_TILE), KT = 64 (bfloat16), 128 (E4M3) or
 * 32 (split forms); blocks keep the operand's storage orientation as above
 * (a_kmajor / b_kmajor), and each holds PLANES planes of MT*KT packed elements
 * one after the other (PLANES = 3 for FIP_BF16X3, 2 for FIP_BF16X3_FAST,
 * else 1): plane t holds term t of the split (bfloat16 bits), or the
 * operand's own bfloat16 / E4M3 bits.  a_copy_bytes counts all planes.
 */
typedef struct {
    int32_t dtype, layout;
    int64_t m, n, k;
    int32_t MT, NT, KT;        /* tile extent along m, along n, and the k-step */
    int32_t tiles_m, tiles_n, ksteps;
    int32_t tile_class;        /* 0: 128x128, 1: 64x64, 2: 32x32 */
    int32_t pack_a, pack_b;    /* operand packed under this plan */
    int32_t copies;            /* pack copies laid out in the workspace */
    int32_t policy;            /* FIP_PACK_* in effect */
    int32_t a_kmajor, b_kmajor;/* packed block orientation: 1 = k-runs contiguous */
    int64_t a_pack_offset, a_copy_bytes;
    int64_t b_pack_offset, b_copy_bytes;
    int64_t a_flag_offset, b_flag_offset;   /* uint64 [copies][tiles][split_k]: panel
                                               (k-slice) complete */
    int64_t a_claim_offset, b_claim_offset; /* uint64 [copies][tiles][split_k] */
    int64_t stats_offset;      /* 4 x uint64: chunks packed, chunks read packed,
                                  chunks of packed panels read unpacked, re-polls */
    int64_t workspace_bytes;   /* bytes this call needs */
    int32_t split_k;           /* k-slices (1: k not split) */
    int32_t slice_ksteps;      /* k-steps per slice (the last one may have fewer) */
    int64_t partial_offset;    /* split_k > 1: the slices' partial products
                                  [split_k][kernel N][kernel M] (C's shape, column-major;
                                  transposed for row-major calls) in C's type, binary32
                                  for the mixed forms (FP8 scales applied); -1 otherwise */
    int32_t a_pack_first;      /* pack_a: the first tile row whose panel is packed (AUTO may
                                  pack only the fringe panel); a copy holds the panels
                                  from it on, panel t at block (t - a_pack_first) */
    int32_t b_pack_first;      /* the same for op(B)'s tile columns */
} fip_plan_t;

int fip_create(fip_handle_t* handle);
int fip_destroy(fip_handle_t handle);

/* hip_stream: a hipStream_t (NULL = the default stream). */
int fip_set_stream(fip_handle_t handle, void* hip_stream);

int fip_set_attr(fip_handle_t handle, int attr, int64_t value);
int fip_get_attr(fip_handle_t handle, int attr, int64_t* value);

/*
 * Hand the handle a caller-owned device buffer (256-byte aligned) for pack
 * panels, publish flags and statistics.  It must stay valid, and must not be
 * used by anyone else, while calls using it may be in flight.  Its initial
 * contents do not matter: flags and claims only count when they carry the
 * current call's unique stamp.  No HIP call is made.  bytes may be 0 (dptr
 * NULL) to detach.
 */
int fip_set_workspace(fip_handle_t handle, void* dptr, size_t bytes);

/*
 * Plan a call without running it: tile class, pack decision and workspace
 * layout for the given shape under the handle's current attributes.
 * dtype: any FIP_F64 .. FIP_BF16X3_FAST.  Writes *plan.  No HIP call is made.
 */
int fip_plan(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
             char transA, char transB, fip_plan_t* plan);

/* The plan of the most recent successful fip_dgemm / fip_sgemm / fip_pack. */
int fip_last_plan(fip_handle_t handle, fip_plan_t* plan);

/*
 * C := alpha*op(A)*op(B) + beta*C in binary64 (argument order follows the
 * BLAS gemm statement after handle and layout).
 * Leading dimensions must satisfy (column-major) lda >= max(1, transA=N ? m : k),
 * ldb >= max(1, transB=N ? k : n), ldc >= max(1, m); row-major swaps the roles
 * (lda >= max(1, transA=N ? k : m), ldb >= max(1, transB=N ? n : k),
 * ldc >= max(1, n)).  A pointer is invalid only if it would be read.
 * Quick returns (BLAS): m = 0 or n = 0 -> nothing; (alpha = 0 or k = 0) and
 * beta = 1 -> nothing; alpha = 0 or k = 0 -> C := beta*C without reading A, B
 * (beta = 0 writes zeros and does not read C).  beta = 0 never reads C.
 */
int fip_dgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, char transA, const double* B, int64_t ldb,
              char transB, double beta, double* C, int64_t ldc);

/*
 * fip_dgemm for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, semantics, argument checks and return codes as
 * fip_dgemm; the caller still owns A, B and C.  Instead of the handle's
 * workspace, the call uses a scratch array that the library owns: 64 MiB of
 * device memory per GPU (one copy on every GPU the library runs on, held until
 * the process ends).  It calls no hipMalloc, hipFree or other allocating
 * routine.  The plan is the one fip_plan reports under the handle's
 * attributes, except that a plan whose workspace would not fit in the array
 * runs without packing (the same kernel and k order, so the same C bit for
 * bit); if the split-k partial products alone need more than 64 MiB the call
 * returns FIP_ERR_WORKSPACE before launching anything.  Nothing in the array
 * needs clearing between calls (claims and flags carry per-call stamps), and
 * FIP_ATTR_STATS is ignored.  Every call on one GPU shares that GPU's array:
 * calls that may overlap in time on one GPU (two streams, two threads, two
 * handles) race on it and must be ordered by the caller.
 */
int fip_dgemm_noalloc(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, char transA, const double* B,
                      int64_t ldb, char transB, double beta, double* C, int64_t ldc);

/* The same in binary32 (FP32 MFMA, FP32 accumulation). */
int fip_sgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, float alpha,
              const float* A, int64_t lda, char transA, const float* B, int64_t ldb,
              char transB, float beta, float* C, int64_t ldc);

/*
 * Complex GEMM through the 1m method (paper Sec. 5: the 1m method encodes
 * complex multiplication in the packing stage so that the real microkernel
 * computes complex products).
 *
 *     C := alpha * op(A) * op(B) + beta * C     (complex; op in N, T, C where
 *                                                'C' is the conjugate transpose)
 *
 * Storage: A, B and C are DEVICE arrays of (re, im) pairs (C99/C++ complex
 * layout: binary64 pairs for fip_zgemm, binary32 for fip_cgemm), owned by the
 * caller; lda, ldb, ldc count complex elements and obey the same minimums as
 * fip_dgemm.  alpha and beta are HOST pointers to one (re, im) pair each,
 * read during the call.
 *
 * Method: the kernel multiplies two real matrices.  Its A side is the
 * 2m x 2k expansion of op(A) (complex element z becomes the 2 x 2 block
 * [[re z, -im z], [im z, re z]]), its B side the 2k x n expansion of op(B)
 * (element w becomes re w over im w), and their real product is the real view
 * of the column-major complex C.  Row-major C runs as C^T = op(B)^T op(A)^T.
 * The expansion is done while loading, so a first pass packs expanded chunks
 * and later passes read them: the packed operands of fip_plan (dtype
 * FIP_C128 / FIP_C64) are the real expanded matrices in the tile layout of the
 * real path, and MT, KT, tiles_m, ksteps are real-expanded quantities (m, n,
 * k stay the caller's).  Split k is not used.  Precision: binary64 (binary32)
 * products and sums, per real component a sum of 2k products.
 *
 * Return codes: as fip_dgemm, with positions handle 1, layout 2, m 3, n 4,
 * k 5, alpha 6, A 7, lda 8, transA 9, B 10, ldb 11, transB 12, beta 13, C 14,
 * ldc 15 (a null alpha or beta is invalid).  Quick returns: m = 0 or n = 0, or
 * (alpha = 0 or k = 0) and beta = 1: nothing; alpha = 0 or k = 0: C := beta C
 * without reading A or B; beta = 0 never reads C.
 */
int fip_zgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
              const double* alpha, const double* A, int64_t lda, char transA, const double* B,
              int64_t ldb, char transB, const double* beta, double* C, int64_t ldc);
int fip_cgemm(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k,
              const float* alpha, const float* A, int64_t lda, char transA, const float* B,
              int64_t ldb, char transB, const float* beta, float* C, int64_t ldc);

/*
 * Standalone pack (Sec. 2.1: conventional pack-then-compute): write copy 0 of
 * the packed op(A) and op(B) that a CONSUME_ONLY call of the same shape,
 * dtype (any FIP_F64 .. FIP_C64; complex dtypes pack the 1m expansions) and tile class reads.  Both operands
 * are packed whatever the shape.  Arguments as in fip_dgemm.
 */
int fip_pack(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
             const void* A, int64_t lda, char transA, const void* B, int64_t ldb, char transB);

/*
 * Other level-3 operations through the same fused-pack tile kernel (paper
 * Sec. 2.2: BLIS casts every level-3 operation onto one packing and
 * microkernel layer; Sec. 5: fused packing for those operations).  binary64
 * (d) and binary32 (s); conventions, quick returns and errors as fip_dgemm.
 *
 * SYRK:  C := alpha * op(A) * op(A)^T + beta * C on the uplo triangle of the
 *        n x n matrix C ('L': row >= column, 'U': row <= column); the other
 *        triangle is neither read nor written.  op(A) is n x k: A for trans
 *        'N', A^T for 'T'/'C'.  Only the tiles of the triangle are launched;
 *        both operand sides of a tile read the one op(A), whose panels are
 *        claimed, packed and published once for both roles.
 *        lda >= max(1, (column-major) == (trans 'N') ? n : k); ldc >= max(1, n).
 *        Positions: layout 2, uplo 3, trans 4, n 5, k 6, alpha 7, A 8, lda 9,
 *        beta 10, C 11, ldc 12.
 * TRMM (out of place, with beta):
 *        C := alpha * op(T) * B + beta * C   (side 'L', T m x m), or
 *        C := alpha * B * op(T) + beta * C   (side 'R', T n x n),
 *        B and C m x n; T is the uplo triangle of the stored A ('L': row >=
 *        column, 'U': row <= column), its diagonal taken as 1 and not read when
 *        diag is 'U'; A's other triangle is not read.  Chunks of the triangular
 *        operand that meet the diagonal get the triangle applied in registers
 *        (zeros elsewhere, ones on a unit diagonal), its all-zero k-steps are
 *        skipped, and its pack holds op(T) with the triangle applied; the dense
 *        B is never packed.  Structural zeros inside a diagonal chunk are
 *        multiplied as +0.0 (an Inf or NaN in B meeting one gives NaN where the
 *        BLAS definition, which never multiplies them, would not).
 *        lda >= max(1, side 'L' ? m : n); ldb, ldc >= max(1, column-major ? m : n).
 *        Positions: layout 2, side 3, uplo 4, transA 5, diag 6, m 7, n 8,
 *        alpha 9, A 10, lda 11, B 12, ldb 13, beta 14, C 15, ldc 16.
 * Packing policies: AUTO and ALL as for fip_dgemm (for AUTO, Sec. 3.3's rule
 * on the one packable operand); NONE never packs; CONSUME_ONLY runs unpacked
 * (there is no standalone pack for these operations).  Split k is not used.
 */
enum { FIP_OP_SYRK = 1, FIP_OP_TRMM = 2, FIP_OP_TRSM = 3 };
int fip_dsyrk(fip_handle_t handle, int layout, char uplo, char trans, int64_t n, int64_t k,
              double alpha, const double* A, int64_t lda, double beta, double* C, int64_t ldc);
int fip_ssyrk(fip_handle_t handle, int layout, char uplo, char trans, int64_t n, int64_t k,
              float alpha, const float* A, int64_t lda, float beta, float* C, int64_t ldc);
int fip_dtrmm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, double alpha, const double* A, int64_t lda, const double* B,
              int64_t ldb, double beta, double* C, int64_t ldc);
int fip_strmm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, float alpha, const float* A, int64_t lda, const float* B,
              int64_t ldb, float beta, float* C, int64_t ldc);
/*
 * TRSM: solve op(T) X = alpha B (side 'L', T m x m) or X op(T) = alpha B
 * (side 'R', T n x n) for X, B m x n; T is the uplo triangle of A, with a
 * unit diagonal (not read) for diag 'U'; the other triangle of A is never
 * read.  X overwrites B (BLAS semantics).  Method: recursive blocking on the
 * column-major view: op(T) is split in two at a multiple of 64 rows; the half
 * solved first takes alpha, the rest of B becomes alpha B minus the coupling
 * block of op(T) times the solved part, a GEMM through the fused-pack tile
 * kernel (with the handle's pack policy and workspace), and the remaining
 * half is solved with alpha = 1; diagonal blocks of at most 64 rows are solved
 * by substitution, one right-hand side per thread.  The workspace must hold
 * what the largest GEMM update needs (fip_plan_l3 with FIP_OP_TRSM reports it);
 * otherwise FIP_ERR_WORKSPACE is returned before anything is launched.  After
 * the call fip_last_plan reports its last GEMM update.  alpha = 0: B := 0
 * without reading A or B.  Positions: layout 2, side 3, uplo 4, transA 5,
 * diag 6, m 7, n 8, alpha 9, A 10, lda 11 (>= max(1, side 'L' ? m : n)),
 * B 12, ldb 13 (>= max(1, column-major ? m : n)).
 */
int fip_dtrsm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, double alpha, const double* A, int64_t lda, double* B,
              int64_t ldb);
int fip_strsm(fip_handle_t handle, int layout, char side, char uplo, char transA, char diag,
              int64_t m, int64_t n, float alpha, const float* A, int64_t lda, float* B,
              int64_t ldb);
/*
 * Plan of a SYRK (op FIP_OP_SYRK: n, k; side and diag ignored), TRMM
 * (FIP_OP_TRMM: m, n; k ignored) or TRSM (FIP_OP_TRSM: m, n; k ignored) call:
 * tile class, pack decision and workspace bytes (FIP_F64 or FIP_F32).  The
 * plan's "A" is op(A) (SYRK; its "B" is the same pack) or the triangular
 * matrix (TRMM); for TRSM the plan is that of the top-level GEMM update, with
 * workspace_bytes the largest any of its updates needs.  No HIP call.
 * Positions: op 2, dtype 3, layout 4, side 5, uplo 6, trans 7, diag 8, m 9,
 * n 10, k 11, plan 12.
 */
int fip_plan_l3(fip_handle_t handle, int op, int dtype, int layout, char side, char uplo,
                char trans, char diag, int64_t m, int64_t n, int64_t k, fip_plan_t* plan);

/*
 * Mixed-precision GEMM (paper Sec. 5: the fused packing carried over to other
 * precisions; the pack is where operands are converted):
 *
 *     C := alpha * op(A) * op(B) + beta * C
 *
 * with binary32 accumulation (MFMA) and the operand forms
 *   FIP_BF16         A, B bfloat16 (uint16 bit patterns).
 *   FIP_E4M3         A, B OCP FP8 E4M3 codes (uint8), the values being q / s:
 *                    a_scale[i] (length m, per row of op(A)) and b_scale[j]
 *                    (length n, per column of op(B)) are the power-of-two
 *                    scales the codes were made with (see fip_quantize_fp8);
 *                    NULL means 1.  The product is divided by
 *                    a_scale[i]*b_scale[j] in the epilogue.
 *   FIP_BF16X3       A, B binary32; while packing, each element x becomes
 *                    x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0),
 *                    x2 = bf16(x - x0 - x1) (round to nearest even), and the
 *                    product keeps the six terms x_i*y_j with i + j <= 2.
 *   FIP_BF16X3_FAST  the same with x0 + x1 and the three terms i + j <= 1.
 * c_type: FIP_F32 (C binary32) or FIP_BF16 (C bfloat16; read, when beta != 0,
 * as binary32, and the result rounded to nearest even).  alpha, beta binary32.
 * a_scale / b_scale must be NULL for the forms other than FIP_E4M3.
 * Packing policy, workspace, quick returns, leading-dimension rules and
 * argument-position errors as in fip_dgemm (positions: dtype 2, layout 3,
 * m 4, n 5, k 6, alpha 7, A 8, lda 9, transA 10, B 11, ldb 12, transB 13,
 * beta 14, C 15, ldc 16, c_type 17, a_scale 18, b_scale 19).  Device pointers.
 */
int fip_gemm_mx(fip_handle_t handle, int dtype, int layout, int64_t m, int64_t n, int64_t k,
                float alpha, const void* A, int64_t lda, char transA, const void* B, int64_t ldb,
                char transB, float beta, void* C, int64_t ldc, int c_type, const float* a_scale,
                const float* b_scale);

/*
 * Quantize a binary32 matrix X (rows x cols, stored in layout with leading
 * dimension ldx) to OCP FP8 E4M3 with one power-of-two scale per row
 * (axis = 0) or per column (axis = 1):
 *   s_line = 2^e, e the largest integer with amax_line * 2^e <= 448
 *            (e = 0 when the line is all zero), clamped to [-126, 126];
 *   Q[r, c] = e4m3(X[r, c] * s_line), round to nearest even, saturating at
 *            +-448 (NaN -> 0x7F); NaNs do not count towards amax.
 * Q (uint8, same layout, leading dimension ldq) and scales (binary32, rows or
 * cols entries) are device buffers owned by the caller; scales is also used
 * as scratch while the call runs.  For fip_gemm_mx, quantize op(A) per row
 * and op(B) per column.  Four kernel launches on the handle's stream.
 * Positions: layout 2, rows 3, cols 4, X 5, ldx 6, axis 7, Q 8, ldq 9, scales 10.
 */
int fip_quantize_fp8(fip_handle_t handle, int layout, int64_t rows, int64_t cols, const float* X,
                     int64_t ldx, int axis, uint8_t* Q, int64_t ldq, float* scales);

/*
 * Batched binary32 GEMM: count independent problems
 *
 *     C_i := alpha * op(A_i) * op(B_i) + beta * C_i,   i = 0 .. count-1,
 *
 * op(A_i) m[i] x k[i], op(B_i) k[i] x n[i], all in one persistent launch (the
 * paper's single code path applied to a whole batch of small and uneven
 * problems: every problem runs the unpacked tile path, Sec. 2.3 and 3.3).
 * Each tile (32 x 32 or 16 x 16, see FIP_ATTR_VB_SPLIT) is computed by one
 * wave; the waves of the grid take tiles from a longest-first list.
 *   m, n, k, transA, transB: HOST arrays of count entries (the planner needs
 *     them; a batch with the same shapes reuses the plan uploaded by the
 *     previous call).
 *   A, B, C: DEVICE arrays of count device pointers; lda, ldb, ldc: DEVICE
 *     arrays of count leading dimensions.  They never reach the host, so the
 *     kernel checks them: a problem whose leading dimension is below the
 *     extent it strides over (as in fip_sgemm), or one of whose matrices spans
 *     2 GiB or more, is skipped (its C is not written) and reported through
 *     FIP_ATTR_VB_STATUS.  All matrices in `layout`, C distinct from A and B.
 *   flags: 0, or FIP_VB_GRAPH: run the batch as a HIP graph, instantiated on
 *     the first call and replayed while the call repeats with the same shapes,
 *     pointer arrays, alpha, beta, workspace and stream.
 * Workspace: fip_vbatched_workspace bytes (problem table and tile list); it
 * must hold the plan between calls of the same batch.  A call with a new batch waits for the stream and
 * copies the new plan in (synchronous host-to-device copies).
 * Quick returns: count = 0, or alpha = 0 and beta = 1.  alpha = 0 reads no
 * A, B; beta = 0 reads no C.  k[i] = 0 gives C_i := beta*C_i.
 * Positions: layout 2, count 3, m 4, n 5, k 6, transA 7, transB 8, alpha 9,
 * A 10, lda 11, B 12, ldb 13, beta 14, C 15, ldc 16, flags 17.
 */
#define FIP_VB_GRAPH 1
int fip_vbatched_workspace(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                           const int32_t* n, const int32_t* k, const char* transA,
                           const char* transB, size_t* bytes);
int fip_sgemm_vbatched(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                       const int32_t* n, const int32_t* k, const char* transA, const char* transB,
                       float alpha, const float* const* A, const int64_t* lda,
                       const float* const* B, const int64_t* ldb, float beta, float* const* C,
                       const int64_t* ldc, int flags);

/*
 * Autotuner of the batched call: times the batch (median of 3 launches after
 * a warm-up) for each candidate FIP_ATTR_VB_SPLIT threshold (0, 8, 16, 24,
 * 32, 48, 64, all), keeps the fastest for this batch's shapes in
 * the handle (later fip_sgemm_vbatched calls with the same shapes use it) and
 * writes it to *split_out.  It runs the batch 32 times: C is overwritten with
 * unspecified values, so pass scratch C matrices of the same shapes.
 * Arguments as in fip_sgemm_vbatched; position 17 is split_out.  Synchronous.
 */
int fip_vbatched_tune(fip_handle_t handle, int layout, int64_t count, const int32_t* m,
                      const int32_t* n, const int32_t* k, const char* transA, const char* transB,
                      float alpha, const float* const* A, const int64_t* lda,
                      const float* const* B, const int64_t* ldb, float beta, float* const* C,
                      const int64_t* ldc, int* split_out);

/*
 * Autotuner of the FP64 / FP32 GEMM plan (the paper's Sec. 3.3 leaves its
 * blocking choices to tuning): times the call (a warm-up, then the median of
 * 3 launches on the handle's stream) for every tile class (128, 64, 32), each
 * with the planner's k split and with none (configurations that plan alike
 * are timed once), under the handle's pack policy and other attributes.  The
 * fastest is kept in the handle for this call shape (dtype, layout, m, n, k,
 * transA, transB): later calls, fip_plan and workspace queries with the same
 * shape use it while FIP_ATTR_TILE and FIP_ATTR_SPLIT_K are -1.  Writes the
 * tile class to *tile_out and the split (-1: the planner's, 1: none) to
 * *split_out.  C is overwritten with unspecified values (several products
 * accumulate into it when beta != 0): pass a scratch C of the same shape.
 * Arguments as in fip_dgemm / fip_sgemm; positions 16 tile_out, 17
 * split_out.  Quick return (nothing timed, the planner's choice reported):
 * m, n or k = 0, or alpha = 0.  Synchronous.
 */
int fip_dgemm_tune(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, double alpha,
                   const double* A, int64_t lda, char transA, const double* B, int64_t ldb,
                   char transB, double beta, double* C, int64_t ldc, int* tile_out,
                   int* split_out);
int fip_sgemm_tune(fip_handle_t handle, int layout, int64_t m, int64_t n, int64_t k, float alpha,
                   const float* A, int64_t lda, char transA, const float* B, int64_t ldb,
                   char transB, float beta, float* C, int64_t ldc, int* tile_out, int* split_out);

/*
 * Persisted tuning table (host only, no HIP call).  fip_tune_save writes
 * every choice the handle holds (fip_dgemm_tune / fip_sgemm_tune entries and
 * fip_vbatched_tune thresholds) to the text file at path (created or
 * replaced): a header line "fipgemm-tune 1", then one line per entry,
 * "gemm dtype layout m n k tA tB tile split" (tA, tB: 1 transposed) or
 * "vb signature split".  fip_tune_load reads such a file into the handle,
 * replacing entries with the same key and keeping the others; the file is
 * checked whole first, so a malformed file changes nothing.  Returns 0, 1 if
 * path is null or the file cannot be opened or written, 2 if its contents
 * are malformed, FIP_ERR_ALLOC.
 */
int fip_tune_save(fip_handle_t handle, const char* path);
int fip_tune_load(fip_handle_t handle, const char* path);

/*
 * Diagnostic (host only, no HIP call): the tile that workgroup w of a launch
 * over tiles_m x tiles_n C tiles computes, for tile order 0 or 1 (see
 * FIP_ATTR_ORDER): tm[w], tn[w] for w = 0 .. tiles_m*tiles_n - 1 (host
 * arrays).  The tile kernels use this same map.
 * Positions: tiles_m 1, tiles_n 2, order 3, tm 4, tn 5.
 */
int fip_tile_map(int64_t tiles_m, int64_t tiles_n, int order, int32_t* tm, int32_t* tn);

/*
 * Diagnostic: launch nblocks one-wave workgroups; workgroup b writes the
 * hardware XCC id it ran on to d_out[b] (device array of nblocks uint32).
 * The fused path's per-XCD pack copies are indexed by this id.
 */
int fip_xcc_map(fip_handle_t handle, uint32_t* d_out, int64_t nblocks);

#ifdef __cplusplus
}
#endif
#endif /* FIPGEMM_H */
