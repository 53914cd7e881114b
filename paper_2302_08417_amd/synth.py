"""Seeded synthetic GEMM operands (shared by tests, benchmark and smoke check).

This module only draws random numbers and sizes storage; it contains none of
the GEMM's arithmetic.  Each operand is returned as a flat NumPy buffer holding
the stored matrix exactly as BLAS arguments (layout, trans, ld) describe it.
Entries between the logical matrix and its leading dimension ("ld padding")
are filled with NaN so that any read of them poisons the result.

Workload shapes follow the paper's experiments: square m = n = k sweeps with
LDim equal to the row count or padded (Sec. 4.2).
"""
from dataclasses import dataclass

import numpy as np

COL, ROW = 0, 1
BASE_SEED = 2302_08417


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def is_trans(t: str) -> bool:
    return t in "TtCc"


def stored_shape(trans: str, rows: int, cols: int):
    """(rows, cols) of the stored matrix whose op() is rows x cols."""
    return (cols, rows) if is_trans(trans) else (rows, cols)


def min_ld(layout: int, srows: int, scols: int) -> int:
    return max(1, srows if layout == COL else scols)


def buffer_len(layout: int, srows: int, scols: int, ld: int) -> int:
    if srows == 0 or scols == 0:
        return 1
    return ld * scols if layout == COL else ld * srows


def fill_stored(layout: int, srows: int, scols: int, ld: int, values: np.ndarray,
                dtype, pad_value=np.nan) -> np.ndarray:
    """Place a (srows, scols) array into a flat buffer with leading dimension ld."""
    buf = np.full(buffer_len(layout, srows, scols, ld), pad_value, dtype=dtype)
    if srows and scols:
        if layout == COL:
            view = buf[: ld * scols].reshape(scols, ld)[:, :srows]
            view[:, :] = values.T
        else:
            view = buf[: ld * srows].reshape(srows, ld)[:, :scols]
            view[:, :] = values
    return buf


@dataclass
class GemmCase:
    layout: int
    m: int
    n: int
    k: int
    transA: str
    transB: str
    lda: int
    ldb: int
    ldc: int
    alpha: float
    beta: float
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    dtype: type


def make_case(layout=COL, m=64, n=64, k=64, transA="N", transB="N", ld_pad=0,
              alpha=1.5, beta=0.5, dtype=np.float64, seed=BASE_SEED, dist="uniform",
              int_range=8, pad_value=np.nan) -> GemmCase:
    """Operands for C := alpha*op(A)*op(B) + beta*C with seeded entries.

    dist: "uniform" -> U[-1, 1]; "int" -> integers in [-int_range, int_range];
          "normal" -> N(0, 1).
    ld_pad: extra leading-dimension padding (0 -> ld = minimal, 7 -> rows + 7).
    """
    g = rng(seed)

    def draw(shape):
        if dist == "uniform":
            return g.uniform(-1.0, 1.0, size=shape)
        if dist == "int":
            return g.integers(-int_range, int_range + 1, size=shape).astype(np.float64)
        if dist == "normal":
            return g.standard_normal(size=shape)
        raise ValueError(dist)

    sa = stored_shape(transA, m, k)
    sb = stored_shape(transB, k, n)
    lda = min_ld(layout, *sa) + ld_pad
    ldb = min_ld(layout, *sb) + ld_pad
    ldc = min_ld(layout, m, n) + ld_pad
    A = fill_stored(layout, sa[0], sa[1], lda, draw(sa), dtype, pad_value)
    B = fill_stored(layout, sb[0], sb[1], ldb, draw(sb), dtype, pad_value)
    C = fill_stored(layout, m, n, ldc, draw((m, n)), dtype, pad_value)
    return GemmCase(layout, m, n, k, transA, transB, lda, ldb, ldc, alpha, beta, A, B, C, dtype)


def op_view(buf: np.ndarray, layout: int, trans: str, rows: int, cols: int, ld: int) -> np.ndarray:
    """op(X) as a (rows, cols) NumPy view of a stored buffer (index plumbing only)."""
    sr, sc = stored_shape(trans, rows, cols)
    if sr == 0 or sc == 0:
        return np.zeros((rows, cols), dtype=buf.dtype)
    if layout == COL:
        st = buf[: ld * sc].reshape(sc, ld)[:, :sr].T
    else:
        st = buf[: ld * sr].reshape(sr, ld)[:, :sc]
    return st.T if is_trans(trans) else st


def sample_entries(m: int, n: int, count: int, seed: int):
    """Entry coordinates: the four corners, the last row/column fringes, then random."""
    g = rng(seed)
    pts = set()
    for i in (0, m - 1):
        for j in (0, n - 1):
            pts.add((i, j))
    for j in range(0, n, max(1, n // 64)):
        pts.add((m - 1, j))
    for i in range(0, m, max(1, m // 64)):
        pts.add((i, n - 1))
    while len(pts) < min(count, m * n):
        pts.add((int(g.integers(0, m)), int(g.integers(0, n))))
    arr = np.array(sorted(pts), dtype=np.int64)
    return arr[:, 0].copy(), arr[:, 1].copy()


# ---------------------------------------------------------------------------
# Complex operands (complex GEMM): real and imaginary parts drawn independently
# with the real recipe; stored as complex128 or complex64 arrays (interleaved
# re, im), ld padding filled with NaN + NaN i.

@dataclass
class CxCase:
    layout: int
    m: int
    n: int
    k: int
    transA: str
    transB: str
    lda: int
    ldb: int
    ldc: int
    alpha: complex
    beta: complex
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    dtype: type


def make_cx_case(layout=COL, m=64, n=64, k=64, transA="N", transB="N", ld_pad=0,
                 alpha=1.5 - 0.5j, beta=0.5 + 0.25j, dtype=np.complex128, seed=BASE_SEED,
                 dist="uniform", int_range=8) -> CxCase:
    """dist: "uniform" -> re, im ~ U[-1, 1]; "int" -> integers in [-int_range, int_range]."""
    g = rng(seed)

    def draw(shape):
        if dist == "uniform":
            return g.uniform(-1.0, 1.0, size=shape) + 1j * g.uniform(-1.0, 1.0, size=shape)
        if dist == "int":
            return (g.integers(-int_range, int_range + 1, size=shape)
                    + 1j * g.integers(-int_range, int_range + 1, size=shape))
        raise ValueError(dist)

    pad = complex(np.nan, np.nan)
    sa = stored_shape(transA, m, k)
    sb = stored_shape(transB, k, n)
    lda = min_ld(layout, *sa) + ld_pad
    ldb = min_ld(layout, *sb) + ld_pad
    ldc = min_ld(layout, m, n) + ld_pad
    A = fill_stored(layout, sa[0], sa[1], lda, draw(sa), dtype, pad)
    B = fill_stored(layout, sb[0], sb[1], ldb, draw(sb), dtype, pad)
    C = fill_stored(layout, m, n, ldc, draw((m, n)), dtype, pad)
    return CxCase(layout, m, n, k, transA, transB, lda, ldb, ldc, complex(alpha), complex(beta),
                  A, B, C, dtype)


def cx_op_view(buf, layout, trans, rows, cols, ld):
    """op(X) of a stored complex buffer, conjugated for 'C' (index plumbing and the
    definition of op; no product arithmetic)."""
    v = op_view(buf, layout, trans, rows, cols, ld)
    return np.conj(v) if trans in "Cc" else v


# ---------------------------------------------------------------------------
# Mixed-precision operands.  Entries are U[-1, 1] with every row of op(A) and
# every column of op(B) scaled by 2^u, u ~ U[-8, 8] (rows and columns of very
# different magnitude).  Operand storage: bfloat16 bit patterns (uint16),
# E4M3 codes (uint8) or binary32, with NaN patterns in the ld padding.
# Conversions to the stored formats use torch's CPU casts (input preparation
# only; the library and the oracle each implement their own).

FORM_BF16, FORM_E4M3, FORM_BF16X3, FORM_BF16X3_FAST = 2, 3, 4, 5
BF16_NAN, E4M3_NAN = 0x7FC0, 0x7F


@dataclass
class MxCase:
    form: int
    layout: int
    m: int
    n: int
    k: int
    transA: str
    transB: str
    lda: int
    ldb: int
    ldc: int
    alpha: float
    beta: float
    A: np.ndarray          # stored operand (uint16 bits, uint8 codes or float32)
    B: np.ndarray
    C: np.ndarray          # float32, or uint16 bfloat16 bits when c_bf16
    c_bf16: bool
    a_scale: np.ndarray    # E4M3: power-of-two scale per row of op(A) (float32), else None
    b_scale: np.ndarray    # E4M3: per column of op(B), else None
    A32: np.ndarray        # binary32 values the operand was made from (same storage)
    B32: np.ndarray


def _to_bf16_bits(x: np.ndarray) -> np.ndarray:
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def _to_e4m3_codes(x: np.ndarray) -> np.ndarray:
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.float8_e4m3fn)
    return t.view(torch.uint8).numpy()


def make_mx_case(form, layout=COL, m=64, n=64, k=64, transA="N", transB="N", ld_pad=0,
                 alpha=1.0, beta=0.0, seed=BASE_SEED, c_bf16=False, spread=8.0) -> MxCase:
    g = rng(seed)
    row_exp = g.uniform(-spread, spread, size=m)   # per row of op(A)
    col_exp = g.uniform(-spread, spread, size=n)   # per column of op(B)
    opA = g.uniform(-1.0, 1.0, size=(m, k)) * np.exp2(row_exp)[:, None]
    opB = g.uniform(-1.0, 1.0, size=(k, n)) * np.exp2(col_exp)[None, :]
    a_scale = b_scale = None
    if form == FORM_E4M3:
        # codes of x * s with s = 2^(8 - round(u)) per line (|x * s| <= 2^8.5 < 448)
        a_scale = np.exp2(8.0 - np.round(row_exp)).astype(np.float32)
        b_scale = np.exp2(8.0 - np.round(col_exp)).astype(np.float32)
        opAq = opA * a_scale[:, None]
        opBq = opB * b_scale[None, :]
    sa = stored_shape(transA, m, k)
    sb = stored_shape(transB, k, n)
    stA = opA.T if is_trans(transA) else opA
    stB = opB.T if is_trans(transB) else opB
    lda = min_ld(layout, *sa) + ld_pad
    ldb = min_ld(layout, *sb) + ld_pad
    ldc = min_ld(layout, m, n) + ld_pad
    A32 = fill_stored(layout, sa[0], sa[1], lda, stA, np.float32)
    B32 = fill_stored(layout, sb[0], sb[1], ldb, stB, np.float32)
    if form == FORM_BF16:
        A = fill_stored(layout, sa[0], sa[1], lda, _to_bf16_bits(stA).astype(np.float64),
                        np.uint16, BF16_NAN)
        B = fill_stored(layout, sb[0], sb[1], ldb, _to_bf16_bits(stB).astype(np.float64),
                        np.uint16, BF16_NAN)
    elif form == FORM_E4M3:
        qA = opAq.T if is_trans(transA) else opAq
        qB = opBq.T if is_trans(transB) else opBq
        A = fill_stored(layout, sa[0], sa[1], lda, _to_e4m3_codes(qA).astype(np.float64),
                        np.uint8, E4M3_NAN)
        B = fill_stored(layout, sb[0], sb[1], ldb, _to_e4m3_codes(qB).astype(np.float64),
                        np.uint8, E4M3_NAN)
    else:
        A, B = A32, B32
    Cv = g.uniform(-1.0, 1.0, size=(m, n))
    if c_bf16:
        C = fill_stored(layout, m, n, ldc, _to_bf16_bits(Cv).astype(np.float64), np.uint16,
                        BF16_NAN)
    else:
        C = fill_stored(layout, m, n, ldc, Cv, np.float32)
    return MxCase(form, layout, m, n, k, transA, transB, lda, ldb, ldc, alpha, beta, A, B, C,
                  c_bf16, a_scale, b_scale, A32, B32)


# ---------------------------------------------------------------------------
# Batches of independent, unevenly sized problems: m, n, k each
# round(exp(U[ln lo, ln hi])) (log-uniform), transA / transB each 'N' or 'T'
# with probability 1/2, entries U[-1, 1], optional ld padding (NaN-filled).

@dataclass
class Batch:
    layout: int
    count: int
    m: np.ndarray        # int32
    n: np.ndarray
    k: np.ndarray
    transA: np.ndarray   # uint8 codes of 'N' / 'T'
    transB: np.ndarray
    lda: np.ndarray      # int64
    ldb: np.ndarray
    ldc: np.ndarray
    alpha: float
    beta: float
    A: list              # per problem: flat float32 buffers
    B: list
    C: list


def make_batch(count, layout=COL, lo=4, hi=512, ld_pad=0, alpha=1.5, beta=0.5,
               seed=BASE_SEED, zero_sizes=False) -> Batch:
    g = rng(seed)

    def dims():
        return np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int32)

    m, n, k = dims(), dims(), dims()
    if zero_sizes and count >= 3:   # a few degenerate problems
        m[0] = 0
        n[1] = 0
        k[2] = 0
    tA = np.where(g.random(count) < 0.5, ord("N"), ord("T")).astype(np.uint8)
    tB = np.where(g.random(count) < 0.5, ord("N"), ord("T")).astype(np.uint8)
    lda = np.empty(count, np.int64)
    ldb = np.empty(count, np.int64)
    ldc = np.empty(count, np.int64)
    As, Bs, Cs = [], [], []
    for i in range(count):
        ta, tb = chr(tA[i]), chr(tB[i])
        sa = stored_shape(ta, int(m[i]), int(k[i]))
        sb = stored_shape(tb, int(k[i]), int(n[i]))
        lda[i] = min_ld(layout, *sa) + ld_pad
        ldb[i] = min_ld(layout, *sb) + ld_pad
        ldc[i] = min_ld(layout, int(m[i]), int(n[i])) + ld_pad
        As.append(fill_stored(layout, sa[0], sa[1], int(lda[i]), g.uniform(-1, 1, sa), np.float32))
        Bs.append(fill_stored(layout, sb[0], sb[1], int(ldb[i]), g.uniform(-1, 1, sb), np.float32))
        Cs.append(fill_stored(layout, int(m[i]), int(n[i]), int(ldc[i]),
                              g.uniform(-1, 1, (int(m[i]), int(n[i]))), np.float32))
    return Batch(layout, count, m, n, k, tA, tB, lda, ldb, ldc, alpha, beta, As, Bs, Cs)


def mx_device_operands(form, n, seed=BASE_SEED, device="cuda"):
    """Large square mixed-precision operands drawn directly on the GPU (torch's seeded
    generator; same value recipe as make_mx_case: U[-1, 1] with rows of A and columns of B
    scaled by 2^u, u ~ U[-8, 8]), column-major, no transpose, ld = n.  Returns
    (A, B, a_scale, b_scale, A32, B32) as torch tensors; A32/B32 are the binary32 values the
    stored operands were made from (for E4M3, the codes are those values times the scales)."""
    import torch
    g = torch.Generator(device=device).manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    u_row = torch.rand(n, device=device, generator=g) * 16 - 8
    u_col = torch.rand(n, device=device, generator=g) * 16 - 8
    # column-major storage: element (i, p) of A at A[p, i] of a row-major (k, m) tensor
    A32 = (torch.rand(n, n, device=device, generator=g) * 2 - 1) * torch.exp2(u_row)[None, :]
    B32 = (torch.rand(n, n, device=device, generator=g) * 2 - 1) * torch.exp2(u_col)[:, None]
    sa = sb = None
    if form == FORM_BF16:
        A, B = A32.to(torch.bfloat16), B32.to(torch.bfloat16)
    elif form == FORM_E4M3:
        sa = torch.exp2(8 - torch.round(u_row))
        sb = torch.exp2(8 - torch.round(u_col))
        A = (A32 * sa[None, :]).to(torch.float8_e4m3fn).view(torch.uint8)
        B = (B32 * sb[:, None]).to(torch.float8_e4m3fn).view(torch.uint8)
    else:
        A, B = A32, B32
    return A, B, sa, sb, A32, B32
