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
