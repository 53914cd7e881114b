"""GPU parity of TRSM (recursive blocking: GEMM updates through the fused-pack tile kernel,
diagonal blocks of at most 64 rows by substitution) against the oracle.

Systems are strongly diagonally dominant (each row's off-diagonal magnitudes sum to less than
half the diagonal), so the solution is well conditioned and a backward-stable solve lands
within a small multiple of k u of the oracle's: the bound used is
    max |X - Xref| <= 16 * k * u * max |Xref|
with k the order of T and u the working unit roundoff, plus the residual
    max |op(T) X - alpha B| <= 8 * k * u * max (|op(T)| |X| + |alpha B|)
(computed in binary64).  Every packing policy of the GEMM updates gives the same bits.  The
entries TRSM must not read (the other triangle, a unit diagonal) hold NaN.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from gemm_util import U, to_dev
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

pytestmark = pytest.mark.gpu

F64, F32 = np.float64, np.float32
CASES = list(itertools.product([COL, ROW], "LR", "LU", "NT", "NU"))


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print("[trsm]", *a, flush=True)
    sys.stdout.flush()


class Case:
    pass


def trsm_case(layout, side, uplo, trans, diag, m, n, dtype, seed, alpha=1.5, pad=3):
    g = synth.rng(seed)
    ka = m if side == "L" else n
    Av = g.uniform(-1, 1, (ka, ka)) / (2 * ka)
    np.fill_diagonal(Av, g.choice([-1.0, 1.0], size=ka) * g.uniform(1, 2, size=ka))
    notref = ~(np.tril(np.ones((ka, ka), bool)) if uplo == "L" else np.triu(np.ones((ka, ka), bool)))
    if diag == "U":
        notref |= np.eye(ka, dtype=bool)
    Ap = Av.copy()
    Ap[notref] = np.nan
    c = Case()
    c.layout, c.side, c.uplo, c.trans, c.diag, c.m, c.n, c.alpha, c.dtype = \
        layout, side, uplo, trans, diag, m, n, alpha, dtype
    c.lda = ka + pad
    c.A = synth.fill_stored(layout, ka, ka, c.lda, Ap, dtype)
    c.ldb = (m if layout == COL else n) + pad
    c.B = synth.fill_stored(layout, m, n, c.ldb, g.uniform(-1, 1, (m, n)), dtype)
    c.T = np.where(notref, 0.0, Av)
    if diag == "U":
        np.fill_diagonal(c.T, 1.0)
    c.T = c.T.astype(dtype).astype(np.float64)
    return c


def run_trsm(F, c, policy=0):
    import torch
    h = F.Handle(policy=policy)
    A, B = to_dev(c.A), to_dev(c.B)
    h.trsm(c.layout, c.side, c.uplo, c.trans, c.diag, c.m, c.n, c.alpha, A, c.lda, B, c.ldb)
    torch.cuda.synchronize()
    out = B.cpu().numpy()
    h.close()
    return out


def check_trsm(c, got):
    Xref = oracle.trsm(c.layout, c.side, c.uplo, c.trans, c.diag, c.m, c.n, c.alpha, c.A, c.lda,
                       c.B, c.ldb)
    # B's ld padding untouched
    mask = np.zeros(c.B.size, bool)
    if c.layout == COL:
        mask[: c.ldb * c.n].reshape(c.n, c.ldb)[:, : c.m] = True
    else:
        mask[: c.ldb * c.m].reshape(c.m, c.ldb)[:, : c.n] = True
    assert np.array_equal(got[~mask], c.B[~mask], equal_nan=True), "B padding was modified"
    X = synth.op_view(got, c.layout, "N", c.m, c.n, c.ldb).astype(np.float64)
    R = synth.op_view(Xref, c.layout, "N", c.m, c.n, c.ldb)
    assert np.isfinite(X).all(), "non-finite result"
    ka = c.m if c.side == "L" else c.n
    u = U[c.dtype]
    err = float(np.abs(X - R).max())
    assert err <= 16 * ka * u * float(np.abs(R).max()), f"forward error {err:.3e}"
    opT = c.T.T if c.trans == "T" else c.T
    B0 = synth.op_view(c.B, c.layout, "N", c.m, c.n, c.ldb).astype(np.float64)
    lhs = opT @ X if c.side == "L" else X @ opT
    absl = np.abs(opT) @ np.abs(X) if c.side == "L" else np.abs(X) @ np.abs(opT)
    res = float(np.abs(lhs - c.alpha * B0).max())
    scale = float((absl + np.abs(c.alpha * B0)).max())
    assert res <= 8 * ka * u * scale, f"residual {res:.3e}"


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,side,uplo,trans,diag", CASES)
def test_trsm_matches_oracle_all_policies_same_bits(F, dtype, layout, side, uplo, trans, diag):
    """k = 300 or 200: three levels of blocking with ragged blocks."""
    say(dtype.__name__, layout, side, uplo, trans, diag)
    c = trsm_case(layout, side, uplo, trans, diag, 300, 200, dtype,
                  seed=CASES.index((layout, side, uplo, trans, diag)) + 900)
    ref = run_trsm(F, c, F.FIP_PACK_NONE)
    check_trsm(c, ref)
    for pol in (F.FIP_PACK_AUTO, F.FIP_PACK_ALL):
        out = run_trsm(F, c, pol)
        assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), pol


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_trsm_small_and_special(F, dtype):
    import torch
    # a single diagonal block, and sizes just above one
    for m, n in [(1, 1), (7, 3), (64, 5), (65, 9), (129, 70)]:
        for side in "LR":
            c = trsm_case(COL, side, "U", "N", "N", m, n, dtype, seed=m * 7 + n)
            check_trsm(c, run_trsm(F, c))
    # alpha = 0: B := 0, A and B not read
    c = trsm_case(COL, "L", "L", "N", "N", 100, 40, dtype, seed=2, alpha=0.0)
    c.A[:] = np.nan
    mask = np.isfinite(c.B)
    c.B[mask] = np.nan
    out = run_trsm(F, c)
    v = synth.op_view(out, COL, "N", 100, 40, c.ldb)
    assert np.array_equal(v, np.zeros((100, 40)))
    # m = 0 or n = 0: nothing happens
    h = F.Handle()
    fn = F.fip_dtrsm if dtype == F64 else F.fip_strsm
    assert fn(h.h, COL, "L", "L", "N", "N", 0, 5, 1.0, 0, 1, 0, 1) == 0
    assert fn(h.h, COL, "L", "L", "N", "X", 4, 5, 1.0, 0, 4, 0, 4) == 6
    assert fn(h.h, COL, "R", "L", "N", "N", 4, 5, 1.0, 1, 4, 1, 4) == 11   # lda < n
    h.close()
    torch.cuda.synchronize()


def test_trsm_large(F):
    """m = 2048, n = 512 (five levels of blocking, GEMM updates of up to 1024 x 512 x 1024)."""
    for side, uplo, trans in [("L", "L", "N"), ("R", "U", "T")]:
        m, n = (2048, 512) if side == "L" else (512, 2048)
        c = trsm_case(COL, side, uplo, trans, "N", m, n, F64, seed=77)
        say("large", side, uplo, trans)
        check_trsm(c, run_trsm(F, c))
