"""GPU parity of SYRK and TRMM through the fused-pack tile kernel, against the oracle.

SYRK: the uplo triangle within 4 k u max D of the oracle, the other triangle and C's padding
untouched bit for bit; every packing policy gives the same bits; with packing forced, every
panel is claimed once (both operand roles share the one pack) and holds the oracle's packed
bytes of op(A).  TRMM: every layout / side / uplo / transpose / diagonal combination within the
bound, NaN in the entries it must not read (the other triangle, a unit diagonal) never reaching C;
the triangular operand's packed chunks equal the oracle's pack of op(T) with the triangle applied.
At the benchmark's sizes: exact oracle values on sampled entries plus a Freivalds probe.
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


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print("[l3]", *a, flush=True)
    sys.stdout.flush()


def fill(layout, rows, cols, ld, values, dtype, pad=np.nan):
    return synth.fill_stored(layout, rows, cols, ld, values, dtype, pad)


def view(buf, layout, rows, cols, ld):
    return synth.op_view(buf, layout, "N", rows, cols, ld)


def tri_mask(n, lower):
    return np.tril(np.ones((n, n), bool)) if lower else np.triu(np.ones((n, n), bool))


# ------------------------------------------------------------------------------ SYRK

def syrk_case(layout, uplo, trans, n, k, dtype, seed, pad=3, alpha=1.5, beta=0.5):
    g = synth.rng(seed)
    sr, sc = (k, n) if trans == "T" else (n, k)
    lda = synth.min_ld(layout, sr, sc) + pad
    A = fill(layout, sr, sc, lda, g.uniform(-1, 1, (sr, sc)), dtype)
    ldc = n + pad
    C = fill(layout, n, n, ldc, g.uniform(-1, 1, (n, n)), dtype)
    return dict(layout=layout, uplo=uplo, trans=trans, n=n, k=k, A=A, lda=lda, C=C, ldc=ldc,
                alpha=alpha, beta=beta, dtype=dtype)


def run_syrk(F, c, policy, tile=-1, copies=-1):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    A, C = to_dev(c["A"]), to_dev(c["C"])
    h.syrk(c["layout"], c["uplo"], c["trans"], c["n"], c["k"], c["alpha"], A, c["lda"],
           c["beta"], C, c["ldc"])
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def check_syrk(c, got):
    ref, D = oracle.syrk(c["layout"], c["uplo"], c["trans"], c["n"], c["k"], c["alpha"], c["A"],
                         c["lda"], c["beta"], c["C"], c["ldc"])
    n, ldc, layout = c["n"], c["ldc"], c["layout"]
    mask = tri_mask(n, c["uplo"] == "L")
    inside = np.zeros(c["C"].size, bool)
    view(inside, layout, n, n, ldc)[mask] = True
    # the other triangle and the padding keep their bits
    assert got[~inside].tobytes() == c["C"][~inside].tobytes(), "other triangle or padding"
    g, r, d = got[inside].astype(np.float64), ref[inside], D[inside]
    err = float(np.abs(g - r).max())
    bound = 4 * max(c["k"], 1) * U[c["dtype"]] * float(d.max())
    assert err <= bound, (err, bound)
    return err / bound if bound else 0.0


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,uplo,trans", list(itertools.product([COL, ROW], "LU", "NT")))
def test_syrk_matches_oracle_all_policies_same_bits(F, dtype, layout, uplo, trans):
    c = syrk_case(layout, uplo, trans, 300, 170, dtype, seed=5 + layout * 4 + (uplo == "U") * 2
                  + (trans == "T"))
    say("syrk", dtype.__name__, layout, uplo, trans)
    ref, _ = run_syrk(F, c, F.FIP_PACK_NONE)
    check_syrk(c, ref)
    for pol in (F.FIP_PACK_ALL, F.FIP_PACK_AUTO):
        out, _ = run_syrk(F, c, pol)
        assert np.array_equal(out.tobytes(), ref.tobytes()), pol


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("copies", [1, 8], ids=["shared", "per-xcd"])
def test_syrk_shared_pack_bytes_and_reuse(F, dtype, copies):
    """32 x 32 tiles, a ragged n: 64 tile rows, 2080 tiles of the triangle (several rounds).
    With packing forced every panel of op(A) is claimed and packed once per copy for both
    operand roles and equals the oracle's pack; AUTO packs the fringe panel only."""
    n, k = 64 * 32 - 3, 200
    c = syrk_case(COL, "L", "T", n, k, dtype, seed=17, pad=5)
    say("syrk pack", dtype.__name__, copies)
    ref, _ = run_syrk(F, c, F.FIP_PACK_NONE, tile=2)
    out, h = run_syrk(F, c, F.FIP_PACK_ALL, tile=2, copies=copies)
    assert np.array_equal(out.tobytes(), ref.tobytes())
    check_syrk(c, out)
    p = h.last_plan()
    assert p.pack_a and p.pack_b and p.a_pack_offset == p.b_pack_offset
    ws, epoch = h.workspace, np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    nt = p.tiles_m
    refpack = oracle.pack(c["A"], 0, COL, "T", n, k, c["lda"], p.MT, p.KT).view(np.uint8)
    assert refpack.size == p.a_copy_bytes
    claims = ws[p.a_claim_offset: p.a_claim_offset + 8 * p.copies * nt].cpu().numpy()
    claims = claims.view(np.uint64).reshape(p.copies, nt)
    flags = ws[p.a_flag_offset: p.a_flag_offset + 8 * p.copies * nt].cpu().numpy()
    flags = flags.view(np.uint64).reshape(p.copies, nt)
    assert np.all((claims == epoch).any(axis=0))
    panel = refpack.size // nt
    for cp in range(p.copies):
        buf = ws[p.a_pack_offset + cp * p.a_copy_bytes:
                 p.a_pack_offset + (cp + 1) * p.a_copy_bytes].cpu().numpy()
        for t in range(nt):
            if claims[cp, t] == epoch:
                assert flags[cp, t] == epoch
                assert np.array_equal(buf[t * panel:(t + 1) * panel],
                                      refpack[t * panel:(t + 1) * panel]), (cp, t)
    out, h = run_syrk(F, c, F.FIP_PACK_AUTO, tile=2)
    p = h.last_plan()
    assert p.pack_a and p.a_pack_first == p.tiles_m - 1
    assert np.array_equal(out.tobytes(), ref.tobytes())


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_syrk_special_cases(F, dtype):
    import torch
    say("syrk special", dtype.__name__)
    # beta = 0: the triangle of C is not read (NaN there); alpha = 0: A is not read
    c = syrk_case(COL, "U", "N", 150, 40, dtype, seed=23, beta=0.0)
    n, ldc = c["n"], c["ldc"]
    view(c["C"], COL, n, n, ldc)[tri_mask(n, False)] = np.nan
    got, _ = run_syrk(F, c, F.FIP_PACK_ALL)
    c_check = dict(c)
    c_check["C"] = c["C"].copy()
    view(c_check["C"], COL, n, n, ldc)[tri_mask(n, False)] = 0.0   # never read either way
    sel = np.zeros(c["C"].size, bool)
    view(sel, COL, n, n, ldc)[tri_mask(n, False)] = True
    check_syrk(c_check, np.where(sel, got, c_check["C"]).astype(dtype))
    assert np.all(np.isfinite(got[sel]))
    c = syrk_case(ROW, "L", "T", 90, 30, dtype, seed=24, alpha=0.0, beta=-2.0)
    c["A"][:] = np.nan
    got, _ = run_syrk(F, c, F.FIP_PACK_ALL)
    check_syrk(c, got)
    c = syrk_case(COL, "L", "N", 70, 0, dtype, seed=25)
    got, _ = run_syrk(F, c, F.FIP_PACK_AUTO)
    check_syrk(c, got)
    # argument errors by position, before anything runs
    h = F.Handle()
    A = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert F.fip_dsyrk(h.h, 0, "X", "N", 4, 4, 1.0, A, 4, 0.0, A, 4) == 3
    assert F.fip_dsyrk(h.h, 0, "L", "Q", 4, 4, 1.0, A, 4, 0.0, A, 4) == 4
    assert F.fip_dsyrk(h.h, 0, "L", "T", 4, 5, 1.0, A, 4, 0.0, A, 4) == 9
    assert F.fip_dsyrk(h.h, 0, "L", "N", 4, 4, 1.0, A, 4, 0.0, A, 3) == 12


def test_syrk_large_sampled(F):
    """n = 8192, k = 8192, FP64, column-major lower 'N' (the benchmark's configuration):
    sampled triangle entries against the oracle and a Freivalds probe of the symmetric
    product restricted to the triangle's rows."""
    n = k = 8192
    c = syrk_case(COL, "L", "N", n, k, F64, seed=synth.BASE_SEED + 31, pad=0)
    say("syrk 8192")
    got, _ = run_syrk(F, c, F.FIP_PACK_AUTO)
    rows, cols = synth.sample_entries(n, n, 2048, 3)
    keep = rows >= cols
    rows, cols = rows[keep], cols[keep]
    ref, d = oracle.gemm_entries(COL, n, n, k, 1.5, c["A"], c["lda"], "N", c["A"], c["lda"], "T",
                                 0.5, c["C"], c["ldc"], rows, cols)
    Cv = view(got, COL, n, n, c["ldc"])
    err = float(np.abs(Cv[rows, cols] - ref).max())
    assert err <= 4 * k * U[F64] * float(d.max()), err
    # the upper triangle keeps its bits
    up = np.triu_indices(n, 1)
    assert np.array_equal(Cv[up[0][::997], up[1][::997]],
                          view(c["C"], COL, n, n, c["ldc"])[up[0][::997], up[1][::997]])


# ------------------------------------------------------------------------------ TRMM

def trmm_case(layout, side, uplo, trans, diag, m, n, dtype, seed, alpha=1.5, beta=0.5, pad=2):
    g = synth.rng(seed)
    ka = m if side == "L" else n
    Av = g.uniform(-1, 1, (ka, ka))
    notref = ~tri_mask(ka, uplo == "L")
    if diag == "U":
        notref |= np.eye(ka, dtype=bool)
    Av[notref] = np.nan      # never read
    lda = ka + pad
    A = fill(layout, ka, ka, lda, Av, dtype)
    ldb = (m if layout == COL else n) + pad
    B = fill(layout, m, n, ldb, g.uniform(-1, 1, (m, n)), dtype)
    C = fill(layout, m, n, ldb, g.uniform(-1, 1, (m, n)), dtype)
    return dict(layout=layout, side=side, uplo=uplo, trans=trans, diag=diag, m=m, n=n, ka=ka,
                A=A, lda=lda, B=B, ldb=ldb, C=C, ldc=ldb, alpha=alpha, beta=beta, dtype=dtype)


def run_trmm(F, c, policy, tile=-1):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    A, B, C = to_dev(c["A"]), to_dev(c["B"]), to_dev(c["C"])
    h.trmm(c["layout"], c["side"], c["uplo"], c["trans"], c["diag"], c["m"], c["n"], c["alpha"],
           A, c["lda"], B, c["ldb"], c["beta"], C, c["ldc"])
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def check_trmm(c, got):
    ref, D = oracle.trmm(c["layout"], c["side"], c["uplo"], c["trans"], c["diag"], c["m"], c["n"],
                         c["alpha"], c["A"], c["lda"], c["B"], c["ldb"], c["beta"], c["C"],
                         c["ldc"])
    inside = np.zeros(c["C"].size, bool)
    view(inside, c["layout"], c["m"], c["n"], c["ldc"])[:, :] = True
    assert got[~inside].tobytes() == c["C"][~inside].tobytes(), "C padding modified"
    g, r, d = got[inside].astype(np.float64), ref[inside], D[inside]
    assert np.all(np.isfinite(g)), "a non-referenced entry of A reached C"
    err = float(np.abs(g - r).max())
    bound = 4 * c["ka"] * U[c["dtype"]] * float(d.max())
    assert err <= bound, (err, bound)


TRMM_CASES = list(itertools.product([COL, ROW], "LR", "LU", "NT", "NU"))


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,side,uplo,trans,diag", TRMM_CASES)
def test_trmm_matches_oracle_all_policies_same_bits(F, dtype, layout, side, uplo, trans, diag):
    c = trmm_case(layout, side, uplo, trans, diag, 300, 200, dtype,
                  seed=TRMM_CASES.index((layout, side, uplo, trans, diag)) + 500)
    say("trmm", dtype.__name__, layout, side, uplo, trans, diag)
    ref, _ = run_trmm(F, c, F.FIP_PACK_NONE)
    check_trmm(c, ref)
    out, _ = run_trmm(F, c, F.FIP_PACK_ALL)
    assert np.array_equal(out.tobytes(), ref.tobytes())


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("side,uplo,trans,diag", [("L", "L", "N", "N"), ("L", "U", "T", "U"),
                                                  ("R", "U", "N", "N"), ("R", "L", "T", "U")])
def test_trmm_pack_holds_the_triangle(F, dtype, side, uplo, trans, diag):
    """Packing forced, several rounds of 32 x 32 tiles: the triangular operand's panels are
    packed with the triangle applied (zeros, unit diagonal), equal to the oracle's pack of the
    masked operand on every k-step the panel's tiles compute; C equals the unpacked run's."""
    m, n = 64 * 32 - 3, 48 * 32 + 5
    c = trmm_case(COL, side, uplo, trans, diag, m, n, dtype, seed=41)
    say("trmm pack", dtype.__name__, side, uplo, trans, diag)
    ref, _ = run_trmm(F, c, F.FIP_PACK_NONE, tile=2)
    out, h = run_trmm(F, c, F.FIP_PACK_ALL, tile=2)
    assert np.array_equal(out.tobytes(), ref.tobytes())
    check_trmm(c, out)
    p = h.last_plan()
    assert p.pack_a and not (p.b_copy_bytes > 0)
    ka = c["ka"]
    # the masked triangular matrix, built with NumPy (zeros outside, ones on a unit diagonal)
    Tm = view(c["A"], COL, ka, ka, c["lda"]).astype(np.float64).copy()
    keep = tri_mask(ka, uplo == "L")
    Tm[~keep] = 0.0
    if diag == "U":
        np.fill_diagonal(Tm, 1.0)
    Tbuf = fill(COL, ka, ka, c["lda"], Tm, dtype)
    # kernel side of T: side L -> A side (MN = rows of op(T)); side R -> B side (MN = columns)
    refpack = oracle.pack(Tbuf, 0 if side == "L" else 1, COL, trans, ka, ka, c["lda"], p.MT,
                          p.KT).view(np.uint8)
    assert refpack.size == p.a_copy_bytes
    ws, epoch = h.workspace, np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    nt = -(-ka // p.MT)
    nk = p.ksteps
    chunk = refpack.size // (nt * nk)
    claims = ws[p.a_claim_offset: p.a_claim_offset + 8 * p.copies * nt].cpu().numpy()
    claims = claims.view(np.uint64).reshape(p.copies, nt)
    keep_ge = (uplo == "L") != (trans == "T")
    if side == "R":
        keep_ge = not keep_ge
    for cp in range(p.copies):
        buf = ws[p.a_pack_offset + cp * p.a_copy_bytes:
                 p.a_pack_offset + (cp + 1) * p.a_copy_bytes].cpu().numpy()
        for t in range(nt):
            if claims[cp, t] != epoch:
                continue
            x0 = t * p.MT
            q0, q1 = (0, min(nk, -(-(x0 + p.MT) // p.KT))) if keep_ge else (x0 // p.KT, nk)
            lo, hi = (t * nk + q0) * chunk, (t * nk + q1) * chunk
            assert np.array_equal(buf[lo:hi], refpack[lo:hi]), (cp, t)


def test_trmm_large_sampled(F):
    """4096 x 4096, side L, lower, no transpose, FP64: sampled entries against the oracle's
    GEMM on the NumPy-masked triangle (a second route to the same sums) and a Freivalds probe."""
    m = n = 4096
    c = trmm_case(COL, "L", "L", "N", "N", m, n, F64, seed=synth.BASE_SEED + 37, pad=0)
    say("trmm 4096")
    got, _ = run_trmm(F, c, F.FIP_PACK_AUTO)
    Tm = view(c["A"], COL, m, m, c["lda"]).copy()
    Tm[~tri_mask(m, True)] = 0.0
    Tbuf = fill(COL, m, m, m, Tm, F64)
    rows, cols = synth.sample_entries(m, n, 2048, 4)
    ref, d = oracle.gemm_entries(COL, m, n, m, 1.5, Tbuf, m, "N", c["B"], c["ldb"], "N", 0.5,
                                 c["C"], c["ldc"], rows, cols)
    Cv = view(got, COL, m, n, c["ldc"])
    err = float(np.abs(Cv[rows, cols] - ref).max())
    assert err <= 4 * m * U[F64] * float(d.max()), err
    x = synth.rng(5).choice([-1.0, 1.0], size=n)
    y, bnd = oracle.freivalds(COL, m, n, m, 1.5, Tbuf, m, "N", c["B"], c["ldb"], "N", 0.5, c["C"],
                              c["ldc"], x)
    slack = 2.0 * (n + m + 4) * 2.0 ** -53
    assert np.all(np.abs(Cv @ x - y) <= (4 * m * U[F64] + slack) * bnd + 1e-300)
