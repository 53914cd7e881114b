"""GPU parity of the complex GEMM (fip_zgemm / fip_cgemm, the 1m method) against the oracle.

The library runs complex products through its real tile kernel on the 1m expansions of the
operands (paper Sec. 5: arithmetic encoded in the packing).  Checked here, through the C-ABI:
  - element-by-element parity with oracle.zgemm on shapes spanning several tiles with ragged
    tails, every op pair in {N, T, C}, both layouts, padded leading dimensions;
  - bitwise identity of fused (AUTO, ALL), unpacked (NONE) and pack-then-compute
    (fip_pack + CONSUME_ONLY) results;
  - packed panels equal, byte for byte, the oracle's pack of the 1m expansions;
  - the BLAS quick-return rules, NaN propagation, and a large sampled case.

Tolerance: every real component satisfies |C - Cref| <= 4 * max(2k, 1) * u * max D, where D is
the oracle's bound with |z|_1 = |re| + |im| (each component of a complex dot product of length
k is a real dot product of length 2k whose |terms| sum to at most D).
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

pytestmark = pytest.mark.gpu

C128, C64 = np.complex128, np.complex64
U = {C128: 2.0 ** -53, C64: 2.0 ** -24}
TRANS = ["N", "T", "C"]


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(buf):
    import torch
    return torch.from_numpy(np.ascontiguousarray(buf)).to("cuda")


def run(F, c, policy=0, copies=-1, tile=-1, no_publish=0):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    h.set_attr(F.FIP_ATTR_NO_PUBLISH, no_publish)
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB)
    h.zgemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
            c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def c_mask(c):
    mask = np.zeros(c.C.size, dtype=bool)
    if c.m and c.n:
        if c.layout == COL:
            mask[: c.ldc * c.n].reshape(c.n, c.ldc)[:, : c.m] = True
        else:
            mask[: c.ldc * c.m].reshape(c.m, c.ldc)[:, : c.n] = True
    return mask


def bits(z):
    return np.ascontiguousarray(z).view(np.uint8)


def check_full(c, got):
    Cref, D = oracle.zgemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                           c.transB, c.beta, c.C, c.ldc)
    mask = c_mask(c)
    assert np.array_equal(bits(got[~mask]), bits(c.C[~mask])), "C padding was modified"
    if not mask.any():
        return 0.0
    g = got[mask].astype(np.complex128)
    r = Cref[mask]
    assert np.isfinite(g.view(np.float64)).all(), "non-finite result"
    err = max(float(np.abs(g.real - r.real).max()), float(np.abs(g.imag - r.imag).max()))
    kk = max(2 * c.k, 1)
    dmax = float(D[mask].max())
    bound = 4 * kk * U[c.dtype] * dmax
    assert err <= bound, f"max err {err:.3e} > bound {bound:.3e}"
    return err / (kk * U[c.dtype] * dmax) if dmax > 0 else 0.0


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", list(itertools.product(TRANS, TRANS)))
def test_parity_all_ops(F, dtype, layout, tA, tB):
    """Several tiles of the expanded problem with ragged tails in m, n and k."""
    say("cx parity", dtype.__name__, layout, tA, tB)
    c = synth.make_cx_case(layout, 133, 301, 77, tA, tB, ld_pad=7 if tA != "N" else 0,
                           dtype=dtype, seed=100 * layout + 10 * TRANS.index(tA) + TRANS.index(tB))
    got, _ = run(F, c)
    check_full(c, got)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "C", "T"), (ROW, "N", "C"),
                                          (ROW, "T", "T")])
def test_modes_bitwise_identical(F, dtype, layout, tA, tB):
    """Fused (AUTO, ALL shared copy, ALL per-XCD copies, ALL without publishing), unpacked and
    pack-then-compute all run the same kernel and k order: C agrees bit for bit."""
    say("cx modes", dtype.__name__, layout, tA, tB)
    c = synth.make_cx_case(layout, 357, 290, 211, tA, tB, ld_pad=5, dtype=dtype, seed=44)
    ref, _ = run(F, c, F.FIP_PACK_NONE)
    check_full(c, ref)
    for pol, copies, nopub in [(F.FIP_PACK_AUTO, -1, 0), (F.FIP_PACK_ALL, 1, 0),
                               (F.FIP_PACK_ALL, 8, 0), (F.FIP_PACK_ALL, 1, 1),
                               (F.FIP_PACK_CONSUME_ONLY, -1, 0)]:
        out, _ = run(F, c, pol, copies=copies, no_publish=nopub)
        assert np.array_equal(bits(out), bits(ref)), (pol, copies, nopub)


def _ws(ws, off, nbytes):
    return ws[off: off + nbytes].cpu().numpy()


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "C", "N"), (ROW, "T", "C"),
                                          (ROW, "N", "N")])
def test_packed_panels_are_the_1m_expansions(F, dtype, layout, tA, tB):
    """Every packed panel (PACK_POLICY ALL, one shared copy) equals the oracle's pack of the
    1m expansion of that operand, byte for byte (zero padding and -0.0 included)."""
    say("cx pack bits", dtype.__name__, layout, tA, tB)
    m, n, k = 150, 97, 45
    c = synth.make_cx_case(layout, m, n, k, tA, tB, ld_pad=3, dtype=dtype, seed=61)
    got, h = run(F, c, F.FIP_PACK_ALL, copies=1)
    check_full(c, got)
    p = h.last_plan()
    assert p.pack_a and p.pack_b and p.copies == 1
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    real = np.float64 if dtype == C128 else np.float32
    # Kernel sides: column-major C runs op(A) (1e expansion) times op(B) (1r); row-major C
    # runs C^T = op(B)^T op(A)^T, so op(B)^T takes the 1e expansion and op(A)^T the 1r one.
    # A row-major buffer read column-major is the transpose, and op(X)^T of the row-major X
    # is op(X) (same trans) of that column-major view.
    swapped = layout == ROW
    for which, X, ld, t, mn, off, nbytes, claim_off, tiles, mnt in [
            ("A", c.A, c.lda, tA, m, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.tiles_m, p.MT),
            ("B", c.B, c.ldb, tB, n, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.tiles_n, p.NT)]:
        kernel_b = (which == "B") != swapped
        ref = oracle.pack_1m(X, kernel_b, COL if swapped else layout, t, mn, k, ld, mnt, p.KT,
                             dtype=real)
        claims = _ws(h.workspace, claim_off, 8 * tiles).view(np.uint64)
        assert np.all(claims == epoch), f"{which}: a panel was not packed"
        buf = _ws(h.workspace, off, nbytes)
        assert buf.size == ref.nbytes, (which, buf.size, ref.nbytes)
        assert np.array_equal(buf, ref.view(np.uint8)), f"{which} pack differs"


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
def test_quick_returns_and_specials(F, dtype):
    import torch
    say("cx specials", dtype.__name__)
    nan = complex(np.nan, np.nan)
    # alpha = 0: A and B (NaN) are not read; C := beta C
    c = synth.make_cx_case(COL, 70, 40, 30, "N", "C", alpha=0, beta=0.5 - 2j, dtype=dtype, seed=3)
    c.A[:] = nan
    c.B[:] = nan
    got, _ = run(F, c)
    check_full(c, got)
    # beta = 0: C (NaN) is not read
    c = synth.make_cx_case(ROW, 70, 40, 30, "T", "N", beta=0, dtype=dtype, seed=4)
    c.C[c_mask(c)] = nan
    got, _ = run(F, c)
    check_full(c, got)
    # k = 0: C := beta C
    c = synth.make_cx_case(COL, 33, 65, 0, "N", "N", beta=1j, dtype=dtype, seed=5)
    got, _ = run(F, c)
    check_full(c, got)
    # beta = 1 with alpha = 0: nothing happens, C untouched bit for bit
    c = synth.make_cx_case(COL, 33, 65, 9, "N", "N", alpha=0, beta=1, dtype=dtype, seed=6)
    got, _ = run(F, c)
    assert np.array_equal(bits(got), bits(c.C))
    # NaN in one element of op(A) and of op(B): exactly row i and column j are non-finite
    c = synth.make_cx_case(COL, 90, 70, 50, "N", "N", dtype=dtype, seed=7)
    c.A[12 + 3 * c.lda] = complex(0.25, np.nan)
    c.B[40 + 9 * c.ldb] = complex(np.nan, 0.0)
    got, _ = run(F, c)
    cv = synth.op_view(got, COL, "N", c.m, c.n, c.ldc)
    bad = ~np.isfinite(np.ascontiguousarray(cv).view(real_of(dtype)).reshape(c.m, c.n, 2)).all(axis=2)
    want = np.zeros((c.m, c.n), bool)
    want[12, :] = True
    want[:, 9] = True
    assert np.array_equal(bad, want)
    torch.cuda.synchronize()


def real_of(dtype):
    return np.float64 if dtype == C128 else np.float32


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
def test_invalid_arguments(F, dtype):
    """Positions of invalid arguments (checked before any HIP call)."""
    h = F.Handle()
    fn = F.fip_zgemm if dtype == C128 else F.fip_cgemm
    assert fn(h.h, 2, 4, 4, 4, 1, 0, 4, "N", 0, 4, "N", 0, 0, 4) == 2
    assert fn(h.h, 0, -1, 4, 4, 1, 0, 4, "N", 0, 4, "N", 0, 0, 4) == 3
    assert fn(h.h, 0, 4, 4, 4, 1, 0, 3, "N", 0, 4, "N", 0, 0, 4) == 7   # A null (read)
    assert fn(h.h, 0, 4, 4, 4, 1, 1, 3, "N", 1, 4, "N", 0, 1, 4) == 8   # lda < m
    assert fn(h.h, 0, 4, 4, 4, 1, 1, 4, "X", 1, 4, "N", 0, 1, 4) == 9
    assert fn(h.h, 0, 4, 4, 4, 1, 1, 4, "N", 1, 4, "Q", 0, 1, 4) == 12
    assert fn(h.h, 0, 4, 4, 4, 1, 1, 4, "N", 1, 4, "N", 0, 1, 3) == 15
    h.close()


@pytest.mark.parametrize("dtype", [C128, C64], ids=["z", "c"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (ROW, "C", "T")])
def test_large_sampled(F, dtype, layout, tA, tB):
    """m = n = 2048, k = 1024 (several rounds of tiles, so AUTO's reuse rule is exercised):
    exact oracle values on sampled entries, corners and fringes included."""
    say("cx large", dtype.__name__, layout, tA, tB)
    c = synth.make_cx_case(layout, 2048, 2048, 1024, tA, tB, dtype=dtype, seed=8)
    got, _ = run(F, c)
    rows, cols = synth.sample_entries(c.m, c.n, 2048, 9)
    ref, d = oracle.zgemm_entries(c.layout, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                                  c.transB, c.beta, c.C, c.ldc, rows, cols)
    cv = synth.op_view(got, c.layout, "N", c.m, c.n, c.ldc)[rows, cols].astype(np.complex128)
    err = max(float(np.abs(cv.real - ref.real).max()), float(np.abs(cv.imag - ref.imag).max()))
    assert err <= 4 * 2 * c.k * U[dtype] * float(d.max()), err
