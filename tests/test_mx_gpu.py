"""GPU parity of the mixed-precision forms (bfloat16, FP8 E4M3 with scales, 3- and 2-term
bfloat16 splits of binary32) through the C-ABI, against the oracle.

Bar: max|C - Cref| <= 4 k 2^-24 max D (+ 2^-8 max|Cref| for a bfloat16 C), Cref the binary64
product of the values the stored operands stand for; packed buffers byte-exact against the
oracle's reference pack; C bitwise identical across packing policies.
"""
import numpy as np
import pytest

import oracle
from gemm_util import c_mask, check_mx, mx_reference_sampled, to_dev
from paper_2302_08417_amd import synth

pytestmark = pytest.mark.gpu

FORMS = [synth.FORM_BF16, synth.FORM_E4M3, synth.FORM_BF16X3, synth.FORM_BF16X3_FAST]
FORM_IDS = ["bf16", "e4m3", "bf16x3", "bf16x3f"]
COL, ROW = synth.COL, synth.ROW
BIG = [(synth.FORM_BF16, 256), (synth.FORM_E4M3, 256)]   # forms with 256 x 256 tiles
BIG_IDS = ["bf16-256", "e4m3-256"]


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print("[mx]", *a, flush=True)


def dev(buf):
    return to_dev(buf)


def run_mx(F, c, policy=0, order=0, no_publish=0, h=None, stats=0, tile=-1, copies=-1):
    import torch
    own = h is None
    if own:
        h = F.Handle(policy=policy)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    h.set_attr(F.FIP_ATTR_MX_TILE, tile)
    h.set_attr(F.FIP_ATTR_ORDER, order)
    h.set_attr(F.FIP_ATTR_NO_PUBLISH, no_publish)
    h.set_attr(F.FIP_ATTR_STATS, stats)
    A, B = dev(c.A), dev(c.B)
    C = dev(c.C)
    if c.c_bf16:
        C = C.view(torch.bfloat16)
    sa = dev(c.a_scale) if c.a_scale is not None else None
    sb = dev(c.b_scale) if c.b_scale is not None else None
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB, dtype=c.form)
    h.gemm_mx(c.form, c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB,
              c.beta, C, c.ldc, sa, sb)
    torch.cuda.synchronize()
    out = (C.view(torch.int16) if c.c_bf16 else C).cpu().numpy()
    out = out.view(np.uint16) if c.c_bf16 else out
    return out, h


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "T", "N"), (ROW, "N", "T"),
                                          (ROW, "T", "T"), (COL, "N", "T"), (ROW, "N", "N")])
@pytest.mark.parametrize("c_bf16", [False, True], ids=["c32", "c16"])
def test_mx_matches_oracle(F, form, layout, tA, tB, c_bf16):
    """Several tiles and ragged tails in m, n and k (k not a multiple of the k-step)."""
    say("oracle", form, layout, tA, tB, c_bf16)
    c = synth.make_mx_case(form, layout, 300, 200, 333, tA, tB, ld_pad=4, alpha=1.5, beta=0.5,
                           seed=form * 31 + layout * 7 + (tA == "T") * 3 + (tB == "T"),
                           c_bf16=c_bf16)
    out, _ = run_mx(F, c, F.FIP_PACK_ALL)
    nerr, truth = check_mx(c, out)
    say(f"normalised error {nerr:.3e}; error vs binary64 product of the binary32 inputs "
        f"{truth:.3e} of max D")


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("pad", [1, 7])
def test_mx_unaligned_leading_dims(F, form, pad):
    """Odd leading dimensions make the unpacked operands unaligned for vector loads; the
    element loader must give the same result."""
    say("unaligned", form, pad)
    c = synth.make_mx_case(form, COL, 150, 140, 200, "T", "N", ld_pad=pad, alpha=1.0, beta=1.0,
                           seed=5 + pad)
    out, _ = run_mx(F, c, F.FIP_PACK_ALL)
    check_mx(c, out)


@pytest.mark.parametrize("form,tile", [(f, -1) for f in FORMS] + [(synth.FORM_E4M3, 256)],
                         ids=FORM_IDS + ["e4m3-256"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (ROW, "N", "T")])
def test_mx_modes_bitwise(F, form, tile, layout, tA, tB):
    """AUTO / ALL / NONE / CONSUME_ONLY / other tile order / no publishing run the same tile
    arithmetic in the same k order: C must agree bit for bit.  The launch has more tiles than
    fit on the GPU at once, so later tiles do read packed panels."""
    say("modes", form, tile, layout, tA, tB)
    # several rounds of tiles: 256 x 256 tiles (bfloat16, E4M3) need 8192^2
    m = n = 8192 if form in (synth.FORM_BF16, synth.FORM_E4M3) else 4096
    k = 160 if form != synth.FORM_E4M3 else 300
    c = synth.make_mx_case(form, layout, m, n, k, tA, tB, alpha=1.0, beta=0.5, seed=77 + form)
    ref, h0 = run_mx(F, c, F.FIP_PACK_NONE, tile=tile)
    if tile == 256:
        assert h0.last_plan().MT == 256
    total_packed = 0
    for pol, order, nopub in [(F.FIP_PACK_AUTO, 0, 0), (F.FIP_PACK_ALL, 0, 0),
                              (F.FIP_PACK_ALL, 1, 0), (F.FIP_PACK_ALL, 0, 1),
                              (F.FIP_PACK_CONSUME_ONLY, 0, 0)]:
        out, h = run_mx(F, c, pol, order=order, no_publish=nopub, stats=1, tile=tile,
                        copies=8 if order == 1 else -1)
        if pol == F.FIP_PACK_ALL and not nopub:
            p = h.last_plan()
            st = h.workspace[p.stats_offset: p.stats_offset + 32].cpu().numpy().view(np.uint64)
            total_packed += int(st[1])
        assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), (pol, order, nopub)
    say("packed-chunk reads", total_packed)
    assert total_packed > 0
    # and the common result is right: sampled check against the oracle
    rows, cols = synth.sample_entries(m, n, 512, 3)
    Cref, D, _ = mx_reference_sampled(c, rows, cols)
    got = synth.op_view(ref, c.layout, "N", m, n, c.ldc)[rows, cols].astype(np.float64)
    assert np.abs(got - Cref).max() <= 4 * k * 2.0 ** -24 * D.max()


@pytest.mark.parametrize("form,tile", BIG, ids=BIG_IDS)
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "T", "N"), (ROW, "N", "T"),
                                          (ROW, "T", "T")])
@pytest.mark.parametrize("c_bf16", [False, True], ids=["c32", "c16"])
def test_mx_big_tile_matches_oracle(F, form, tile, layout, tA, tB, c_bf16):
    """256 x 256 tiles (128 x 128 per wave): several tiles, ragged m, n and k."""
    say("big tile", form, layout, tA, tB, c_bf16)
    c = synth.make_mx_case(form, layout, 600, 520, 333, tA, tB, ld_pad=4, alpha=1.5, beta=0.5,
                           seed=form * 13 + layout * 5 + (tA == "T") * 3 + (tB == "T") + 1000,
                           c_bf16=c_bf16)
    out, h = run_mx(F, c, F.FIP_PACK_ALL, tile=tile)
    assert h.last_plan().MT == 256
    check_mx(c, out)


@pytest.mark.parametrize("form,tile", [(f, 128) for f in FORMS] + BIG,
                         ids=[i + "-128" for i in FORM_IDS] + BIG_IDS)
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "T", "T"), (ROW, "N", "T"),
                                          (ROW, "T", "N")])
@pytest.mark.parametrize("copies", [1, 8], ids=["shared", "per-xcd"])
def test_mx_packed_buffers_bit_exact(F, form, tile, layout, tA, tB, copies):
    """Every claimed and published panel equals the oracle's reference pack byte for byte
    (K-major planes; the split forms hold the bfloat16 terms), with one shared copy or one
    per XCD."""
    say("mx pack bits", form, tile, layout, tA, tB, copies)
    c = synth.make_mx_case(form, layout, 600, 400, 170, tA, tB, ld_pad=4, seed=19 + form)
    out, h = run_mx(F, c, F.FIP_PACK_ALL, tile=tile, copies=copies)
    assert h.last_plan().copies == copies
    check_mx(c, out)
    p = h.last_plan()
    ws = h.workspace
    epoch = h.get_attr(F.FIP_ATTR_EPOCH)
    kt = p.KT
    for which, ntiles, mnt, off_pack, copy_bytes, off_claim, off_flag, X, ld, t, mn, is_b in [
            ("A", p.tiles_m, p.MT, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.a_flag_offset, c.A, c.lda, tA, c.m, 0),
            ("B", p.tiles_n, p.NT, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.b_flag_offset, c.B, c.ldb, tB, c.n, 1)]:
        exp = oracle.pack_mx(form, X, is_b, layout, t, mn, c.k, ld, mnt)
        assert exp.size == copy_bytes
        packs = ws[off_pack: off_pack + p.copies * copy_bytes].cpu().numpy().reshape(p.copies, -1)
        claims = ws[off_claim: off_claim + 8 * p.copies * ntiles].cpu().numpy().view(np.uint64)
        flags = ws[off_flag: off_flag + 8 * p.copies * ntiles].cpu().numpy().view(np.uint64)
        claims = claims.reshape(p.copies, ntiles)
        flags = flags.reshape(p.copies, ntiles)
        panel = exp.size // ntiles
        for tt in range(ntiles):
            owners = [cp for cp in range(p.copies) if claims[cp, tt] == epoch]
            assert owners, f"{which} panel {tt} packed by nobody"
            for cp in owners:
                assert flags[cp, tt] == epoch, f"{which} copy {cp} panel {tt} unpublished"
                got = packs[cp, tt * panel: (tt + 1) * panel]
                assert np.array_equal(got, exp[tt * panel: (tt + 1) * panel]), (which, cp, tt)
    assert kt == oracle.MX_KT[form]


@pytest.mark.parametrize("form,tile", [(f, 128) for f in FORMS] + BIG,
                         ids=[i + "-128" for i in FORM_IDS] + BIG_IDS)
def test_mx_standalone_pack_bit_exact(F, form, tile):
    import torch
    say("standalone mx pack", form, tile)
    c = synth.make_mx_case(form, ROW, 560, 300, 150, "T", "N", ld_pad=4, seed=23 + form)
    h = F.Handle(policy=F.FIP_PACK_CONSUME_ONLY)
    h.set_attr(F.FIP_ATTR_MX_TILE, tile)
    A, B = dev(c.A), dev(c.B)
    h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB, dtype=form)
    torch.cuda.synchronize()
    p = h.last_plan()
    for off, nbytes, X, ld, t, mn, is_b in [(p.a_pack_offset, p.a_copy_bytes, c.A, c.lda, "T",
                                             c.m, 0),
                                            (p.b_pack_offset, p.b_copy_bytes, c.B, c.ldb, "N",
                                             c.n, 1)]:
        exp = oracle.pack_mx(form, X, is_b, c.layout, t, mn, c.k, ld, p.MT)
        got = h.workspace[off: off + nbytes].cpu().numpy()
        assert np.array_equal(got, exp)
    assert p.MT == tile


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_mx_special_cases(F, form):
    import torch
    say("mx special", form)
    h = F.Handle()
    # beta = 0 never reads C (NaN-filled C); alpha = 0 never reads A, B; k = 0 scales C
    c = synth.make_mx_case(form, COL, 40, 30, 20, "N", "N", alpha=2.0, beta=0.0, seed=2)
    c.C[c_mask(c)] = np.nan
    out, _ = run_mx(F, c, h=h)
    check_mx(c, out)  # beta = 0: the oracle does not read C0 either
    for alpha, beta, k in [(0.0, 0.5, 20), (1.0, 0.25, 0), (0.0, 0.0, 20)]:
        c = synth.make_mx_case(form, COL, 40, 30, k, "N", "N", alpha=alpha, beta=beta, seed=4)
        A = torch.full((8,), float("nan"), device="cuda")  # never read
        C = dev(c.C)
        h.gemm_mx(form, c.layout, c.m, c.n, c.k, alpha, A, c.lda, "N", A, c.ldb, "N", beta, C,
                  c.ldc)
        torch.cuda.synchronize()
        out = C.cpu().numpy()
        m = c_mask(c)
        expect = np.float32(beta) * c.C[m] if beta != 0 else np.zeros(m.sum(), np.float32)
        assert np.array_equal(out[m], expect)
    # argument checks (rejected before any launch): scales only with E4M3; C type
    s = torch.ones(40 * 30, device="cuda")
    args = (h.h, form, COL, 40, 30, 20, 1.0, s, 40, "N", s, 20, "N", 0.0, s, 40)
    if form != F.FIP_E4M3:
        assert F.fip_gemm_mx(*args, F.FIP_F32, s, None) == 18
        assert F.fip_gemm_mx(*args, F.FIP_F32, None, s) == 19
    assert F.fip_gemm_mx(*args, 7, None, None) == 17
    assert F.fip_gemm_mx(h.h, 9, *args[2:], F.FIP_F32, None, None) == 2


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("axis", [0, 1])
def test_quantize_fp8_bit_exact(F, layout, axis):
    """fip_quantize_fp8 gives the oracle's codes and scales bit for bit (including an
    all-zero line, lines of very different magnitude and values near rounding ties)."""
    import torch
    say("quantize", layout, axis)
    g = synth.rng(40 + 2 * layout + axis)
    rows, cols, pad = 517, 389, 3
    X = (g.uniform(-1, 1, (rows, cols)) * np.exp2(g.uniform(-20, 20, (rows, 1))) *
         np.exp2(g.uniform(-20, 20, (1, cols)))).astype(np.float32)
    X[7, :] = 0.0
    X[:, 11] = 0.0
    ld = (rows if layout == COL else cols) + pad
    buf = synth.fill_stored(layout, rows, cols, ld, X, np.float32)
    Qexp, sexp = oracle.quantize_fp8(layout, rows, cols, buf, ld, axis)
    h = F.Handle()
    Xd = dev(buf)
    Q = torch.zeros(Qexp.size, dtype=torch.uint8, device="cuda")
    S = torch.empty(rows if axis == 0 else cols, dtype=torch.float32, device="cuda")
    h.quantize_fp8(layout, rows, cols, Xd, ld, axis, Q, ld, S)
    torch.cuda.synchronize()
    assert np.array_equal(S.cpu().numpy(), sexp)
    inside = synth.fill_stored(layout, rows, cols, ld, np.ones((rows, cols)), np.uint8, 0) == 1
    assert np.array_equal(Q.cpu().numpy()[inside], Qexp[inside])


def test_fp8_end_to_end_quantize_then_gemm(F):
    """binary32 operands -> fip_quantize_fp8 (op(A) per row, op(B) per column) -> E4M3 GEMM:
    within the bound of the quantized operands; the error against the binary64 product of
    the binary32 operands is reported."""
    import torch
    say("fp8 end to end")
    m, n, k = 640, 512, 768
    c = synth.make_mx_case(synth.FORM_BF16X3, COL, m, n, k, "N", "T", alpha=1.0, beta=0.0,
                           seed=123)
    h = F.Handle()
    A32, B32 = dev(c.A32), dev(c.B32)
    QA = torch.zeros(c.A32.size, dtype=torch.uint8, device="cuda")
    QB = torch.zeros(c.B32.size, dtype=torch.uint8, device="cuda")
    sa = torch.empty(m, device="cuda")
    sb = torch.empty(n, device="cuda")
    h.quantize_fp8(COL, m, k, A32, c.lda, 0, QA, c.lda, sa)       # op(A) = A: per row
    h.quantize_fp8(COL, n, k, B32, c.ldb, 0, QB, c.ldb, sb)       # op(B) = B^T: B's rows
    C = torch.zeros(c.C.size, dtype=torch.float32, device="cuda")
    h.gemm_mx(F.FIP_E4M3, COL, m, n, k, 1.0, QA, c.lda, "N", QB, c.ldb, "T", 0.0, C, c.ldc, sa, sb)
    torch.cuda.synchronize()
    # the oracle's own quantization is the reference input; the GPU's must equal it
    qa, s_a = oracle.quantize_fp8(COL, m, k, c.A32, c.lda, 0)
    qb, s_b = oracle.quantize_fp8(COL, n, k, c.B32, c.ldb, 0)
    assert np.array_equal(QA.cpu().numpy(), qa) and np.array_equal(sa.cpu().numpy(), s_a)
    assert np.array_equal(QB.cpu().numpy(), qb) and np.array_equal(sb.cpu().numpy(), s_b)
    q = synth.MxCase(synth.FORM_E4M3, COL, m, n, k, "N", "T", c.lda, c.ldb, c.ldc, 1.0, 0.0,
                     qa, qb, c.C, False, s_a, s_b, c.A32, c.B32)
    nerr, truth = check_mx(q, C.cpu().numpy())
    say(f"fp8 normalised error {nerr:.3e}; vs binary64 product of binary32 inputs {truth:.3e}")
    assert truth < 0.1
