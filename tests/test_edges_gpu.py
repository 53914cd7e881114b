"""GPU parity on the edge cases and at the full sizes of the sweep and mixed workloads.

- NaN / Inf in op(A) and op(B): a NaN anywhere in row i of op(A) makes row i of C NaN, an
  infinity in column j of op(B) makes column j of C infinite (the oracle gives the same
  pattern, by IEEE arithmetic in its own loop); every other entry stays finite and within the
  usual bound.  Run with packing forced (the pack carries the special values) and without.
- Subnormal operands: a product of a subnormal and a normal number, and products that are
  themselves subnormal, through every MFMA type.  Integer multiples of powers of two keep
  every product and sum exact, so the result either equals the oracle bit for bit or, if the
  matrix unit flushes subnormals, is zero; the test records which, and any other outcome fails.
- The packed copy keeps NaN payloads, signalling NaNs, -0.0, subnormals and infinities bit for
  bit (paper Sec. 3.2: the packed panel holds the operand itself): compared byte for byte with
  the oracle's reference pack, binary64, binary32, bfloat16 and E4M3.
- The sweep's transposed, row-major and padded variants at m = n = k = 4096, and the four
  mixed-precision forms at m = n = k = 4096: exact oracle values on sampled entries plus a
  Freivalds probe of every row.
"""
import sys

import numpy as np
import pytest

import oracle
from gemm_util import (U, c_mask, check_mx, check_mx_sampled, check_sampled, run_gpu, to_dev)
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
    print("[edges]", *a, flush=True)
    sys.stdout.flush()


def run_policy(F, c, policy, tile=-1):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
           c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def compare_special(c, got):
    """Same NaN / Inf pattern as the oracle (signs of the infinities included); finite
    entries within 4 k u max D over the finite part."""
    ref, D = oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                         c.transB, c.beta, c.C, c.ldc)
    mask = c_mask(c)
    g = got[mask].astype(np.float64)
    r = ref[mask]
    d = D[mask]
    assert np.array_equal(np.isnan(g), np.isnan(r)), "NaN pattern differs"
    assert np.array_equal(np.isposinf(g), np.isposinf(r)), "+Inf pattern differs"
    assert np.array_equal(np.isneginf(g), np.isneginf(r)), "-Inf pattern differs"
    fin = np.isfinite(r)
    dmax = float(d[fin].max())
    err = float(np.abs(g[fin] - r[fin]).max())
    assert err <= 4 * max(c.k, 1) * U[c.dtype] * dmax, err
    return ref


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB,pad", [(COL, "N", "N", 0), (COL, "T", "N", 7),
                                              (ROW, "N", "T", 7), (ROW, "T", "T", 0)])
@pytest.mark.parametrize("policy", [1, 2], ids=["all", "none"])
def test_nan_inf_propagate_along_row_and_column(F, dtype, layout, tA, tB, pad, policy):
    m, n, k = 300, 260, 170
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, alpha=1.5, beta=0.5, dtype=dtype,
                        seed=41 + layout * 4 + (tA == "T") * 2 + (tB == "T"))
    opA = synth.op_view(c.A, c.layout, tA, m, k, c.lda)
    opB = synth.op_view(c.B, c.layout, tB, k, n, c.ldb)
    i0, p0, p1, j1, p2, j2 = 131, 77, 5, 200, 169, 3
    opA[i0, p0] = np.nan
    opB[p1, j1] = np.inf
    opB[p2, j2] = -np.inf
    say("nan/inf", dtype.__name__, layout, tA, tB, pad, "policy", policy)
    got, _ = run_policy(F, c, policy)
    ref = compare_special(c, got)
    Cv = synth.op_view(got, c.layout, "N", m, n, c.ldc)
    assert np.isnan(Cv[i0, :]).all()
    others = np.ones(m, bool)
    others[i0] = False
    assert np.isinf(Cv[others, j1]).all() and np.isinf(Cv[others, j2]).all()
    fin = np.ones((m, n), bool)
    fin[i0, :] = False
    fin[:, [j1, j2]] = False
    assert np.isfinite(Cv[fin]).all()
    assert np.isfinite(synth.op_view(ref, c.layout, "N", m, n, c.ldc)[fin]).all()


def test_bf16_nan_inf_propagate(F):
    """The bfloat16 form: a NaN code in op(A) and an infinity in op(B)."""
    import torch
    m, n, k = 300, 260, 170
    c = synth.make_mx_case(synth.FORM_BF16, COL, m, n, k, "T", "N", ld_pad=4, alpha=1.0,
                           beta=0.5, seed=43)
    opA = synth.op_view(c.A, COL, "T", m, k, c.lda)
    opB = synth.op_view(c.B, COL, "N", k, n, c.ldb)
    opA[17, 100] = 0x7FC1        # a quiet NaN with a payload
    opB[3, 250] = 0x7F80         # +Inf
    for policy in (1, 2):
        say("bf16 nan/inf policy", policy)
        h = F.Handle(policy=policy)
        A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
        h.gemm_mx(c.form, COL, m, n, k, c.alpha, A, c.lda, "T", B, c.ldb, "N", c.beta, C, c.ldc)
        torch.cuda.synchronize()
        Cv = synth.op_view(C.cpu().numpy(), COL, "N", m, n, c.ldc)
        assert np.isnan(Cv[17, :]).all()
        rows = np.arange(m) != 17
        assert np.isinf(Cv[rows, 250]).all()
        fin = np.ones((m, n), bool)
        fin[17, :] = False
        fin[:, 250] = False
        assert np.isfinite(Cv[fin]).all()


def _pow2_int_case(layout, m, n, k, dtype, ea, eb, seed):
    """op(A) = integers in [-8, 8] times 2^ea, op(B) the same times 2^eb; alpha = 1, beta = 0:
    every product and partial sum is exact (far fewer than 53 / 24 significant bits)."""
    g = synth.rng(seed)
    c = synth.make_case(layout, m, n, k, "N", "N", alpha=1.0, beta=0.0, dtype=dtype, seed=seed)
    opA = synth.op_view(c.A, layout, "N", m, k, c.lda)
    opB = synth.op_view(c.B, layout, "N", k, n, c.ldb)
    opA[:, :] = (g.integers(-8, 9, size=(m, k)) * 2.0 ** ea).astype(dtype)
    opB[:, :] = (g.integers(-8, 9, size=(k, n)) * 2.0 ** eb).astype(dtype)
    return c


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_subnormal_operands_recorded(F, dtype):
    tiny = -1040 if dtype == F64 else -140       # 8 * 2^tiny is below the smallest normal
    cases = {
        # a subnormal operand times a normal one: normal products
        "subnormal inputs": (tiny, 20 if dtype == F64 else 20),
        # normal operands whose products are subnormal
        "subnormal products": ((tiny // 2), (tiny // 2) - 8),
    }
    for name, (ea, eb) in cases.items():
        for policy in (1, 2):
            c = _pow2_int_case(COL, 130, 70, 40, dtype, ea, eb, seed=5)
            got, _ = run_policy(F, c, policy)
            ref, _ = oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, "N", c.B, c.ldb,
                                 "N", 0.0, c.C, c.ldc)
            mask = c_mask(c)
            g, r = got[mask], ref[mask].astype(dtype)
            exact = np.array_equal(g.view(np.uint8), r.view(np.uint8))
            flushed = bool(np.all(g == 0))
            say(f"{dtype.__name__} {name} policy {policy}: "
                f"{'kept exactly' if exact else 'flushed to zero' if flushed else 'OTHER'}")
            assert exact or flushed, (name, float(np.abs(g - r).max()))
            if name == "subnormal inputs":
                # the oracle's products are normal numbers here, so an exact result proves the
                # subnormal inputs reached the products
                assert np.any(r != 0)


def _special_values(dtype, count, seed):
    """An array mixing ordinary values with NaN payloads, signalling NaNs, -0.0, subnormals and
    infinities (as raw bit patterns)."""
    g = synth.rng(seed)
    vals = g.uniform(-1, 1, count).astype(dtype)
    if dtype == F64:
        specials = np.array([0x7FF8000000001234, 0xFFF800000000ABCD, 0x7FF0000000000001,
                             0x8000000000000000, 0x0000000000000001, 0x800FFFFFFFFFFFFF,
                             0x7FF0000000000000, 0xFFF0000000000000], dtype=np.uint64)
        bits = vals.view(np.uint64)
    else:
        specials = np.array([0x7FC01234, 0xFFC0ABCD, 0x7F800001, 0x80000000, 0x00000001,
                             0x807FFFFF, 0x7F800000, 0xFF800000], dtype=np.uint32)
        bits = vals.view(np.uint32)
    where = g.choice(count, size=count // 3, replace=False)
    bits[where] = specials[g.integers(0, specials.size, size=where.size)]
    return vals


def _check_claimed_packs(F, h, c, items, pack_fn):
    p = h.last_plan()
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    for which, ntiles, off_pack, copy_bytes, off_claim, off_flag, args in items(p):
        ref = pack_fn(*args).view(np.uint8)
        assert ref.size == copy_bytes
        claims = ws[off_claim: off_claim + 8 * p.copies * ntiles].cpu().numpy().view(np.uint64)
        flags = ws[off_flag: off_flag + 8 * p.copies * ntiles].cpu().numpy().view(np.uint64)
        claims = claims.reshape(p.copies, ntiles)
        flags = flags.reshape(p.copies, ntiles)
        packs = ws[off_pack: off_pack + p.copies * copy_bytes].cpu().numpy().reshape(p.copies, -1)
        panel = copy_bytes // ntiles
        checked = 0
        for t in range(ntiles):
            owners = [cp for cp in range(p.copies) if claims[cp, t] == epoch]
            assert owners, f"{which} panel {t} packed by nobody"
            for cp in owners:
                assert flags[cp, t] == epoch
                assert np.array_equal(packs[cp, t * panel: (t + 1) * panel],
                                      ref[t * panel: (t + 1) * panel]), (which, cp, t)
                checked += 1
        assert checked >= ntiles


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB,pad", [(COL, "N", "T", 7), (ROW, "T", "N", 0)])
def test_pack_keeps_special_bits(F, dtype, layout, tA, tB, pad):
    m, n, k = 300, 200, 77
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, dtype=dtype, seed=61)
    for buf, rows, cols, t, ld, s in ((c.A, m, k, tA, c.lda, 1), (c.B, k, n, tB, c.ldb, 2)):
        v = synth.op_view(buf, layout, t, rows, cols, ld)
        v[:, :] = _special_values(dtype, rows * cols, s).reshape(rows, cols)
    say("pack special bits", dtype.__name__, layout, tA, tB, pad)
    _, h = run_policy(F, c, F.FIP_PACK_ALL)

    def items(p):
        return [("A", p.tiles_m, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
                 p.a_flag_offset, (c.A, 0, layout, tA, m, k, c.lda, p.MT, p.KT)),
                ("B", p.tiles_n, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
                 p.b_flag_offset, (c.B, 1, layout, tB, n, k, c.ldb, p.NT, p.KT))]
    _check_claimed_packs(F, h, c, items, oracle.pack)


@pytest.mark.parametrize("form", [synth.FORM_BF16, synth.FORM_E4M3], ids=["bf16", "e4m3"])
def test_mx_pack_keeps_special_bits(F, form):
    import torch
    m, n, k = 600, 400, 170
    layout, tA, tB = COL, "T", "N"
    c = synth.make_mx_case(form, layout, m, n, k, tA, tB, ld_pad=4, seed=63 + form)
    g = synth.rng(form)
    specials = (np.array([0x7FC1, 0xFFC3, 0x7F81, 0x8000, 0x0001, 0x807F, 0x7F80, 0xFF80],
                         np.uint16) if form == synth.FORM_BF16 else
                np.array([0x7F, 0xFF, 0x80, 0x01, 0x87, 0x07], np.uint8))
    for buf, rows, cols, t, ld in ((c.A, m, k, tA, c.lda), (c.B, k, n, tB, c.ldb)):
        v = synth.op_view(buf, layout, t, rows, cols, ld)
        sel = g.random((rows, cols)) < 0.3
        v[sel] = specials[g.integers(0, specials.size, size=int(sel.sum()))]
    say("mx pack special bits", form)
    h = F.Handle(policy=F.FIP_PACK_ALL)
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    sa = to_dev(c.a_scale) if c.a_scale is not None else None
    sb = to_dev(c.b_scale) if c.b_scale is not None else None
    h.gemm_mx(form, layout, m, n, k, c.alpha, A, c.lda, tA, B, c.ldb, tB, c.beta, C, c.ldc, sa, sb)
    torch.cuda.synchronize()

    def items(p):
        return [("A", p.tiles_m, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
                 p.a_flag_offset, (form, c.A, 0, layout, tA, m, k, c.lda, p.MT)),
                ("B", p.tiles_n, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
                 p.b_flag_offset, (form, c.B, 1, layout, tB, n, k, c.ldb, p.NT))]
    _check_claimed_packs(F, h, c, items, oracle.pack_mx)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB,pad", [(ROW, "T", "N", 7), (COL, "T", "T", 7),
                                              (ROW, "N", "T", 0)])
def test_sweep_variants_4096_sampled(F, dtype, layout, tA, tB, pad):
    """The sweep's transposed / row-major / padded variants at its largest FP64-FP32 size that
    every variant runs (4096), in the benchmark's launch configuration (AUTO policy)."""
    n = 4096
    say("4096 variant", dtype.__name__, layout, tA, tB, pad)
    c = synth.make_case(layout, n, n, n, tA, tB, ld_pad=pad, alpha=1.5, beta=0.5, dtype=dtype,
                        seed=synth.BASE_SEED + 17 * n)
    h = F.Handle()
    e = check_sampled(c, run_gpu(h, c), count=2048)
    say("normalised sampled error", e)


@pytest.mark.parametrize("form", [synth.FORM_BF16, synth.FORM_E4M3, synth.FORM_BF16X3,
                                  synth.FORM_BF16X3_FAST],
                         ids=["bf16", "e4m3", "bf16x3", "bf16x3f"])
def test_mx_4096_sampled(F, form):
    """The mixed-precision forms at m = n = k = 4096 (column-major NN, alpha = 1, beta = 0, the
    benchmark's configuration): sampled entries against the oracle, a Freivalds probe of every
    row, and the error against the binary64 product of the unquantized binary32 values."""
    import torch
    n = 4096
    say("mx 4096", form)
    c = synth.make_mx_case(form, COL, n, n, n, "N", "N", alpha=1.0, beta=0.0,
                           seed=synth.BASE_SEED + n + form)
    h = F.Handle()
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    sa = to_dev(c.a_scale) if c.a_scale is not None else None
    sb = to_dev(c.b_scale) if c.b_scale is not None else None
    h.gemm_mx(form, COL, n, n, n, c.alpha, A, c.lda, "N", B, c.ldb, "N", c.beta, C, c.ldc, sa, sb)
    torch.cuda.synchronize()
    nerr, truth = check_mx_sampled(c, C.cpu().numpy(), count=512)
    say(f"normalised sampled error {nerr:.3e}; vs binary64 product of the binary32 values "
        f"{truth:.3e} of max D")
