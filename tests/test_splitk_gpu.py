"""GPU parity of the split-k path (FP64 / FP32, and the mixed-precision forms on the 128 x 128
tile): k cut into slices computed by separate workgroups, their partial products summed in
slice order by a second kernel.

Checked against the oracle within 4 k u max D (the mixed forms: check_mx's bound on the
values the stored operands stand for), and for bit-identical results across pack policies,
tile classes (at one split), repeated calls and stale workspaces; packed chunks of every
claimed (panel, k-slice) byte-exact against the oracle's pack."""
import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

from gemm_util import c_mask, check_full, check_mx, to_dev

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
    print("[splitk]", *a, flush=True)


def dcode(F, dtype):
    return F.FIP_F64 if dtype == F64 else F.FIP_F32


def run(F, c, policy=0, split=-1, tile=-1, h=None, C0=None):
    """One call on a fresh handle (or h); returns (C host buffer, handle)."""
    import torch
    if h is None:
        h = F.Handle(policy=policy, tile=tile)
        h.set_attr(F.FIP_ATTR_SPLIT_K, split)
    A, B = to_dev(c.A), to_dev(c.B)
    C = to_dev(c.C if C0 is None else C0)
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
           c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def same_bits(x, y):
    return np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape,layout,tA,tB,pad", [
    ((32, 2500, 3000), COL, "N", "N", 0),      # the skinny k-heavy shapes, ragged
    ((2100, 40, 2900), COL, "T", "N", 7),
    ((40, 1900, 2700), ROW, "N", "T", 3),
    ((300, 200, 1900), ROW, "T", "T", 0),
])
def test_auto_split_matches_oracle(F, dtype, shape, layout, tA, tB, pad):
    m, n, k = shape
    say("auto split", dtype.__name__, shape, layout, tA, tB, pad)
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, alpha=1.5, beta=0.5, dtype=dtype,
                        seed=m + 3 * n + 7 * k)
    out, h = run(F, c)
    p = h.last_plan()
    say("  split", p.split_k, "x", p.slice_ksteps, "k-steps, class", p.tile_class)
    assert p.split_k > 1
    check_full(c, out)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_split_modes_bitwise(F, dtype):
    """All pack policies run the same slices in the same k order: C agrees bit for bit
    (ALL packs per (panel, k-slice) and publishes per slice)."""
    say("modes", dtype.__name__)
    c = synth.make_case(COL, 200, 170, 2300, "N", "T", ld_pad=5, dtype=dtype, seed=31)
    for split in (-1, 3):
        ref, h = run(F, c, F.FIP_PACK_NONE, split=split)
        assert h.last_plan().split_k > 1
        check_full(c, ref)
        for pol in (F.FIP_PACK_AUTO, F.FIP_PACK_ALL, F.FIP_PACK_CONSUME_ONLY):
            say("  split", split, "policy", pol)
            out, h2 = run(F, c, pol, split=split)
            assert h2.last_plan().split_k == h.last_plan().split_k
            assert same_bits(out, ref), (split, pol)
        hn = F.Handle(policy=F.FIP_PACK_ALL)
        hn.set_attr(F.FIP_ATTR_SPLIT_K, split)
        hn.set_attr(F.FIP_ATTR_NO_PUBLISH, 1)
        out, _ = run(F, c, F.FIP_PACK_ALL, h=hn)
        assert same_bits(out, ref), (split, "no publish")


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("split", [1, 2, 5, 7, 32])
def test_forced_split_values(F, dtype, split):
    """Forced slice counts, k not a multiple of the k-step: within tolerance, and the plan
    reports the slices it ran (no empty slice)."""
    say("forced", dtype.__name__, split)
    c = synth.make_case(COL, 70, 90, 1000, "T", "N", alpha=-0.75, beta=1.25, dtype=dtype,
                        seed=41 + split)
    out, h = run(F, c, split=split)
    p = h.last_plan()
    kt = p.KT
    nk = -(-1000 // kt)
    # slices of ceil(nk / split) k-steps; the count is trimmed so that none is empty
    assert 1 <= p.split_k <= split and p.slice_ksteps == -(-nk // split)
    assert (p.split_k - 1) * p.slice_ksteps < nk <= p.split_k * p.slice_ksteps
    check_full(c, out)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_tile_classes_bitwise_at_one_split(F, dtype):
    """The slices cut k at the same k-steps for every tile class, so the classes agree bit
    for bit at one split."""
    say("classes", dtype.__name__)
    c = synth.make_case(COL, 260, 300, 1500, "N", "N", dtype=dtype, seed=51)
    ref, _ = run(F, c, split=4, tile=0)
    check_full(c, ref)
    for tile in (1, 2):
        out, h = run(F, c, split=4, tile=tile)
        assert h.last_plan().split_k == 4 and h.last_plan().tile_class == tile
        assert same_bits(out, ref), tile


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_repeated_calls_and_stale_workspace(F, dtype):
    """Partials left by earlier calls (or garbage) never leak into C: same handle, workspace
    poisoned with 0xFF or zeroed between calls, identical bits."""
    import torch
    say("repeat", dtype.__name__)
    c = synth.make_case(ROW, 36, 3100, 2600, "N", "N", dtype=dtype, seed=61)
    h = F.Handle()
    ref, _ = run(F, c, h=h)
    assert h.last_plan().split_k > 1
    check_full(c, ref)
    for trial, fill in enumerate((0xFF, 0x00, None, 0xFF)):
        if fill is not None:
            h.workspace.fill_(fill)
            torch.cuda.synchronize()
        say("  trial", trial, "fill", fill)
        out, _ = run(F, c, h=h)
        assert same_bits(out, ref), trial


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_split_special_cases(F, dtype):
    """beta = 0 does not read C (NaN C stays out of the result); beta = 1 accumulates."""
    say("special", dtype.__name__)
    c = synth.make_case(COL, 48, 64, 2048, "N", "N", alpha=2.0, beta=0.0, dtype=dtype, seed=71)
    nanC = c.C.copy()
    mask = np.zeros(c.C.size, bool)
    mask[: c.ldc * c.n].reshape(c.n, c.ldc)[:, : c.m] = True
    nanC[mask] = np.nan
    out, h = run(F, c, C0=nanC)
    assert h.last_plan().split_k > 1
    assert np.all(np.isfinite(out[mask]))
    check_full(c, np.where(mask, out, c.C))
    c1 = synth.make_case(COL, 48, 64, 2048, "N", "N", alpha=1.0, beta=1.0, dtype=dtype, seed=72)
    out1, _ = run(F, c1)
    check_full(c1, out1)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_split_packed_chunks_bit_exact(F, dtype):
    """PACK_POLICY=ALL with k split: every (panel, k-slice) is claimed on some XCD and
    published, and the chunks of each claimed slice equal the oracle's pack byte for byte."""
    say("split pack bits", dtype.__name__)
    m, n, k = 70, 100, 1500
    c = synth.make_case(COL, m, n, k, "T", "N", ld_pad=3, dtype=dtype, seed=81)
    h = F.Handle(policy=F.FIP_PACK_ALL)
    h.set_attr(F.FIP_ATTR_SPLIT_K, 4)
    out, _ = run(F, c, h=h)
    check_full(c, out)
    p = h.last_plan()
    S, per, nk = p.split_k, p.slice_ksteps, p.ksteps
    assert S == 4 and p.pack_a and p.pack_b
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))

    def u64(off, count):
        return ws[off: off + 8 * count].cpu().numpy().view(np.uint64)

    for which, ntiles, mnt, off_pack, copy_bytes, off_claim, off_flag, X, ld, t, mn in [
            ("A", p.tiles_m, p.MT, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.a_flag_offset, c.A, c.lda, "T", m),
            ("B", p.tiles_n, p.NT, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.b_flag_offset, c.B, c.ldb, "N", n)]:
        ref = oracle.pack(X, which == "B", c.layout, t, mn, k, ld, mnt, p.KT).view(np.uint8)
        claims = u64(off_claim, p.copies * ntiles * S).reshape(p.copies, ntiles, S)
        flags = u64(off_flag, p.copies * ntiles * S).reshape(p.copies, ntiles, S)
        assert np.all((claims == epoch).any(axis=0)), f"{which}: a (panel, slice) never packed"
        chunk_bytes = p.KT * mnt * c.A.itemsize
        for cp in range(p.copies):
            buf = ws[off_pack + cp * copy_bytes: off_pack + (cp + 1) * copy_bytes].cpu().numpy()
            for t_ in range(ntiles):
                for sl in range(S):
                    if claims[cp, t_, sl] != epoch:
                        continue
                    assert flags[cp, t_, sl] == epoch, (which, cp, t_, sl)
                    q0, q1 = sl * per, min(nk, (sl + 1) * per)
                    lo = (t_ * nk + q0) * chunk_bytes
                    hi = (t_ * nk + q1) * chunk_bytes
                    assert np.array_equal(buf[lo:hi], ref[lo:hi]), (which, cp, t_, sl)


# ---- mixed-precision forms (128 x 128 tiles) -------------------------------------------------

MX_FORMS = [synth.FORM_BF16, synth.FORM_E4M3, synth.FORM_BF16X3, synth.FORM_BF16X3_FAST]
MX_IDS = ["bf16", "e4m3", "bf16x3", "bf16x3f"]


def min_slice_k(form):
    """The planner's minimum k per slice: the split forms share their first pass's split
    work; bfloat16 and E4M3 only copy and split for deep k only."""
    return 256 if form in (synth.FORM_BF16X3, synth.FORM_BF16X3_FAST) else 1024


def deep_k(form):
    """A k deep enough for several default slices on a few tiles."""
    return 2000 if min_slice_k(form) == 256 else 4100


def run_mx(F, c, policy=0, split=-1, h=None, no_publish=0, C0=None):
    """One mixed-precision call on a fresh handle (or h) with the 128 tile; returns (C host
    buffer, handle)."""
    import torch
    if h is None:
        h = F.Handle(policy=policy)
        h.set_attr(F.FIP_ATTR_SPLIT_K, split)
        h.set_attr(F.FIP_ATTR_NO_PUBLISH, no_publish)
    h.set_attr(F.FIP_ATTR_MX_TILE, 128)
    A, B = to_dev(c.A), to_dev(c.B)
    C = to_dev(c.C if C0 is None else C0)
    if c.c_bf16:
        C = C.view(torch.bfloat16)
    sa = to_dev(c.a_scale) if c.a_scale is not None else None
    sb = to_dev(c.b_scale) if c.b_scale is not None else None
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB, dtype=c.form)
    h.gemm_mx(c.form, c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB,
              c.beta, C, c.ldc, sa, sb)
    torch.cuda.synchronize()
    out = (C.view(torch.int16) if c.c_bf16 else C).cpu().numpy()
    return (out.view(np.uint16) if c.c_bf16 else out), h


@pytest.mark.parametrize("form", MX_FORMS, ids=MX_IDS)
@pytest.mark.parametrize("layout,tA,tB,pad,c_bf16", [
    (COL, "N", "N", 0, False),
    (ROW, "T", "N", 5, False),
    (COL, "T", "T", 3, True),
])
def test_mx_auto_split_matches_oracle(F, form, layout, tA, tB, pad, c_bf16):
    """Few tiles, deep k: the planner splits k (slices of >= 256 k); FP8 scales are applied
    per slice (exact powers of two) and alpha, beta, C by the reduction, for a binary32 or a
    bfloat16 C."""
    m, n, k = 300, 260, deep_k(form)
    say("mx auto split", form, layout, tA, tB, pad, c_bf16)
    c = synth.make_mx_case(form, layout, m, n, k, tA, tB, ld_pad=pad, alpha=1.5, beta=0.5,
                           seed=form * 17 + layout * 3 + pad, c_bf16=c_bf16)
    out, h = run_mx(F, c)
    p = h.last_plan()
    say("  split", p.split_k, "x", p.slice_ksteps, "k-steps of", p.KT)
    assert p.MT == 128 and p.split_k > 1 and p.slice_ksteps * p.KT >= min_slice_k(form)
    nerr, truth = check_mx(c, out)
    say(f"  normalised error {nerr:.3e}; vs binary64 product of binary32 inputs {truth:.3e}")


@pytest.mark.parametrize("form", MX_FORMS, ids=MX_IDS)
def test_mx_split_modes_bitwise(F, form):
    """At a given split every pack policy (and ALL without publishing) runs the same slices
    in the same k order: C agrees bit for bit."""
    say("mx split modes", form)
    c = synth.make_mx_case(form, COL, 260, 200, deep_k(form) - 200, "N", "T", ld_pad=3,
                           alpha=1.0, beta=0.5, seed=91 + form)
    for split in (-1, 3):
        ref, h = run_mx(F, c, F.FIP_PACK_NONE, split=split)
        S = h.last_plan().split_k
        assert S > 1
        check_mx(c, ref)
        for pol, nopub in [(F.FIP_PACK_AUTO, 0), (F.FIP_PACK_ALL, 0), (F.FIP_PACK_ALL, 1),
                           (F.FIP_PACK_CONSUME_ONLY, 0)]:
            say("  split", split, "policy", pol, "no publish", nopub)
            out, h2 = run_mx(F, c, pol, split=split, no_publish=nopub)
            assert h2.last_plan().split_k == S
            assert same_bits(out, ref), (split, pol, nopub)


@pytest.mark.parametrize("form", MX_FORMS, ids=MX_IDS)
@pytest.mark.parametrize("split", [2, 5, 32])
def test_mx_forced_split_values(F, form, split):
    """Forced slice counts, k not a multiple of the k-step: within the bound, and the plan
    reports the slices it ran (none empty)."""
    say("mx forced", form, split)
    c = synth.make_mx_case(form, ROW, 150, 90, 1100, "N", "N", alpha=-0.75, beta=1.25,
                           seed=101 + split + form)
    out, h = run_mx(F, c, split=split)
    p = h.last_plan()
    nk = -(-1100 // p.KT)
    assert 1 <= p.split_k <= split and p.slice_ksteps == -(-nk // split)
    assert (p.split_k - 1) * p.slice_ksteps < nk <= p.split_k * p.slice_ksteps
    check_mx(c, out)


@pytest.mark.parametrize("form", MX_FORMS, ids=MX_IDS)
def test_mx_split_packed_chunks_bit_exact(F, form):
    """PACK_POLICY=ALL with k split: every (panel, k-slice) is claimed on some XCD and
    published, and the chunks of each claimed slice equal the oracle's pack byte for byte."""
    say("mx split pack bits", form)
    m, n, k = 300, 170, 1500
    c = synth.make_mx_case(form, COL, m, n, k, "T", "N", ld_pad=4, seed=111 + form)
    out, h = run_mx(F, c, F.FIP_PACK_ALL, split=4)
    check_mx(c, out)
    p = h.last_plan()
    S, per, nk = p.split_k, p.slice_ksteps, p.ksteps
    assert S == 4 and p.pack_a and p.pack_b
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))

    def u64(off, count):
        return ws[off: off + 8 * count].cpu().numpy().view(np.uint64)

    for which, ntiles, off_pack, copy_bytes, off_claim, off_flag, X, ld, t, mn, is_b in [
            ("A", p.tiles_m, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.a_flag_offset, c.A, c.lda, "T", m, 0),
            ("B", p.tiles_n, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.b_flag_offset, c.B, c.ldb, "N", n, 1)]:
        ref = oracle.pack_mx(form, X, is_b, c.layout, t, mn, k, ld, p.MT)
        assert ref.size == copy_bytes
        chunk_bytes = copy_bytes // (ntiles * nk)
        claims = u64(off_claim, p.copies * ntiles * S).reshape(p.copies, ntiles, S)
        flags = u64(off_flag, p.copies * ntiles * S).reshape(p.copies, ntiles, S)
        assert np.all((claims == epoch).any(axis=0)), f"{which}: a (panel, slice) never packed"
        for cp in range(p.copies):
            buf = ws[off_pack + cp * copy_bytes: off_pack + (cp + 1) * copy_bytes].cpu().numpy()
            for t_ in range(ntiles):
                for sl in range(S):
                    if claims[cp, t_, sl] != epoch:
                        continue
                    assert flags[cp, t_, sl] == epoch, (which, cp, t_, sl)
                    lo = (t_ * nk + sl * per) * chunk_bytes
                    hi = (t_ * nk + min(nk, (sl + 1) * per)) * chunk_bytes
                    assert np.array_equal(buf[lo:hi], ref[lo:hi]), (which, cp, t_, sl)


@pytest.mark.parametrize("form", MX_FORMS, ids=MX_IDS)
def test_mx_split_stale_workspace_and_special_cases(F, form):
    """Partials of earlier calls (or garbage) never leak into C; beta = 0 does not read C
    (NaN C stays out of the result)."""
    import torch
    say("mx split stale", form)
    c = synth.make_mx_case(form, COL, 64, 300, deep_k(form) - 400, "N", "N", alpha=2.0,
                           beta=0.0, seed=121 + form)
    nanC = c.C.copy()
    nanC[c_mask(c)] = np.nan
    h = F.Handle()
    ref, _ = run_mx(F, c, h=h, C0=nanC)
    assert h.last_plan().split_k > 1
    check_mx(c, ref)
    for trial, fill in enumerate((0xFF, 0x00, None)):
        if fill is not None:
            h.workspace.fill_(fill)
            torch.cuda.synchronize()
        say("  trial", trial, "fill", fill)
        out, _ = run_mx(F, c, h=h, C0=nanC)
        assert same_bits(out, ref), trial
