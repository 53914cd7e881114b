"""GPU parity of each decision of AUTO's stride rule (paper Sec. 3.3's conditions read for this
GPU): an operand whose extent is a multiple of the tile is read unpacked; one with a fringe has
only its fringe panel packed, on first touch, and that panel's packed bytes equal the oracle's
reference pack; a k-loop of fewer than 4 k-steps packs nothing; binary64 launches of 8 or more
rounds whose operands share one orientation pack every panel.  Every result is checked against
the oracle and bit for bit against the unpacked path (the same kernel and k order)."""
import sys

import numpy as np
import pytest

import oracle
from gemm_util import check_full, check_mx, check_sampled, to_dev
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print("[stride rule]", *a, flush=True)
    sys.stdout.flush()


def run(F, c, policy, tile=2):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
           c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


def _u64(ws, off, count):
    return ws[off: off + 8 * count].cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (ROW, "T", "N")])
def test_fringe_panels_only(F, dtype, layout, tA, tB):
    """32 x 32 tiles, 256 x 64 of them (several rounds, several bands of tile rows per XCD, so
    both operands' panels recur), both extents ragged: AUTO packs the last tile row's A panel
    and the last tile column's B panel, nothing else."""
    m, n, k = 256 * 32 - 3, 64 * 32 - 5, 200
    if layout == ROW:   # row-major C is computed as C^T: the kernel's tile rows are C's columns
        m, n = 64 * 32 - 3, 256 * 32 - 5
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=7, alpha=1.5, beta=0.5, dtype=dtype,
                        seed=91)
    say("fringe", dtype.__name__, layout, tA, tB)
    ref, _ = run(F, c, F.FIP_PACK_NONE)
    out, h = run(F, c, F.FIP_PACK_AUTO)
    p = h.last_plan()
    assert (p.pack_a, p.pack_b) == (1, 1)
    assert (p.a_pack_first, p.b_pack_first) == (p.tiles_m - 1, p.tiles_n - 1)
    assert p.split_k == 1
    check_full(c, out)
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    for X, ld, t, mn, mnt, ntiles, first, off_pack, copy_bytes, off_claim, off_flag, is_b in [
            (c.A, c.lda, tA, m, p.MT, p.tiles_m, p.a_pack_first, p.a_pack_offset,
             p.a_copy_bytes, p.a_claim_offset, p.a_flag_offset, 0),
            (c.B, c.ldb, tB, n, p.NT, p.tiles_n, p.b_pack_first, p.b_pack_offset,
             p.b_copy_bytes, p.b_claim_offset, p.b_flag_offset, 1)]:
        refpack = oracle.pack(X, is_b, layout, t, mn, k, ld, mnt, p.KT).view(np.uint8)
        panel = refpack.size // ntiles
        assert copy_bytes == panel
        claims = _u64(ws, off_claim, p.copies * ntiles).reshape(p.copies, ntiles)
        flags = _u64(ws, off_flag, p.copies * ntiles).reshape(p.copies, ntiles)
        assert not (claims[:, :first] == epoch).any(), "an interior panel was claimed"
        owners = np.flatnonzero(claims[:, first] == epoch)
        assert owners.size >= 1
        for cp in owners:
            assert flags[cp, first] == epoch
            got = ws[off_pack + cp * copy_bytes: off_pack + (cp + 1) * copy_bytes].cpu().numpy()
            assert np.array_equal(got, refpack[first * panel:]), (is_b, cp)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_tile_multiples_read_unpacked(F, dtype):
    m, n, k = 64 * 32, 64 * 32, 200
    c = synth.make_case(COL, m, n, k, "T", "N", alpha=1.5, beta=0.5, dtype=dtype, seed=92)
    say("multiples", dtype.__name__)
    out, h = run(F, c, F.FIP_PACK_AUTO)
    p = h.last_plan()
    assert (p.pack_a, p.pack_b, p.workspace_bytes) == (0, 0, 0)
    check_full(c, out)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_short_k_loop_packs_nothing(F, dtype):
    kt = 16 if dtype == np.float64 else 32
    m, n, k = 64 * 32 - 3, 64 * 32 - 5, 3 * kt
    c = synth.make_case(ROW, m, n, k, "N", "T", alpha=1.5, beta=0.5, dtype=dtype, seed=93)
    say("short k", dtype.__name__)
    out, h = run(F, c, F.FIP_PACK_AUTO)
    p = h.last_plan()
    assert (p.pack_a, p.pack_b) == (0, 0)
    check_full(c, out)


def test_bf16_fringe_panels_only(F):
    """The bfloat16 form on its 128 tile, 32 x 32 tiles (two rounds), ragged extents."""
    import torch
    m, n, k = 32 * 128 - 3, 32 * 128 - 5, 320
    c = synth.make_mx_case(synth.FORM_BF16, COL, m, n, k, "N", "T", ld_pad=4, alpha=1.0,
                           beta=0.5, seed=94)
    say("bf16 fringe")
    outs = {}
    for pol in (F.FIP_PACK_NONE, F.FIP_PACK_AUTO):
        h = F.Handle(policy=pol)
        h.set_attr(F.FIP_ATTR_MX_TILE, 128)
        A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
        h.gemm_mx(c.form, COL, m, n, k, c.alpha, A, c.lda, "N", B, c.ldb, "T", c.beta, C, c.ldc)
        torch.cuda.synchronize()
        outs[pol] = C.cpu().numpy()
        if pol == F.FIP_PACK_AUTO:
            p = h.last_plan()
            assert p.pack_a and p.a_pack_first == p.tiles_m - 1 and p.MT == 128
    assert np.array_equal(outs[F.FIP_PACK_AUTO].view(np.uint8), outs[F.FIP_PACK_NONE].view(np.uint8))
    check_mx(c, outs[F.FIP_PACK_AUTO])


@pytest.mark.parametrize("layout,tA,tB", [(COL, "T", "N"), (ROW, "N", "T")])
def test_whole_panels_same_orientation(F, layout, tA, tB):
    """binary64, 8192 x 8192 (8 rounds of 128 x 128 tiles), k = 1024 (64 k-steps), both operands
    K-major in the kernel: AUTO packs every panel of both on first touch; C equals the unpacked
    launch's bit for bit and the oracle on sampled entries; the first and last panels of each
    operand equal the oracle's reference pack."""
    m = n = 8192
    k = 1024
    c = synth.make_case(layout, m, n, k, tA, tB, alpha=1.5, beta=0.5, dtype=np.float64, seed=95)
    say("whole panels", layout, tA, tB)
    ref, _ = run(F, c, F.FIP_PACK_NONE, tile=-1)
    out, h = run(F, c, F.FIP_PACK_AUTO, tile=-1)
    p = h.last_plan()
    assert (p.pack_a, p.pack_b, p.a_pack_first, p.b_pack_first, p.copies) == (1, 1, 0, 0, 1)
    assert p.MT == 128 and p.a_kmajor == p.b_kmajor
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))
    check_sampled(c, out, count=2048)
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    for X, ld, t, mn, ntiles, off_pack, copy_bytes, off_claim, off_flag, is_b in [
            (c.A, c.lda, tA, m, p.tiles_m, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.a_flag_offset, 0),
            (c.B, c.ldb, tB, n, p.tiles_n, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.b_flag_offset, 1)]:
        claims = _u64(ws, off_claim, ntiles)
        flags = _u64(ws, off_flag, ntiles)
        assert (claims == epoch).all() and (flags == epoch).all(), is_b
        refpack = oracle.pack(X, is_b, layout, t, mn, k, ld, 128, p.KT).view(np.uint8)
        panel = refpack.size // ntiles
        assert copy_bytes == refpack.size
        for tt in (0, ntiles - 1):
            got = ws[off_pack + tt * panel: off_pack + (tt + 1) * panel].cpu().numpy()
            assert np.array_equal(got, refpack[tt * panel:(tt + 1) * panel]), (is_b, tt)
