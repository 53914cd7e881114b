"""GPU parity tests: the HIP path through the C-ABI against the oracle.

Every case prints its name before it touches the GPU.  Inputs are seeded
synthetic matrices (uniform [-1, 1] entries, ld padding filled with NaN so any
out-of-matrix read poisons C).
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

from gemm_util import check_full, check_sampled, run_gpu, to_dev

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
    print(*a, flush=True)
    sys.stdout.flush()


def handle(F, policy=0, tile=-1):
    return F.Handle(policy=policy, tile=tile)


def test_xcc_map(F):
    import torch
    say("xcc_map 2048 blocks")
    h = handle(F)
    out = torch.full((2048,), 0xFFFF, dtype=torch.int32, device="cuda")
    assert F.fip_xcc_map(h.h, out, 2048) == 0
    torch.cuda.synchronize()
    ids = out.cpu().numpy()
    assert ids.min() >= 0 and ids.max() < 8, ids[:32]
    distinct = np.unique(ids)
    match = float(np.mean(ids == (np.arange(2048) % 8)))
    say("distinct XCC ids", distinct.tolist(), "fraction with id == block % 8:", match)
    assert distinct.size >= 2


def test_plain_dgemm_256(F):
    """DGEMM, column-major, no transpose, m=n=k=256, ld=256, alpha=beta=1."""
    say("plain dgemm 256")
    c = synth.make_case(COL, 256, 256, 256, "N", "N", alpha=1.0, beta=1.0, dtype=F64,
                        seed=synth.BASE_SEED)
    h = handle(F)
    e = check_full(c, run_gpu(h, c))
    say("normalised error", e)


SIZES = [16, 33, 100, 257]


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", [COL, ROW], ids=["col", "row"])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
@pytest.mark.parametrize("pad", [0, 7])
def test_square_sweep_small(F, dtype, layout, tA, tB, pad):
    h = handle(F)
    for n in SIZES:
        say("sweep", dtype.__name__, layout, tA, tB, pad, n)
        c = synth.make_case(layout, n, n, n, tA, tB, ld_pad=pad, alpha=1.5, beta=0.5,
                            dtype=dtype, seed=synth.BASE_SEED + 1 + n)
        check_full(c, run_gpu(h, c))


RAGGED = [(300, 200, 77), (129, 65, 33), (1, 1, 1), (1000, 3, 500), (3, 1000, 500),
          (517, 259, 1031), (64, 64, 1), (17, 300, 16)]


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("policy", [0, 1, 2], ids=["auto", "all", "none"])
def test_ragged_shapes(F, dtype, policy):
    h = handle(F, policy=policy)
    g = synth.rng(3)
    for (m, n, k) in RAGGED:
        layout = int(g.integers(0, 2))
        tA, tB = "NT"[int(g.integers(0, 2))], "NT"[int(g.integers(0, 2))]
        pad = 7 * int(g.integers(0, 2))
        say("ragged", dtype.__name__, policy, m, n, k, layout, tA, tB, pad)
        c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, dtype=dtype,
                            seed=int(g.integers(1 << 30)))
        check_full(c, run_gpu(h, c))


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("tile", [0, 1, 2])
def test_every_tile_class(F, dtype, tile):
    h = handle(F, policy=1, tile=tile)
    for layout, tA, tB in [(COL, "N", "N"), (COL, "T", "T"), (ROW, "N", "T"), (ROW, "T", "N")]:
        say("tile", tile, dtype.__name__, layout, tA, tB)
        c = synth.make_case(layout, 300, 280, 150, tA, tB, ld_pad=7, dtype=dtype, seed=tile + 5)
        check_full(c, run_gpu(h, c))


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(1024, 1024, 32), (32, 1024, 1024), (1024, 32, 1024)])
def test_skinny(F, dtype, shape):
    h = handle(F)
    for tA, tB in [("N", "N"), ("T", "T")]:
        say("skinny", dtype.__name__, shape, tA, tB)
        c = synth.make_case(COL, *shape, tA, tB, dtype=dtype, seed=sum(shape))
        check_full(c, run_gpu(h, c))


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_special_cases(F, dtype):
    import torch
    h = handle(F)
    say("special alpha=0", dtype.__name__)
    c = synth.make_case(COL, 50, 40, 30, "N", "T", ld_pad=7, alpha=0.0, beta=0.5, dtype=dtype,
                        seed=1)
    c.A[:] = np.nan
    c.B[:] = np.nan
    check_full(c, run_gpu(h, c))
    say("special beta=0 with NaN C", dtype.__name__)
    c = synth.make_case(ROW, 150, 140, 30, "T", "N", alpha=1.5, beta=0.0, dtype=dtype, seed=2)
    Cn = c.C.copy()
    mask = np.zeros(c.C.size, bool)
    v = mask.reshape(c.m, c.ldc)[:, : c.n]
    v[:, :] = True
    c.C[mask] = np.nan
    out = run_gpu(h, c)
    c.C = np.where(mask, 0.0, c.C).astype(dtype)  # oracle with beta=0 never reads C either
    check_full(c, np.where(mask, out, c.C))
    assert np.all(np.isfinite(out[mask]))
    say("special k=0", dtype.__name__)
    c = synth.make_case(COL, 33, 31, 0, "N", "N", ld_pad=7, alpha=2.0, beta=-0.5, dtype=dtype,
                        seed=3)
    check_full(c, run_gpu(h, c))
    say("special m=0 / n=0 / alpha=0,beta=1 are no-ops", dtype.__name__)
    c = synth.make_case(COL, 20, 20, 20, "N", "N", alpha=0.0, beta=1.0, dtype=dtype, seed=4)
    out = run_gpu(h, c)
    assert np.array_equal(out, c.C, equal_nan=True)
    fn = F.fip_dgemm if dtype == F64 else F.fip_sgemm
    C = to_dev(c.C)
    assert fn(h.h, 0, 0, 20, 20, 1.0, None, 20, "N", None, 20, "N", 0.0, C, 20) == 0
    assert fn(h.h, 0, 20, 0, 20, 1.0, None, 20, "N", None, 20, "N", 0.0, C, 20) == 0
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), c.C, equal_nan=True)


def _run_policy(F, c, policy, no_publish=0, ws=None, order=0, tile=-1, split=-1, copies=-1):
    import torch
    h = handle(F, policy=policy, tile=tile)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    h.set_attr(F.FIP_ATTR_NO_PUBLISH, no_publish)
    h.set_attr(F.FIP_ATTR_ORDER, order)
    h.set_attr(F.FIP_ATTR_SPLIT_K, split)
    if ws is not None:
        h.attach_workspace(ws)
    A, B = to_dev(c.A), to_dev(c.B)
    C = to_dev(c.C)
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
           c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy(), h


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB", [(COL, "N", "N"), (COL, "T", "N"), (ROW, "N", "T"),
                                          (ROW, "T", "T")])
def test_modes_bitwise_identical(F, dtype, layout, tA, tB):
    """Fused (AUTO, ALL, ALL without publishing, both tile orders, waiting or not), unpacked
    (NONE) and pack-then-compute (fip_pack + CONSUME_ONLY) run the same tile kernel with the
    same k order, so C must agree bit for bit; and with the oracle within tolerance."""
    say("modes", dtype.__name__, layout, tA, tB)
    c = synth.make_case(layout, 700, 600, 333, tA, tB, ld_pad=7 if tA == "T" else 0,
                        dtype=dtype, seed=99)
    ref, _ = _run_policy(F, c, F.FIP_PACK_NONE)
    check_full(c, ref)
    for pol, nopub, order in [(F.FIP_PACK_AUTO, 0, 0), (F.FIP_PACK_ALL, 0, 1), (F.FIP_PACK_ALL, 1, 0),
                              (F.FIP_PACK_ALL, 0, 0), (F.FIP_PACK_CONSUME_ONLY, 0, 0),
                              (F.FIP_PACK_AUTO, 0, 1)]:
        say("  policy", pol, "no_publish", nopub, "order", order)
        out, _ = _run_policy(F, c, pol, nopub, order=order)
        assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), (pol, nopub, order)


@pytest.mark.parametrize("dtype,shape,tile", [(F64, (2048, 2048, 256), 2), (F32, (2048, 2048, 333), 2),
                                              (F64, (4096, 4096, 64), 0)])
@pytest.mark.parametrize("copies", [1, 8], ids=["shared", "per-xcd"])
def test_fused_repeated_calls_bitwise(F, dtype, shape, tile, copies):
    """Repeated fused calls on launches with several rounds of tiles (so later tiles do read
    packed panels) must equal the unpacked path bit for bit every time; the workspace is
    poisoned before each call.  Tile classes change the blocking only, so at the same k split
    (here none) they round identically."""
    import torch
    m, n, k = shape
    c = synth.make_case(COL, m, n, k, "N", "N", dtype=dtype, seed=7)
    ref, _ = _run_policy(F, c, F.FIP_PACK_NONE, tile=tile, split=1)
    check_full(c, ref)
    ref_default, _ = _run_policy(F, c, F.FIP_PACK_NONE, split=1)
    assert np.array_equal(ref.view(np.uint8), ref_default.view(np.uint8)), \
        ("tile classes round differently", _diff_summary(ref, ref_default))
    A, B = to_dev(c.A), to_dev(c.B)
    h = handle(F, policy=F.FIP_PACK_ALL, tile=tile)
    h.set_attr(F.FIP_ATTR_STATS, 1)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    dt = F.FIP_F64 if dtype == F64 else F.FIP_F32
    p = h.plan(dt, COL, m, n, k, "N", "N")
    h.ensure_workspace(p.workspace_bytes)
    total_packed_reads = 0
    for trial in range(4):
        say("repeat", dtype.__name__, shape, copies, trial)
        h.workspace.fill_(0xFF)
        h.workspace[:64].zero_()
        C = to_dev(c.C)
        h.gemm(COL, m, n, k, c.alpha, A, c.lda, "N", B, c.ldb, "N", c.beta, C, c.ldc)
        torch.cuda.synchronize()
        out = C.cpu().numpy()
        st = h.workspace[p.stats_offset: p.stats_offset + 24].cpu().numpy().view(np.uint64)
        total_packed_reads += int(st[1])
        check_full(c, out)
        assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), \
            (trial, st.tolist(), _diff_summary(out, ref))
    say("packed-chunk reads over the trials:", total_packed_reads)
    assert total_packed_reads > 0


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_graph_capture_replays_with_new_inputs(F, dtype):
    """A GEMM captured into a graph on a shape that packs when run eagerly (many rounds of 32 x
    32 tiles, a fringe panel) replays correctly while its inputs change between replays: under capture the
    call is planned unpacked.  Eager work and synchronisations sit between the replays, and
    every replay is checked against the oracle for that replay's inputs."""
    import torch
    m, n, k = 2045, 2043, 256   # ragged: AUTO packs the fringe panel when run eagerly
    cases = [synth.make_case(COL, m, n, k, "N", "T", alpha=1.5, beta=0.5, dtype=dtype,
                             seed=300 + i) for i in range(4)]
    c0 = cases[0]
    h = handle(F, policy=F.FIP_PACK_AUTO, tile=2)
    dt = F.FIP_F64 if dtype == F64 else F.FIP_F32
    eager_plan = h.plan(dt, COL, m, n, k, "N", "T")
    assert eager_plan.pack_a or eager_plan.pack_b, "the shape should pack when run eagerly"
    A, B, C = to_dev(c0.A), to_dev(c0.B), to_dev(c0.C)
    say("graph: eager warm-up", dtype.__name__)
    h.gemm(COL, m, n, k, c0.alpha, A, c0.lda, "N", B, c0.ldb, "T", c0.beta, C, c0.ldc)
    torch.cuda.synchronize()
    check_full(c0, C.cpu().numpy())
    g = torch.cuda.CUDAGraph()
    say("graph: capture")
    with torch.cuda.graph(g):
        h.gemm(COL, m, n, k, c0.alpha, A, c0.lda, "N", B, c0.ldb, "T", c0.beta, C, c0.ldc)
    assert h.last_plan().policy == F.FIP_PACK_NONE
    assert (h.last_plan().pack_a, h.last_plan().pack_b) == (0, 0)
    for rep, c in enumerate(cases[1:] + cases[:1]):
        say("graph: replay", rep)
        A.copy_(to_dev(c.A))          # eager work between replays: new operands and C
        B.copy_(to_dev(c.B))
        C.copy_(to_dev(c.C))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_full(c, C.cpu().numpy())


def _diff_summary(x, y):
    """Where two C buffers differ: count, first flat index and largest difference."""
    d = np.flatnonzero(x != y)
    if d.size == 0:
        return "no differing entries (NaN payloads?)"
    return (int(d.size), int(d[0]), float(np.abs(x.ravel()[d] - y.ravel()[d]).max()))


def _ws_u64(ws, off, count):
    return ws[off: off + 8 * count].cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout,tA,tB,pad", [(COL, "N", "N", 0), (COL, "T", "N", 7),
                                              (ROW, "N", "T", 7), (ROW, "T", "T", 0)])
@pytest.mark.parametrize("copies", [1, 8], ids=["shared", "per-xcd"])
def test_packed_buffers_bit_exact(F, dtype, layout, tA, tB, pad, copies):
    """Every panel a producer claimed must equal the oracle's reference pack byte for byte,
    and every panel must have been packed (PACK_POLICY=ALL), with one copy shared by all XCDs
    or one per XCD."""
    say("pack bits", dtype.__name__, layout, tA, tB, pad, copies)
    m, n, k = 300, 200, 77
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, dtype=dtype, seed=17)
    out, h = _run_policy(F, c, F.FIP_PACK_ALL, copies=copies)
    check_full(c, out)
    p = h.last_plan()
    ws = h.workspace
    epoch = np.uint64(h.get_attr(F.FIP_ATTR_EPOCH))
    assert p.pack_a and p.pack_b and p.copies == copies
    nk = p.ksteps
    for which, ntiles, mnt, off_pack, copy_bytes, off_claim, off_flag, X, ld, t, mn in [
            ("A", p.tiles_m, p.MT, p.a_pack_offset, p.a_copy_bytes, p.a_claim_offset,
             p.a_flag_offset, c.A, c.lda, tA, m),
            ("B", p.tiles_n, p.NT, p.b_pack_offset, p.b_copy_bytes, p.b_claim_offset,
             p.b_flag_offset, c.B, c.ldb, tB, n)]:
        ref = oracle.pack(X, which == "B", layout, t, mn, k, ld, mnt, p.KT)
        ref_u8 = ref.view(np.uint8)
        claims = _ws_u64(ws, off_claim, p.copies * ntiles).reshape(p.copies, ntiles)
        flags = _ws_u64(ws, off_flag, p.copies * ntiles).reshape(p.copies, ntiles)
        assert np.all((claims == epoch).any(axis=0)), f"{which}: a panel was never packed"
        panel_bytes = nk * p.KT * mnt * c.A.itemsize
        for cp in range(p.copies):
            base = off_pack + cp * copy_bytes
            buf = ws[base: base + copy_bytes].cpu().numpy()
            for t_ in range(ntiles):
                if claims[cp, t_] != epoch:
                    continue
                assert flags[cp, t_] == epoch, f"{which} copy {cp} tile {t_} unpublished"
                got = buf[t_ * panel_bytes: (t_ + 1) * panel_bytes]
                exp = ref_u8[t_ * panel_bytes: (t_ + 1) * panel_bytes]
                assert np.array_equal(got, exp), f"{which} copy {cp} tile {t_} differs"


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_standalone_pack_bit_exact(F, dtype):
    say("standalone pack", dtype.__name__)
    for layout, tA, tB, pad in [(COL, "N", "T", 7), (ROW, "T", "N", 0)]:
        c = synth.make_case(layout, 300, 200, 77, tA, tB, ld_pad=pad, dtype=dtype, seed=18)
        out, h = _run_policy(F, c, F.FIP_PACK_CONSUME_ONLY)
        check_full(c, out)
        p = h.last_plan()
        ws = h.workspace
        for X, ld, t, mn, mnt, off, nb, is_b in [
                (c.A, c.lda, tA, c.m, p.MT, p.a_pack_offset, p.a_copy_bytes, 0),
                (c.B, c.ldb, tB, c.n, p.NT, p.b_pack_offset, p.b_copy_bytes, 1)]:
            ref = oracle.pack(X, is_b, layout, t, mn, c.k, ld, mnt, p.KT).view(np.uint8)
            assert ref.size == nb
            assert np.array_equal(ws[off: off + nb].cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_poisoned_and_stale_workspace(F, dtype):
    import torch
    say("poisoned workspace", dtype.__name__)
    h = handle(F, policy=F.FIP_PACK_ALL)
    c1 = synth.make_case(COL, 260, 300, 140, "T", "N", dtype=dtype, seed=21)
    c2 = synth.make_case(ROW, 300, 260, 100, "N", "T", ld_pad=7, dtype=dtype, seed=22)
    dt = F.FIP_F64 if dtype == F64 else F.FIP_F32
    need = max(h.plan(dt, c.layout, c.m, c.n, c.k, c.transA, c.transB).workspace_bytes
               for c in (c1, c2))
    h.ensure_workspace(need)
    check_full(c1, run_gpu(h, c1))
    h.workspace.fill_(0xFF)  # poison: stale flags/claims/panels everywhere
    torch.cuda.synchronize()
    check_full(c2, run_gpu(h, c2))
    check_full(c1, run_gpu(h, c1))  # same workspace, different data and shape again
    c1b = synth.make_case(COL, 260, 300, 140, "T", "N", dtype=dtype, seed=23)
    check_full(c1b, run_gpu(h, c1b))


def test_reuse_statistics(F):
    """With many more tiles than resident workgroups, later tiles find published panels."""
    import torch
    say("stats")
    h = handle(F, policy=F.FIP_PACK_ALL, tile=2)
    h.set_attr(F.FIP_ATTR_STATS, 1)
    c = synth.make_case(COL, 2048, 2048, 256, "N", "N", dtype=F64, seed=5)
    out = run_gpu(h, c)
    p = h.last_plan()
    st = h.workspace[p.stats_offset: p.stats_offset + 24].cpu().numpy().view(np.uint64)
    say("chunks packed / read packed / read unpacked:", st.tolist())
    assert st[0] > 0
    assert st[1] > 0
    check_sampled(c, out, count=1024)


@pytest.mark.parametrize("dtype,n", [(F64, 8192), (F32, 8192), (F64, 4096)],
                         ids=["f64-8192", "f32-8192", "f64-4096"])
def test_large_sampled(F, dtype, n):
    """The benchmark's own launch configuration: sampled exact entries + Freivalds."""
    say("large", dtype.__name__, n)
    c = synth.make_case(COL, n, n, n, "N", "N", alpha=1.5, beta=0.5, dtype=dtype,
                        seed=synth.BASE_SEED + n)
    h = handle(F)
    e = check_sampled(c, run_gpu(h, c))
    say("normalised sampled error", e)
