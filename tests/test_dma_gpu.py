"""GPU parity of the direct global-to-LDS variant of the tile kernel (FIP_ATTR_DMA).

Launches in which no tile produces a pack and every chunk can be fetched whole (pack-then-
compute's CONSUME_ONLY call; unpacked calls with k a multiple of KT) fetch their chunks with
global_load_lds_dwordx4 instead of through registers (the paper's Sec. 5 footnote: DMA-fed
packing on GPUs).  The elements land in the same LDS places, so C must equal the register
path's bit for bit, and the oracle within the usual tolerance; launches that are not eligible
run the register path whatever the attribute says.
"""
import sys

import numpy as np
import pytest

from gemm_util import check_full, to_dev
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
    print(*a, flush=True)
    sys.stdout.flush()


def run(F, c, policy, dma, tile=-1):
    import torch
    h = F.Handle(policy=policy, tile=tile)
    h.set_attr(F.FIP_ATTR_DMA, dma)
    A, B, C = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    if policy == F.FIP_PACK_CONSUME_ONLY:
        h.pack(c.layout, c.m, c.n, c.k, A, c.lda, c.transA, B, c.ldb, c.transB)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta, C,
           c.ldc)
    torch.cuda.synchronize()
    used = h.get_attr(F.FIP_ATTR_LAST_DMA)
    h.close()
    return C.cpu().numpy(), used


CASES = [
    # (layout, m, n, k, tA, tB, pad, tile): k a multiple of 32 (every KT), m and n multiples of
    # the 16-byte vector (fringe tiles read through redirected offsets), several tiles
    (COL, 512, 384, 256, "N", "N", 0, -1),
    (COL, 300, 200, 160, "T", "N", 7, -1),
    (ROW, 260, 516, 96, "N", "T", 0, -1),
    (ROW, 1000, 1000, 512, "T", "T", 4, 0),
    (COL, 96, 160, 64, "N", "T", 0, 2),
    (COL, 200, 136, 128, "N", "N", 0, 1),
]


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}x{c[3]}-{c[4]}{c[5]}-t{c[7]}"
                                             for c in CASES])
def test_dma_matches_register_path_bitwise(F, dtype, case):
    layout, m, n, k, tA, tB, pad, tile = case
    say("dma", dtype.__name__, case)
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, dtype=dtype, seed=m + n + k)
    for policy in (F.FIP_PACK_NONE, F.FIP_PACK_CONSUME_ONLY):
        ref, used0 = run(F, c, policy, 0, tile)
        assert used0 == 0
        check_full(c, ref)
        got, used1 = run(F, c, policy, 1, tile)
        assert used1 == 1, "the launch should have been eligible for the DMA variant"
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), policy


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_ineligible_launches_fall_back(F, dtype):
    """k not a multiple of KT (an unpacked k tail needs zero fill), an m that splits a vector
    of an MN-major operand, and a fused call that packs: all run the register path."""
    for (m, n, k, policy) in [(256, 256, 100, F.FIP_PACK_NONE), (257, 256, 128, F.FIP_PACK_NONE),
                              (256, 256, 128, F.FIP_PACK_ALL)]:
        c = synth.make_case(COL, m, n, k, "N", "N", dtype=dtype, seed=5)
        got, used = run(F, c, policy, 1)
        assert used == 0, (m, n, k, policy)
        check_full(c, got)


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
def test_dma_large_sampled(F, dtype):
    """2048 x 2048 x 1024 through the DMA variant (AUTO plans no packs here): sampled oracle
    entries plus a Freivalds probe."""
    from gemm_util import check_sampled
    c = synth.make_case(COL, 2048, 2048, 1024, "N", "N", dtype=dtype, seed=3)
    got, used = run(F, c, F.FIP_PACK_AUTO, 1)
    assert used == 1
    check_sampled(c, got, count=2048)


def test_default_picks_binary64_unpacked(F):
    """FIP_ATTR_DMA = -1 (the default): eligible binary64 launches that read their operands
    unpacked take the DMA variant; binary32 launches and pack-then-compute consumers do not."""
    for dtype, policy, want in [(F64, F.FIP_PACK_NONE, 1), (F64, F.FIP_PACK_AUTO, 1),
                                (F64, F.FIP_PACK_CONSUME_ONLY, 0), (F32, F.FIP_PACK_NONE, 0)]:
        c = synth.make_case(COL, 512, 512, 256, "N", "N", dtype=dtype, seed=11)
        got, used = run(F, c, policy, -1)
        assert used == want, (dtype, policy)
        check_full(c, got)
