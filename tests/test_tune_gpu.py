"""GPU tests of the GEMM plan autotuner (fip_dgemm_tune / fip_sgemm_tune) and its persisted
table: the tuned choice is a valid tile class and split, the planner then uses it for that call
shape, the product with it matches the oracle, and a saved table steers a fresh handle the
same way."""
import sys

import numpy as np
import pytest

from gemm_util import check_full, to_dev
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
    print("[tune]", *a, flush=True)
    sys.stdout.flush()


CASES = [(COL, 1000, 1000, 500, "N", "N"), (ROW, 300, 2100, 1500, "T", "N"),
         (COL, 64, 96, 4000, "N", "T")]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}x{c[3]}-{c[4]}{c[5]}"
                                             for c in CASES])
def test_tune_then_gemm(F, dtype, case, tmp_path):
    import torch
    layout, m, n, k, tA, tB = case
    say(dtype.__name__, case)
    c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=3, dtype=dtype, seed=m + 7 * n + k)
    dt = F.FIP_F64 if dtype == np.float64 else F.FIP_F32
    h = F.Handle()
    A, B = to_dev(c.A), to_dev(c.B)
    scratch = to_dev(c.C)
    tile, split = h.tune(layout, m, n, k, c.alpha, A, c.lda, tA, B, c.ldb, tB, c.beta, scratch,
                         c.ldc)
    say("chose tile class", tile, "split", split)
    assert tile in (0, 1, 2) and split in (-1, 1)
    p = h.plan(dt, layout, m, n, k, tA, tB)
    assert p.tile_class == tile
    if split == 1:
        assert p.split_k == 1
    C = to_dev(c.C)
    h.gemm(layout, m, n, k, c.alpha, A, c.lda, tA, B, c.ldb, tB, c.beta, C, c.ldc)
    torch.cuda.synchronize()
    check_full(c, C.cpu().numpy())
    path = tmp_path / "tune.txt"
    h.tune_save(str(path))
    h.close()
    h2 = F.Handle()
    h2.tune_load(str(path))
    p2 = h2.plan(dt, layout, m, n, k, tA, tB)
    assert (p2.tile_class, p2.split_k) == (p.tile_class, p.split_k)
    h2.close()
