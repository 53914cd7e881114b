"""GPU parity of the batched binary32 GEMM (one persistent launch over many uneven problems),
its autotuner and its graph replay, against the oracle: every checked problem within
4 k 2^-24 max D; replays bitwise equal to the eager launch."""
import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth

pytestmark = pytest.mark.gpu
COL, ROW = synth.COL, synth.ROW
U = 2.0 ** -24


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2302_08417_amd import fipgemm
    return fipgemm


def say(*a):
    print("[batched]", *a, flush=True)


def check_problem(b, i, got):
    m, n, k = int(b.m[i]), int(b.n[i]), int(b.k[i])
    Cref, D = oracle.gemm(b.layout, m, n, k, b.alpha, b.A[i], int(b.lda[i]), chr(b.transA[i]),
                          b.B[i], int(b.ldb[i]), chr(b.transB[i]), b.beta, b.C[i], int(b.ldc[i]))
    mask = np.zeros(b.C[i].size, bool)
    if m and n:
        ld = int(b.ldc[i])
        v = (mask[: ld * n].reshape(n, ld)[:, :m] if b.layout == COL
             else mask[: ld * m].reshape(m, ld)[:, :n])
        v[:, :] = True
    assert got[~mask].tobytes() == b.C[i][~mask].tobytes(), f"problem {i}: padding modified"
    if not mask.any():
        return 0.0
    err = float(np.abs(got[mask].astype(np.float64) - Cref[mask]).max())
    dmax = float(D[mask].max())
    assert err <= 4 * max(k, 1) * U * dmax, f"problem {i} ({m},{n},{k}): err {err:.3e}"
    return err / (max(k, 1) * U * dmax) if dmax else 0.0


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("pad", [0, 3])
def test_batched_matches_oracle(F, layout, pad):
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("oracle", layout, pad)
    b = synth.make_batch(400, layout, lo=1, hi=300, ld_pad=pad, seed=10 + layout * 2 + pad,
                         zero_sizes=True)
    db = DeviceBatch(b)
    h = F.Handle()
    db.run(h)
    torch.cuda.synchronize()
    worst = max(check_problem(b, i, db.C_host(i)) for i in range(b.count))
    say(f"worst normalised error {worst:.3e}")


@pytest.mark.parametrize("split", [0, 24, 1 << 20])
def test_batched_tile_classes_bitwise(F, split):
    """The tile class changes the blocking, not the k order of any C entry: results of every
    threshold (all 32 x 32, mixed, all 16 x 16) agree bit for bit."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("split", split)
    b = synth.make_batch(300, COL, lo=4, hi=200, seed=33)
    db = DeviceBatch(b)
    h = F.Handle()
    h.set_attr(F.FIP_ATTR_VB_SPLIT, 16)
    db.run(h)
    torch.cuda.synchronize()
    ref = db.C_host().copy()
    db.reset_C()
    h.set_attr(F.FIP_ATTR_VB_SPLIT, split)
    db.run(h)
    torch.cuda.synchronize()
    assert np.array_equal(db.C_host().view(np.uint32), ref.view(np.uint32))
    for i in range(0, b.count, 37):
        check_problem(b, i, db.C_host(i))


def test_batched_graph_replays(F):
    """A graph replay equals the eager launch bit for bit, every time, with eager work and
    synchronisations between the replays."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("graph replay")
    b = synth.make_batch(500, ROW, lo=4, hi=256, seed=44)
    db = DeviceBatch(b)
    h = F.Handle()
    db.run(h)
    torch.cuda.synchronize()
    eager = db.C_host().copy()
    for rep in range(4):
        db.reset_C()                                # eager torch work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        db.run(h, graph=True)
        torch.cuda.synchronize()
        got = db.C_host()
        assert np.array_equal(got.view(np.uint32), eager.view(np.uint32)), f"replay {rep}"
        del junk
    for i in range(0, b.count, 50):
        check_problem(b, i, db.C_host(i))


def test_batched_autotuner(F):
    """The tuner picks a candidate threshold, leaves the real C untouched, and the tuned
    call is right."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("tuner")
    b = synth.make_batch(600, COL, seed=55)
    db = DeviceBatch(b)
    h = F.Handle()
    split = db.tune(h)
    say("tuned split", split)
    assert split in (0, 8, 16, 24, 32, 48, 64, 1 << 30)
    assert np.array_equal(db.C_host().view(np.uint32), db.C0.cpu().numpy().view(np.uint32))
    db.run(h)
    torch.cuda.synchronize()
    for i in range(0, b.count, 7):
        check_problem(b, i, db.C_host(i))


def test_batched_special_cases(F):
    """alpha = 0 reads no A or B (NaN operands), beta = 0 reads no C (NaN C)."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("special")
    b = synth.make_batch(50, COL, lo=1, hi=100, alpha=0.0, beta=0.5, seed=66)
    for x in b.A + b.B:
        x[:] = np.nan
    db = DeviceBatch(b)
    h = F.Handle()
    db.run(h)
    torch.cuda.synchronize()
    for i in range(b.count):
        check_problem(b, i, db.C_host(i))
    b2 = synth.make_batch(50, ROW, lo=1, hi=100, alpha=1.0, beta=0.0, seed=67)
    for x in b2.C:
        x[:] = np.nan
    db2 = DeviceBatch(b2)
    db2.run(h)
    torch.cuda.synchronize()
    for i in range(b2.count):
        got = db2.C_host(i)
        m, n, ld = int(b2.m[i]), int(b2.n[i]), int(b2.ldc[i])
        inside = got[: ld * m].reshape(m, ld)[:, :n] if m and n else got[:0]
        assert np.all(np.isfinite(inside)), i
    # argument errors are reported by position before anything runs
    bad_m = b.m.copy()
    bad_m[3] = -1
    rc = F.fip_sgemm_vbatched(h.h, COL, b.count, bad_m, b.n, b.k, b.transA, b.transB, 1.0,
                              db.A_ptrs, db.lda, db.B_ptrs, db.ldb, 0.0, db.C_ptrs, db.ldc, 0)
    assert rc == 4
    bad_t = b.transA.copy()
    bad_t[0] = ord("x")
    rc = F.fip_sgemm_vbatched(h.h, COL, b.count, b.m, b.n, b.k, bad_t, b.transB, 1.0,
                              db.A_ptrs, db.lda, db.B_ptrs, db.ldb, 0.0, db.C_ptrs, db.ldc, 0)
    assert rc == 7
    assert F.fip_sgemm_vbatched(h.h, COL, b.count, b.m, b.n, b.k, b.transA, b.transB, 1.0,
                                db.A_ptrs, db.lda, db.B_ptrs, db.ldb, 0.0, db.C_ptrs, db.ldc,
                                8) == 17


def test_batched_full_workload_sampled(F):
    """10,000 problems, m, n, k log-uniform in [4, 512], random transposes: one persistent
    launch; 400 problems checked in full against the oracle."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("full workload")
    b = synth.make_batch(10000, COL, lo=4, hi=512, seed=synth.BASE_SEED + 3)
    db = DeviceBatch(b)
    h = F.Handle()
    db.run(h, graph=True)
    torch.cuda.synchronize()
    host = db.C_host()
    pick = synth.rng(9).choice(b.count, 400, replace=False)
    worst = 0.0
    for i in pick:
        got = host[db.c_off[i]: db.c_off[i] + b.C[i].size]
        worst = max(worst, check_problem(b, int(i), got))
    say(f"worst normalised error {worst:.3e}")


def test_batched_invalid_device_leading_dims_are_skipped_and_reported(F):
    """Leading dimensions live in device arrays the host never reads: a problem whose ld is
    below the extent it strides over is not run (its C keeps its bits), the others are
    computed, and FIP_ATTR_VB_STATUS reports 1 + the largest skipped index, then resets."""
    from paper_2302_08417_amd.batched import DeviceBatch
    import torch
    say("invalid device leading dimensions")
    b = synth.make_batch(60, COL, lo=2, hi=80, seed=71)
    db = DeviceBatch(b)
    h = F.Handle()
    bad = {7: "lda", 23: "ldb", 41: "ldc"}
    for i, which in bad.items():
        arr = getattr(db, which)
        arr[i] = 0 if which == "ldc" else 1
    # make sure the shrunk leading dimensions really are too small for their problems
    for i, which in bad.items():
        m, n, k = int(b.m[i]), int(b.n[i]), int(b.k[i])
        need = {"lda": k if chr(b.transA[i]) in "Tt" else m,
                "ldb": n if chr(b.transB[i]) in "Tt" else k, "ldc": m}[which]
        assert need > 1 or which == "ldc", (i, which, need)
    db.run(h)
    torch.cuda.synchronize()
    assert h.get_attr(F.FIP_ATTR_VB_STATUS) == 42
    assert h.get_attr(F.FIP_ATTR_VB_STATUS) == 0
    host = db.C_host()
    for i in range(b.count):
        got = host[db.c_off[i]: db.c_off[i] + b.C[i].size]
        if i in bad:
            assert got.tobytes() == b.C[i].tobytes(), i
        else:
            check_problem(b, i, got)
