"""fip_dgemm_noalloc (the entry point that allocates nothing) against fip_dgemm: two calls in a
row on the library's scratch array, the second smaller, each equal to the workspace entry
point's C bit for bit (same plan, same kernel) and within the oracle's bound; a call whose
packed plan does not fit the array runs unpacked with the same bits; a call whose split-k
partials exceed the array is rejected before anything runs."""
import sys

import numpy as np
import pytest

import oracle  # noqa: F401  (the oracle's bound is checked through gemm_util)
from gemm_util import check_full, check_sampled, to_dev
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
    print("[noalloc]", *a, flush=True)
    sys.stdout.flush()


def _both(F, c, policy, split=-1, copies=-1):
    """C from fip_dgemm (a handle with its own workspace) and from fip_dgemm_noalloc."""
    import torch
    h = F.Handle(policy=policy)
    h.set_attr(F.FIP_ATTR_SPLIT_K, split)
    h.set_attr(F.FIP_ATTR_COPIES, copies)
    A, B = to_dev(c.A), to_dev(c.B)
    C1, C2 = to_dev(c.C), to_dev(c.C)
    h.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta,
           C1, c.ldc)
    plan_ws = h.last_plan()
    h2 = F.Handle(policy=policy)
    h2.set_attr(F.FIP_ATTR_SPLIT_K, split)
    h2.set_attr(F.FIP_ATTR_COPIES, copies)
    h2.bind_stream()
    rc = F.fip_dgemm_noalloc(h2.h, c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B,
                             c.ldb, c.transB, c.beta, C2, c.ldc)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return C1.cpu().numpy(), C2.cpu().numpy(), plan_ws, h2.last_plan()


@pytest.mark.parametrize("policy", [0, 1], ids=["auto", "all"])
def test_noalloc_two_calls_second_smaller(F, policy):
    cases = [synth.make_case(COL, 700, 600, 333, "T", "N", ld_pad=7, alpha=1.5, beta=0.5,
                             dtype=np.float64, seed=81),
             synth.make_case(ROW, 300, 200, 77, "N", "T", ld_pad=0, alpha=-0.5, beta=2.0,
                             dtype=np.float64, seed=82)]
    for i, c in enumerate(cases):
        say("call", i, c.m, c.n, c.k, "policy", policy)
        ref, got, p1, p2 = _both(F, c, policy)
        assert p1.workspace_bytes <= F.SCRATCH_BYTES
        assert (p2.pack_a, p2.pack_b, p2.split_k) == (p1.pack_a, p1.pack_b, p1.split_k)
        if policy == 1:
            assert p2.pack_a and p2.pack_b
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
        check_full(c, got)


def test_noalloc_split_k_then_smaller(F):
    """Split-k partials live in the scratch array: a k-deep skinny call, then a smaller one."""
    cases = [synth.make_case(COL, 32, 2048, 4096, "N", "N", alpha=1.5, beta=0.5,
                             dtype=np.float64, seed=83),
             synth.make_case(COL, 64, 300, 1024, "T", "T", ld_pad=7, alpha=1.0, beta=0.0,
                             dtype=np.float64, seed=84)]
    for i, c in enumerate(cases):
        say("split call", i, c.m, c.n, c.k)
        ref, got, p1, p2 = _both(F, c, 0)
        assert p2.split_k == p1.split_k and (i > 0 or p2.split_k > 1)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
        check_full(c, got)


def test_noalloc_large_call_runs_unpacked_with_same_bits(F):
    """A packed plan larger than the array (pack everything at 4096^2, one copy per XCD) runs
    unpacked: C equals the workspace entry point's bit for bit (the policies share the kernel
    and k order)."""
    n = 4096
    c = synth.make_case(COL, n, n, 512, "N", "N", alpha=1.5, beta=0.5, dtype=np.float64, seed=85)
    say("large", n)
    ref, got, p1, p2 = _both(F, c, 1, copies=8)
    assert p1.workspace_bytes > F.SCRATCH_BYTES
    assert (p2.pack_a, p2.pack_b) == (0, 0)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
    check_sampled(c, got, count=1024)


def test_noalloc_rejects_oversized_split_partials(F):
    import torch
    say("reject")
    h = F.Handle()
    h.set_attr(F.FIP_ATTR_SPLIT_K, 32)
    p = h.plan(F.FIP_F64, COL, 1024, 1024, 8192, "N", "N")
    assert p.split_k > 1 and p.workspace_bytes > F.SCRATCH_BYTES
    C = torch.full((1024 * 1024,), 7.0, dtype=torch.float64, device="cuda")
    A = torch.zeros(1024 * 8192, dtype=torch.float64, device="cuda")
    h.bind_stream()
    rc = F.fip_dgemm_noalloc(h.h, COL, 1024, 1024, 8192, 1.0, A, 1024, "N", A, 8192, "N", 0.0,
                             C, 1024)
    assert rc == F.FIP_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())
    # argument errors are positional, as for fip_dgemm
    assert F.fip_dgemm_noalloc(h.h, COL, -1, 4, 4, 1.0, A, 4, "N", A, 4, "N", 0.0, C, 4) == 3
