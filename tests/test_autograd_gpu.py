"""GPU tests of the autograd Function over the fused-pack GEMM.

- torch.autograd.gradcheck in binary64 on the 64 x 48 x 32 instance (X 64 x 32, W 48 x 32,
  Y = X W^T) and on every transpose combination: the forward and both gradients go through
  fip_dgemm, and GEMM is linear in each argument, so central differences are exact up to
  rounding: the forward's rounding (about u |Y| ~ 2e-15 here) divided by 2 eps (eps = 1e-6)
  is ~1e-9, far inside the tolerances used (atol 1e-7, rtol 1e-6; torch's defaults are
  1e-5 / 1e-3).
- binary32 and bfloat16 gradients against the oracle's binary64 products of the same
  (decoded) inputs, within 4 k u max D (plus the bfloat16 rounding of the result).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def AG():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2302_08417_amd import autograd
    return autograd


def say(*a):
    print("[autograd]", *a, flush=True)


def test_gradcheck_linear_fp64(AG):
    import torch
    say("gradcheck 64x48x32")
    g = torch.Generator(device="cpu").manual_seed(5)
    X = torch.randn(64, 32, generator=g, dtype=torch.float64).cuda().requires_grad_()
    W = torch.randn(48, 32, generator=g, dtype=torch.float64).cuda().requires_grad_()
    assert torch.autograd.gradcheck(AG.fip_linear, (X, W), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gradcheck_matmul_transposes_fp64(AG, tA, tB):
    import torch
    say("gradcheck transposes", tA, tB)
    g = torch.Generator(device="cpu").manual_seed(7 + 2 * tA + tB)
    m, n, k = 37, 29, 41   # ragged: no tile or k-step divides them
    A = torch.randn(*((k, m) if tA else (m, k)), generator=g, dtype=torch.float64).cuda()
    B = torch.randn(*((n, k) if tB else (k, n)), generator=g, dtype=torch.float64).cuda()
    A.requires_grad_()
    B.requires_grad_()
    f = lambda a, b: AG.fip_matmul(a, b, tA, tB)  # noqa: E731
    assert torch.autograd.gradcheck(f, (A, B), eps=1e-6, atol=1e-7, rtol=1e-6)


def _op(x, t):
    return x.T if t else x


def _ref_products(A, B, dC, tA, tB):
    """binary64 oracle values of C = op(A) op(B), dA and dB (same shapes as A, B), and the
    |.| bounds, from numpy arrays already holding the exact input values."""
    def mm(X, Y):
        # row-major X (p x q) and Y (q x r) as column-major transposes: C^T = Y^T X^T
        p, q = X.shape
        r = Y.shape[1]
        Xc = np.ascontiguousarray(X.T).reshape(-1)   # column-major X
        Yc = np.ascontiguousarray(Y.T).reshape(-1)
        C, D = oracle.gemm(0, p, r, q, 1.0, Xc, p, "N", Yc, q, "N", 0.0, np.zeros(p * r), p)
        return C.reshape(r, p).T, D.reshape(r, p).T
    opA, opB = _op(A, tA), _op(B, tB)
    C, Dc = mm(opA, opB)
    dOpA, Da = mm(dC, opB.T)          # d op(A) = dC op(B)^T
    dOpB, Db = mm(opA.T, dC)          # d op(B) = op(A)^T dC
    return (C, Dc), (_op(dOpA, tA), _op(Da, tA)), (_op(dOpB, tB), _op(Db, tB))


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
@pytest.mark.parametrize("tA,tB", [(False, True), (True, False), (False, False), (True, True)])
def test_gradients_match_oracle(AG, dtype, tA, tB):
    import torch
    say("gradients", dtype, tA, tB)
    dt = getattr(torch, dtype)
    g = torch.Generator(device="cpu").manual_seed(11)
    m, n, k = 300, 260, 170
    A = torch.randn(*((k, m) if tA else (m, k)), generator=g).to(dt)
    B = (torch.randn(*((n, k) if tB else (k, n)), generator=g) / 16).to(dt)
    dC = torch.randn(m, n, generator=g).to(dt)
    Ad, Bd = A.cuda().requires_grad_(), B.cuda().requires_grad_()
    C = AG.fip_matmul(Ad, Bd, tA, tB)
    C.backward(dC.cuda())
    refs = _ref_products(A.double().numpy(), B.double().numpy(), dC.double().numpy(), tA, tB)
    u = 2.0 ** -24
    for name, got, (ref, D), kk in [("C", C, refs[0], k), ("dA", Ad.grad, refs[1], n),
                                    ("dB", Bd.grad, refs[2], m)]:
        got = got.detach().double().cpu().numpy()
        err = float(np.abs(got - ref).max())
        bound = 4 * kk * u * float(D.max())
        if dtype == "bfloat16":
            bound += 2.0 ** -8 * float(np.abs(ref).max())
        say(f"{name}: err {err:.3e} bound {bound:.3e}")
        assert got.shape == ref.shape and err <= bound, name


def test_bf16_linear_full_size_sampled(AG):
    """The autograd workload at full size: X 8192 x 4096 ~ N(0,1), W 4096 x 4096 ~
    N(0, 1/4096), dY ~ N(0,1), bfloat16 storage: Y, dX and dW checked on sampled entries
    against the oracle."""
    import torch
    say("bf16 linear 8192x4096x4096")
    g = torch.Generator(device="cuda").manual_seed(3)
    X = torch.randn(8192, 4096, device="cuda", generator=g).to(torch.bfloat16)
    W = (torch.randn(4096, 4096, device="cuda", generator=g) / 64).to(torch.bfloat16)
    dY = torch.randn(8192, 4096, device="cuda", generator=g).to(torch.bfloat16)
    Xr, Wr = X.clone().requires_grad_(), W.clone().requires_grad_()
    Y = AG.fip_linear(Xr, Wr)
    Y.backward(dY)
    torch.cuda.synchronize()
    Xh, Wh, dYh = (t.float().cpu().numpy().astype(np.float64).reshape(-1) for t in (X, W, dY))
    rng = np.random.default_rng(1)
    u = 2.0 ** -24
    ROWM = 1
    zero = np.zeros(1)
    for name, got, args, rows_n, cols_n, kk in [
            ("Y", Y, (Xh, 4096, "N", Wh, 4096, "T"), 8192, 4096, 4096),
            ("dX", Xr.grad, (dYh, 4096, "N", Wh, 4096, "N"), 8192, 4096, 4096),
            ("dW", Wr.grad, (dYh, 4096, "T", Xh, 4096, "N"), 4096, 4096, 8192)]:
        ri = rng.integers(0, rows_n, 256)
        ci = rng.integers(0, cols_n, 256)
        ref, D = oracle.gemm_entries(ROWM, rows_n, cols_n, kk, 1.0, *args, 0.0, zero, cols_n,
                                     ri, ci)
        gv = got.detach().float().cpu().numpy().astype(np.float64)[ri, ci]
        err = float(np.abs(gv - ref).max())
        bound = 4 * kk * u * float(D.max()) + 2.0 ** -8 * float(np.abs(ref).max())
        say(f"{name}: sampled err {err:.3e} bound {bound:.3e}")
        assert err <= bound, name


def test_two_streams_do_not_share_a_workspace(AG):
    """fip_linear on two streams at once, packing forced, in binary32: each stream's calls use
    their own handle and workspace, so the results match the oracle on both (a shared
    workspace would let one stream's pack panels and flags overwrite the other's)."""
    import torch
    from paper_2302_08417_amd import fipgemm as F
    say("two streams, packing forced")
    AG.set_pack_policy(F.FIP_PACK_ALL)
    try:
        g = torch.Generator(device="cpu").manual_seed(13)
        shapes = [(1024, 768, 512), (896, 1024, 640)]   # (batch, out, in): several tile rounds
        Xs = [torch.randn(b, i, generator=g) for b, o, i in shapes]
        Ws = [torch.randn(o, i, generator=g) for b, o, i in shapes]
        dYs = [torch.randn(b, o, generator=g) for b, o, i in shapes]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        torch.cuda.synchronize()
        outs = [None, None]
        for rep in range(3):
            dev = []
            for s, X, W, dY in zip(streams, Xs, Ws, dYs):
                with torch.cuda.stream(s):
                    x = X.cuda().requires_grad_()
                    w = W.cuda().requires_grad_()
                    y = AG.fip_linear(x, w)
                    y.backward(dY.cuda())
                    dev.append((y, x, w))
            torch.cuda.synchronize()
            outs = [(y.detach().cpu(), x.grad.cpu(), w.grad.cpu()) for y, x, w in dev]
            for (Y, dX, dW), X, W, dY in zip(outs, Xs, Ws, dYs):
                for got, a, b, ta, tb in ((Y, X, W, "N", "T"), (dX, dY, W, "N", "N"),
                                          (dW, dY, X, "T", "N")):
                    m, n = got.shape
                    k = a.shape[0] if ta == "T" else a.shape[1]
                    A64 = a.double().numpy().reshape(-1)
                    B64 = b.double().numpy().reshape(-1)
                    ref, D = oracle.gemm(1, m, n, k, 1.0, A64, a.shape[1], ta, B64, b.shape[1],
                                         tb, 0.0, np.zeros(m * n), n)
                    err = np.abs(got.double().numpy().reshape(-1) - ref).max()
                    assert err <= 4 * k * 2.0 ** -24 * D.max(), (rep, m, n, k, err)
        assert len(AG._local.handles) >= 2
    finally:
        AG.set_pack_policy(F.FIP_PACK_AUTO)
