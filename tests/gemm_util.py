"""Helpers for GPU parity tests: run a synth case through the C-ABI, compare with the oracle.

Tolerance (the acceptance bound for floating-point results):
    max_ij |C - Cref|_ij  <=  4 * max(k, 1) * u * max_ij D_ij
with u the unit roundoff of the working precision (2^-53 binary64, 2^-24
binary32) and D = |alpha| |opA| |opB| + |beta| |C0| the oracle's bound.  The
classical dot-product error bound |fl(s) - s| <= gamma_k sum |a||b| (gamma_k =
k u / (1 - k u)) plus the alpha/beta roundings fits inside it.
"""
import numpy as np

import oracle
from paper_2302_08417_amd import synth

U = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}


def torch_dtype(dtype):
    import torch
    return torch.float64 if dtype == np.float64 else torch.float32


def to_dev(buf):
    import torch
    return torch.from_numpy(np.ascontiguousarray(buf)).to("cuda")


def run_gpu(handle, c: synth.GemmCase, C_dev=None):
    """Run the case on the GPU through the C-ABI; returns the whole C buffer (numpy)."""
    import torch
    A = to_dev(c.A)
    B = to_dev(c.B)
    C = to_dev(c.C) if C_dev is None else C_dev
    handle.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb, c.transB, c.beta,
                C, c.ldc)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def c_mask(c):
    """Boolean mask of the m x n entries inside C's buffer."""
    mask = np.zeros(c.C.size, dtype=bool)
    if c.m == 0 or c.n == 0:
        return mask
    if c.layout == synth.COL:
        v = mask[: c.ldc * c.n].reshape(c.n, c.ldc)[:, : c.m]
    else:
        v = mask[: c.ldc * c.m].reshape(c.m, c.ldc)[:, : c.n]
    v[:, :] = True
    return mask


def check_full(c, Cgpu, tol_factor=4.0):
    """Element-by-element check of the whole m x n result against the oracle; returns the
    normalised error max|dC| / (k u max D)."""
    Cref, D = oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                          c.transB, c.beta, c.C, c.ldc)
    mask = c_mask(c)
    # entries outside the m x n matrix must be untouched (bit for bit, NaN padding included)
    outside = ~mask
    assert np.array_equal(Cgpu[outside], c.C[outside], equal_nan=True), "C padding was modified"
    if not mask.any():
        return 0.0
    got = Cgpu[mask].astype(np.float64)
    ref = Cref[mask]
    dmax = float(D[mask].max())
    err = float(np.abs(got - ref).max()) if got.size else 0.0
    u = U[c.dtype]
    kk = max(c.k, 1)
    assert np.all(np.isfinite(got)), "non-finite result"
    bound = tol_factor * kk * u * dmax
    assert err <= bound, f"max err {err:.3e} > bound {bound:.3e} (dmax {dmax:.3e})"
    return err / (kk * u * dmax) if dmax > 0 else 0.0


def check_sampled(c, Cgpu, count=4096, seed=7, tol_factor=4.0):
    """Large sizes: exact oracle values on sampled entries (corners and fringes included)
    plus a Freivalds probe of every row."""
    rows, cols = synth.sample_entries(c.m, c.n, count, seed)
    ref, d = oracle.gemm_entries(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B,
                                 c.ldb, c.transB, c.beta, c.C, c.ldc, rows, cols)
    Cv = synth.op_view(Cgpu, c.layout, "N", c.m, c.n, c.ldc)
    got = Cv[rows, cols].astype(np.float64)
    u = U[c.dtype]
    kk = max(c.k, 1)
    dmax = float(d.max())
    err = float(np.abs(got - ref).max())
    assert err <= tol_factor * kk * u * dmax, f"sampled err {err:.3e}"
    # Freivalds: |C x - y| <= 4 k u bound + the probe's own binary64 rounding
    x = synth.rng(seed + 1).choice([-1.0, 1.0], size=c.n)
    y, bnd = oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B,
                              c.ldb, c.transB, c.beta, c.C, c.ldc, x)
    cx = Cv.astype(np.float64) @ x
    slack = 2.0 * (c.n + c.k + 4) * 2.0 ** -53
    assert np.all(np.abs(cx - y) <= (tol_factor * kk * u + slack) * bnd + 1e-300), "Freivalds"
    return err / (kk * u * dmax)
