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


# ---------------------------------------------------------------------------
# Mixed-precision forms

MX_KT = {2: 64, 3: 128, 4: 32, 5: 32}
U32 = 2.0 ** -24          # binary32 accumulation
U_BF16 = 2.0 ** -8        # rounding of a bfloat16 C


def mx_effective(form, buf, layout, trans, rows, cols, ld, scale=None, along_rows=True):
    """binary64 buffer of the values a stored mixed-precision operand stands for: decoded
    bits, E4M3 codes divided by their line scale (rows of op(A) / columns of op(B))."""
    vals = oracle.mx_values(form, buf).copy()
    if form == 3 and scale is not None:
        v = synth.op_view(vals, layout, trans, rows, cols, ld)
        if along_rows:
            v /= scale.astype(np.float64)[:, None]
        else:
            v /= scale.astype(np.float64)[None, :]
    return vals


def mx_c0(c):
    return oracle.bf16_decode(c.C) if c.c_bf16 else c.C.astype(np.float64)


def mx_reference(c):
    """(Cref, D) in C's storage: the product of the values the stored operands stand for
    (for the split forms, the sum of the kept term products), in binary64."""
    C0 = mx_c0(c)
    if c.form in (2, 3):
        A = mx_effective(c.form, c.A, c.layout, c.transA, c.m, c.k, c.lda, c.a_scale, True)
        B = mx_effective(c.form, c.B, c.layout, c.transB, c.k, c.n, c.ldb, c.b_scale, False)
        return oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb,
                           c.transB, c.beta, C0, c.ldc)
    pa = oracle.split3(c.A)
    pb = oracle.split3(c.B)
    ta = [oracle.bf16_decode(pa[t]) for t in range(3)]
    tb = [oracle.bf16_decode(pb[t]) for t in range(3)]
    if c.form == 4:   # sum_{i+j<=2} A_i B_j = A0 (B0+B1+B2) + A1 (B0+B1) + A2 B0
        pairs = [(ta[0], tb[0] + tb[1] + tb[2]), (ta[1], tb[0] + tb[1]), (ta[2], tb[0])]
    else:             # sum_{i+j<=1} = A0 (B0+B1) + A1 B0
        pairs = [(ta[0], tb[0] + tb[1]), (ta[1], tb[0])]
    Cref = None
    for idx, (a, b) in enumerate(pairs):
        r, _ = oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, a, c.lda, c.transA, b, c.ldb,
                           c.transB, c.beta if idx == 0 else 0.0, C0, c.ldc)
        Cref = r if Cref is None else Cref + np.where(c_mask(c), r, 0.0)
    _, D = oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A32, c.lda, c.transA, c.B32, c.ldb,
                       c.transB, c.beta, C0, c.ldc)
    return Cref, D


def mx_fp64_truth(c):
    """binary64 product of the binary32 values the operands were made from."""
    return oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A32, c.lda, c.transA, c.B32, c.ldb,
                       c.transB, c.beta, mx_c0(c), c.ldc)[0]


def check_mx(c, Cgpu, tol_factor=4.0):
    """Compare a mixed-precision result with the oracle: max|C - Cref| <= 4 k u32 max D
    (+ u_bf16 max|Cref| when C is stored in bfloat16).  Returns (normalised error, error
    against the binary64 product of the unquantized binary32 values, relative to max D)."""
    Cref, D = mx_reference(c)
    mask = c_mask(c)
    outside = ~mask
    assert Cgpu[outside].tobytes() == c.C[outside].tobytes(), "C padding was modified"
    if not mask.any():
        return 0.0, 0.0
    got = (oracle.bf16_decode(Cgpu) if c.c_bf16 else Cgpu.astype(np.float64))[mask]
    ref = Cref[mask]
    assert np.all(np.isfinite(got)), "non-finite result"
    dmax = float(D[mask].max())
    err = float(np.abs(got - ref).max())
    kk = max(c.k, 1)
    bound = tol_factor * kk * U32 * dmax + (U_BF16 * float(np.abs(ref).max()) if c.c_bf16 else 0)
    assert err <= bound, f"max err {err:.3e} > bound {bound:.3e} (dmax {dmax:.3e})"
    truth = mx_fp64_truth(c)[mask]
    terr = float(np.abs(got - truth).max())
    assert terr <= mx_truth_bound(c, kk, dmax, float(np.abs(ref).max())), \
        f"error vs the binary64 product of the binary32 values {terr:.3e}"
    return err / (kk * U32 * dmax), terr / dmax


# Error of a split form against the binary64 product of the binary32 values it was made from.
# bfloat16 keeps 8 significant bits (unit roundoff 2^-8), and a term x_t is the rounding of
# x - x_0 - ... - x_(t-1), so |x_1| <= 2^-8 |x| (1 + 2^-8) and |x_2| <= 2^-16 |x| (1 + 2^-7).
# Every kept product x_i y_j of two bfloat16 values is exact in binary32.
#   3-term split: x0 + x1 + x2 = x exactly; the dropped x1 y2 + x2 y1 + x2 y2 are at most
#                 (2 * 2^-24 + 2^-32)(1 + 2^-6) |x||y| <= 2^-22 |x||y|;
#   2-term split: the dropped x0 y2 + x2 y0 + x1 y1 + x1 y2 + x2 y1 + x2 y2 are at most
#                 (3 * 2^-16 + 2 * 2^-24 + 2^-32)(1 + 2^-6) |x||y| <= 2^-14 |x||y|.
# Summed over k these are bounded by that factor times D; the binary32 accumulation adds the
# usual 4 k 2^-24 max D.
SPLIT_DROP = {4: 2.0 ** -22, 5: 2.0 ** -14}


def mx_truth_bound(c, kk, dmax, refmax):
    if c.form not in SPLIT_DROP:
        return float("inf")
    bf = U_BF16 * refmax if c.c_bf16 else 0.0
    return (4 * kk * U32 + SPLIT_DROP[c.form]) * dmax + bf


def mx_reference_sampled(c, rows, cols):
    """Oracle values at sampled entries, via a full reference on a row/column subset."""
    sub_r = np.unique(rows)
    sub_c = np.unique(cols)
    opA = synth.op_view(c.A, c.layout, c.transA, c.m, c.k, c.lda)[sub_r, :]
    opB = synth.op_view(c.B, c.layout, c.transB, c.k, c.n, c.ldb)[:, sub_c]
    A32 = synth.op_view(c.A32, c.layout, c.transA, c.m, c.k, c.lda)[sub_r, :]
    B32 = synth.op_view(c.B32, c.layout, c.transB, c.k, c.n, c.ldb)[:, sub_c]
    C0 = synth.op_view(c.C, c.layout, "N", c.m, c.n, c.ldc)[np.ix_(sub_r, sub_c)]
    mm, nn = sub_r.size, sub_c.size
    sub = synth.MxCase(c.form, synth.COL, mm, nn, c.k, "N", "N", mm, c.k, mm, c.alpha, c.beta,
                       np.asfortranarray(opA).reshape(-1, order="F").copy(),
                       np.asfortranarray(opB).reshape(-1, order="F").copy(),
                       np.asfortranarray(C0).reshape(-1, order="F").copy(), c.c_bf16,
                       None if c.a_scale is None else c.a_scale[sub_r],
                       None if c.b_scale is None else c.b_scale[sub_c],
                       np.asfortranarray(A32).reshape(-1, order="F").copy(),
                       np.asfortranarray(B32).reshape(-1, order="F").copy())
    Cref, D = mx_reference(sub)
    truth = mx_fp64_truth(sub)
    ri = np.searchsorted(sub_r, rows)
    ci = np.searchsorted(sub_c, cols)
    pick = lambda X: X.reshape(nn, mm).T[ri, ci]  # noqa: E731
    return pick(Cref), pick(D), pick(truth)


def mx_freivalds(c, x):
    """(y, bound): y = C_ref x for the product the stored operands stand for (the kept term
    products for the split forms), bound = the |.| version on the binary32 values."""
    C0 = mx_c0(c)
    if c.form in (2, 3):
        A = mx_effective(c.form, c.A, c.layout, c.transA, c.m, c.k, c.lda, c.a_scale, True)
        B = mx_effective(c.form, c.B, c.layout, c.transB, c.k, c.n, c.ldb, c.b_scale, False)
        return oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, A, c.lda, c.transA, B, c.ldb,
                                c.transB, c.beta, C0, c.ldc, x)
    pa, pb = oracle.split3(c.A), oracle.split3(c.B)
    ta = [oracle.bf16_decode(pa[t]) for t in range(3)]
    tb = [oracle.bf16_decode(pb[t]) for t in range(3)]
    if c.form == 4:
        pairs = [(ta[0], tb[0] + tb[1] + tb[2]), (ta[1], tb[0] + tb[1]), (ta[2], tb[0])]
    else:
        pairs = [(ta[0], tb[0] + tb[1]), (ta[1], tb[0])]
    y = None
    for idx, (a, b) in enumerate(pairs):
        r, _ = oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, a, c.lda, c.transA, b, c.ldb,
                                c.transB, c.beta if idx == 0 else 0.0, C0, c.ldc, x)
        y = r if y is None else y + r
    _, bnd = oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, c.A32, c.lda, c.transA, c.B32,
                              c.ldb, c.transB, c.beta, C0, c.ldc, x)
    return y, bnd


def check_mx_sampled(c, Cgpu, count=512, seed=11, tol_factor=4.0):
    """Large mixed-precision results: the oracle on sampled entries (corners and fringes
    included) and a Freivalds probe of every row.  Returns (normalised sampled error, sampled
    error against the binary64 product of the binary32 values relative to max D)."""
    assert not c.c_bf16
    rows, cols = synth.sample_entries(c.m, c.n, count, seed)
    ref, d, truth = mx_reference_sampled(c, rows, cols)
    Cv = synth.op_view(Cgpu, c.layout, "N", c.m, c.n, c.ldc)
    got = Cv[rows, cols].astype(np.float64)
    kk = max(c.k, 1)
    dmax = float(d.max())
    err = float(np.abs(got - ref).max())
    assert err <= tol_factor * kk * U32 * dmax, f"sampled err {err:.3e}"
    terr = float(np.abs(got - truth).max())
    assert terr <= mx_truth_bound(c, kk, dmax, float(np.abs(ref).max())), terr
    x = synth.rng(seed + 1).choice([-1.0, 1.0], size=c.n)
    y, bnd = mx_freivalds(c, x)
    cx = Cv.astype(np.float64) @ x
    slack = 2.0 * (c.n + c.k + 4) * 2.0 ** -53
    assert np.all(np.abs(cx - y) <= (tol_factor * kk * U32 + slack) * bnd + 1e-300), "Freivalds"
    return err / (kk * U32 * dmax), terr / dmax
