"""torch.autograd.Function over the fused-pack GEMM (forward and both gradients are library
calls in transposed modes; no torch arithmetic).

    C = op(A) @ op(B)                      op(X) = X or X^T (row-major 2-D tensors)
    dA = dC @ op(B)^T   (stored as its transpose when A is used transposed)
    dB = op(A)^T @ dC   (likewise for B)

Each product is one fip_dgemm / fip_sgemm / fip_gemm_mx(FIP_BF16) call on row-major
storage with the transposes expressed through transA / transB, so a transposed operand is
never copied: the first pass over it packs it, later passes read the packed copy (paper
Sec. 3.1-3.2).  bfloat16 tensors use the bfloat16 form with binary32 accumulation and a
bfloat16 result (round to nearest even).  Tensors must be contiguous 2-D CUDA tensors.

    from paper_2302_08417_amd.autograd import fip_matmul, fip_linear
    Y = fip_linear(X, W)            # X @ W^T, as torch.nn.functional.linear without bias
"""
import threading

import torch

from . import fipgemm as F

ROW = F.FIP_ROW_MAJOR
_local = threading.local()
_policy = F.FIP_PACK_AUTO


def set_pack_policy(policy):
    """Packing policy (FIP_PACK_*) of the library handles this module uses (default AUTO)."""
    global _policy
    _policy = policy
    for h in getattr(_local, "handles", {}).values():
        h.set_attr(F.FIP_ATTR_PACK_POLICY, policy)


def _handle():
    """The calling thread's library handle for the current torch stream.  A handle owns one
    workspace (pack panels, flags, split partials), so calls on different streams must not
    share one: each (device, stream) gets its own."""
    s = torch.cuda.current_stream()
    handles = getattr(_local, "handles", None)
    if handles is None:
        handles = _local.handles = {}
    key = (s.device.index, s.cuda_stream)
    h = handles.get(key)
    if h is None:
        h = handles[key] = F.Handle(policy=_policy)
    return h


def _check(t, name):
    if not t.is_cuda or t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D CUDA tensor")
    if t.dtype not in (torch.float64, torch.float32, torch.bfloat16):
        raise TypeError(f"{name}: unsupported dtype {t.dtype}")


def gemm_rowmajor(A, transA, B, transB, m, n, k):
    """C (m x n, new row-major tensor) = op(A) op(B) through the library."""
    C = torch.empty((m, n), dtype=A.dtype, device=A.device)
    if m == 0 or n == 0:
        return C
    h = _handle()
    tA, tB = ("T" if transA else "N"), ("T" if transB else "N")
    lda, ldb = A.shape[1], B.shape[1]
    if A.dtype == torch.bfloat16:
        h.gemm_mx(F.FIP_BF16, ROW, m, n, k, 1.0, A, max(lda, 1), tA, B, max(ldb, 1), tB, 0.0, C,
                  max(n, 1))
    else:
        h.gemm(ROW, m, n, k, 1.0, A, max(lda, 1), tA, B, max(ldb, 1), tB, 0.0, C, max(n, 1))
    return C


class FipMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, transA, transB):
        _check(A, "A")
        _check(B, "B")
        if A.dtype != B.dtype:
            raise TypeError("A and B must have the same dtype")
        m, k = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
        kb, n = (B.shape[1], B.shape[0]) if transB else (B.shape[0], B.shape[1])
        if k != kb:
            raise ValueError(f"inner dimensions differ: {k} vs {kb}")
        ctx.save_for_backward(A, B)
        ctx.transA, ctx.transB = transA, transB
        ctx.mnk = (m, n, k)
        return gemm_rowmajor(A, transA, B, transB, m, n, k)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        transA, transB = ctx.transA, ctx.transB
        m, n, k = ctx.mnk
        dC = dC.contiguous()  # autograd may hand over an expanded or strided gradient
        if dC.dtype != A.dtype:
            raise TypeError("gradient dtype differs from the inputs'")
        dA = dB = None
        if ctx.needs_input_grad[0]:
            if not transA:   # dA (m x k) = dC op(B)^T
                dA = gemm_rowmajor(dC, False, B, not transB, m, k, n)
            else:            # A is k x m: dA = op(B) dC^T
                dA = gemm_rowmajor(B, transB, dC, True, k, m, n)
        if ctx.needs_input_grad[1]:
            if not transB:   # dB (k x n) = op(A)^T dC
                dB = gemm_rowmajor(A, not transA, dC, False, k, n, m)
            else:            # B is n x k: dB = dC^T op(A)
                dB = gemm_rowmajor(dC, True, A, transA, n, k, m)
        return dA, dB, None, None


def fip_matmul(A, B, transA=False, transB=False):
    """op(A) @ op(B) with gradients through the fused-pack GEMM."""
    return FipMatmul.apply(A, B, bool(transA), bool(transB))


def fip_linear(X, W):
    """X @ W^T (X: batch x in, W: out x in), the forward of a bias-free linear layer."""
    return FipMatmul.apply(X, W, False, True)
