"""Marshalling for the batched C-ABI calls (no arithmetic): places a batch's matrices in one
device arena, builds the device arrays of pointers and leading dimensions, and calls
fip_sgemm_vbatched / fip_vbatched_tune.

    db = DeviceBatch(batch)          # batch: synth.Batch (host buffers)
    h = fipgemm.Handle()
    db.run(h)                        # C_i := alpha op(A_i) op(B_i) + beta C_i on the GPU
    db.C_host(i)                     # problem i's C buffer back on the host
"""
import numpy as np
import torch

from . import fipgemm as F


class DeviceBatch:
    ALIGN = 64  # floats (256 bytes) between matrices

    def __init__(self, batch, device="cuda"):
        self.b = batch
        self.count = batch.count

        def arena(bufs):
            offs, total = [], 0
            for x in bufs:
                offs.append(total)
                total += -(-max(x.size, 1) // self.ALIGN) * self.ALIGN
            host = np.zeros(max(total, 1), dtype=np.float32)
            for x, o in zip(bufs, offs):
                host[o: o + x.size] = x
            dev = torch.from_numpy(host).to(device)
            ptrs = torch.tensor([dev.data_ptr() + 4 * o for o in offs], dtype=torch.int64,
                                device=device)
            return dev, np.array(offs, dtype=np.int64), ptrs

        self.A, self.a_off, self.A_ptrs = arena(batch.A)
        self.B, self.b_off, self.B_ptrs = arena(batch.B)
        self.C, self.c_off, self.C_ptrs = arena(batch.C)
        self.C0 = self.C.clone()   # the initial C, to restore between runs
        self.lda = torch.from_numpy(batch.lda).to(device)
        self.ldb = torch.from_numpy(batch.ldb).to(device)
        self.ldc = torch.from_numpy(batch.ldc).to(device)

    def workspace_bytes(self, h):
        b = self.b
        rc, nbytes = F.fip_vbatched_workspace(h.h, b.layout, b.count, b.m, b.n, b.k, b.transA,
                                              b.transB)
        if rc:
            raise F.FipError("fip_vbatched_workspace", rc)
        return nbytes

    def _args(self, C_ptrs=None):
        b = self.b
        return (b.layout, b.count, b.m, b.n, b.k, b.transA, b.transB, b.alpha, self.A_ptrs,
                self.lda, self.B_ptrs, self.ldb, b.beta,
                self.C_ptrs if C_ptrs is None else C_ptrs, self.ldc)

    def run(self, h, graph=False):
        h.ensure_workspace(self.workspace_bytes(h))
        h.bind_stream()
        rc = F.fip_sgemm_vbatched(h.h, *self._args(), F.FIP_VB_GRAPH if graph else 0)
        if rc:
            raise F.FipError("fip_sgemm_vbatched", rc)

    def tune(self, h):
        """Autotune the tile threshold on a scratch copy of C (C itself is left alone)."""
        h.ensure_workspace(self.workspace_bytes(h))
        h.bind_stream()
        scratch = self.C.clone()
        ptrs = self.C_ptrs - self.C.data_ptr() + scratch.data_ptr()
        rc, split = F.fip_vbatched_tune(h.h, *self._args(ptrs))
        torch.cuda.synchronize()
        if rc:
            raise F.FipError("fip_vbatched_tune", rc)
        return split

    def reset_C(self):
        self.C.copy_(self.C0)

    def C_host(self, i=None):
        host = self.C.cpu().numpy()
        if i is None:
            return host
        return host[self.c_off[i]: self.c_off[i] + self.b.C[i].size]
