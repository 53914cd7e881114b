"""The oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU binary64 reference for the fused-pack GEMM (see fip_oracle.c for
the definition and the paper passages it follows).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The GPU library never imports it and shares no code
with it.

Operands are passed as flat NumPy buffers holding the stored matrices exactly
as the BLAS arguments describe them (layout, trans, ld).  Single-precision
buffers are widened to binary64 first, which is exact.
"""
import ctypes
import os

import numpy as np

from . import build as _build

COL, ROW = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, dbl, ch, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_char, ctypes.c_void_p
        L.oracle_gemm.argtypes = [ctypes.c_int, i64, i64, i64, dbl, vp, i64, ch, vp, i64, ch,
                                  dbl, vp, i64, vp, vp]
        L.oracle_gemm.restype = ctypes.c_int
        L.oracle_gemm_entries.argtypes = [ctypes.c_int, i64, i64, i64, dbl, vp, i64, ch, vp, i64,
                                          ch, dbl, vp, i64, i64, vp, vp, vp, vp]
        L.oracle_gemm_entries.restype = None
        L.oracle_freivalds.argtypes = [ctypes.c_int, i64, i64, i64, dbl, vp, i64, ch, vp, i64, ch,
                                       dbl, vp, i64, vp, vp, vp]
        L.oracle_freivalds.restype = ctypes.c_int
        L.oracle_pack.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ch, i64, i64, vp, i64,
                                  i64, i64, vp]
        L.oracle_pack.restype = None
        L.oracle_materialize_op.argtypes = [ctypes.c_int, ch, i64, i64, vp, i64, vp]
        L.oracle_materialize_op.restype = None
        L.oracle_mn_contiguous.argtypes = [ctypes.c_int, ctypes.c_int, ch]
        L.oracle_mn_contiguous.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads():
    return int(lib().oracle_num_threads())


def _f64(x):
    if x is None:
        return np.zeros(1, dtype=np.float64)
    return np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _t(t):
    return ctypes.c_char(t.encode() if isinstance(t, str) else t)


def gemm(layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C0, ldc):
    """Return (Cref, D) as flat binary64 buffers in C's storage (layout, ldc).

    Entries of the buffer outside the m x n matrix are copied from C0.
    """
    A64, B64, C64 = _f64(A), _f64(B), _f64(C0)
    Cref = C64.copy()
    D = np.zeros_like(C64)
    rc = lib().oracle_gemm(layout, m, n, k, float(alpha), _ptr(A64), lda, _t(transA), _ptr(B64),
                           ldb, _t(transB), float(beta), _ptr(C64), ldc, _ptr(Cref), _ptr(D))
    if rc != 0:
        raise MemoryError("oracle_gemm failed to allocate scratch")
    return Cref, D


def gemm_entries(layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C0, ldc,
                 rows, cols):
    """Reference values and bounds at the entries (rows[t], cols[t])."""
    A64, B64, C64 = _f64(A), _f64(B), _f64(C0)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(r.size, dtype=np.float64)
    d = np.empty(r.size, dtype=np.float64)
    lib().oracle_gemm_entries(layout, m, n, k, float(alpha), _ptr(A64), lda, _t(transA),
                              _ptr(B64), ldb, _t(transB), float(beta), _ptr(C64), ldc, r.size,
                              _ptr(r), _ptr(c), _ptr(out), _ptr(d))
    return out, d


def freivalds(layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C0, ldc, x):
    """(y, bound) with y = alpha*opA*(opB*x) + beta*C0*x, bound its |.| version."""
    A64, B64, C64, x64 = _f64(A), _f64(B), _f64(C0), _f64(x)
    y = np.empty(max(m, 1), dtype=np.float64)
    b = np.empty(max(m, 1), dtype=np.float64)
    rc = lib().oracle_freivalds(layout, m, n, k, float(alpha), _ptr(A64), lda, _t(transA),
                                _ptr(B64), ldb, _t(transB), float(beta), _ptr(C64), ldc,
                                _ptr(x64), _ptr(y), _ptr(b))
    if rc != 0:
        raise MemoryError("oracle_freivalds failed to allocate scratch")
    return y[:m], b[:m]


def materialize_op(layout, trans, rows, cols, X, ld):
    """op(X) as a (rows, cols) binary64 array."""
    X64 = _f64(X)
    out = np.empty(rows * cols if rows * cols else 1, dtype=np.float64)
    lib().oracle_materialize_op(layout, _t(trans), rows, cols, _ptr(X64), ld, _ptr(out))
    return out[: rows * cols].reshape(cols, rows).T.copy()


def mn_contiguous(is_b, layout, trans):
    """True when op(X)'s storage runs along its M (for A) or N (for B) index."""
    return bool(lib().oracle_mn_contiguous(int(bool(is_b)), layout, _t(trans)))


def pack(X, is_b, layout, trans, mn, k, ld, MNT, KT):
    """Reference pack of op(X) into the contiguous tile layout (element bits copied).

    X keeps its own dtype (the pack is a bit copy).  Returns a flat array of
    ceil(mn/MNT)*MNT * ceil(k/KT)*KT elements of X's dtype.
    """
    Xc = np.ascontiguousarray(np.asarray(X).reshape(-1))
    nt, nk = -(-mn // MNT), -(-k // KT)
    out = np.empty(max(nt * nk * MNT * KT, 1), dtype=Xc.dtype)
    lib().oracle_pack(Xc.dtype.itemsize, int(bool(is_b)), layout, _t(trans), mn, k, _ptr(Xc), ld,
                      MNT, KT, _ptr(out))
    return out[: nt * nk * MNT * KT]
