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
        L.oracle_pack_oriented.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ch, i64, i64,
                                           vp, i64, i64, i64, ctypes.c_int, vp]
        L.oracle_pack_oriented.restype = None
        L.oracle_materialize_op.argtypes = [ctypes.c_int, ch, i64, i64, vp, i64, vp]
        L.oracle_materialize_op.restype = None
        L.oracle_mn_contiguous.argtypes = [ctypes.c_int, ctypes.c_int, ch]
        L.oracle_mn_contiguous.restype = ctypes.c_int
        u8p = vp
        L.oracle_bf16_round.argtypes = [vp, i64, vp]
        L.oracle_bf16_round.restype = None
        L.oracle_bf16_decode.argtypes = [vp, i64, vp]
        L.oracle_bf16_decode.restype = None
        L.oracle_split3.argtypes = [vp, i64, vp]
        L.oracle_split3.restype = None
        L.oracle_e4m3_decode.argtypes = [u8p, i64, vp]
        L.oracle_e4m3_decode.restype = None
        L.oracle_e4m3_encode.argtypes = [vp, i64, u8p]
        L.oracle_e4m3_encode.restype = None
        L.oracle_fp8_scale_exponent.argtypes = [dbl]
        L.oracle_fp8_scale_exponent.restype = ctypes.c_int
        L.oracle_quantize_fp8.argtypes = [ctypes.c_int, i64, i64, vp, i64, ctypes.c_int, u8p, i64,
                                          vp]
        L.oracle_quantize_fp8.restype = None
        L.oracle_syrk.argtypes = [ctypes.c_int, ch, ch, i64, i64, dbl, vp, i64, dbl, vp, i64,
                                  vp, vp]
        L.oracle_syrk.restype = None
        L.oracle_trmm.argtypes = [ctypes.c_int, ch, ch, ch, ch, i64, i64, dbl, vp, i64, vp, i64,
                                  dbl, vp, i64, vp, vp]
        L.oracle_trmm.restype = None
        L.oracle_trsm.argtypes = [ctypes.c_int, ch, ch, ch, ch, i64, i64, dbl, vp, i64, vp, i64,
                                  vp, i64]
        L.oracle_trsm.restype = None
        L.oracle_zgemm.argtypes = [ctypes.c_int, i64, i64, i64, dbl, dbl, vp, i64, ch, vp, i64,
                                   ch, dbl, dbl, vp, i64, vp, vp]
        L.oracle_zgemm.restype = None
        L.oracle_zgemm_entries.argtypes = [ctypes.c_int, i64, dbl, dbl, vp, i64, ch, vp, i64, ch,
                                           dbl, dbl, vp, i64, i64, vp, vp, vp, vp]
        L.oracle_zgemm_entries.restype = None
        L.oracle_expand_1m.argtypes = [ctypes.c_int, ctypes.c_int, ch, i64, i64, vp, i64, vp]
        L.oracle_expand_1m.restype = None
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
    need = (ldc * n if layout == COL else ldc * m) if m and n else 0
    if C64.size < need:
        raise ValueError(f"C0 holds {C64.size} entries; the m x n result needs {need}")
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


# ---------------------------------------------------------------------------
# Number formats of the mixed-precision forms (fip_oracle_mx.c)


def bf16_round(x):
    """bfloat16 bits (uint16) of binary32 values, round to nearest even."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))
    out = np.empty(max(x32.size, 1), dtype=np.uint16)
    lib().oracle_bf16_round(_ptr(x32), x32.size, _ptr(out))
    return out[: x32.size]


def bf16_decode(h):
    """binary64 values of bfloat16 bit patterns."""
    h16 = np.ascontiguousarray(np.asarray(h, dtype=np.uint16).reshape(-1))
    out = np.empty(max(h16.size, 1), dtype=np.float64)
    lib().oracle_bf16_decode(_ptr(h16), h16.size, _ptr(out))
    return out[: h16.size]


def split3(x):
    """Three bfloat16 planes (3, n) with x = x0 + x1 + x2 (see fip_oracle_mx.c)."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))
    out = np.empty(max(3 * x32.size, 1), dtype=np.uint16)
    lib().oracle_split3(_ptr(x32), x32.size, _ptr(out))
    return out[: 3 * x32.size].reshape(3, x32.size)


def e4m3_decode(q):
    """binary64 values of OCP FP8 E4M3 codes (NaN codes -> NaN)."""
    q8 = np.ascontiguousarray(np.asarray(q, dtype=np.uint8).reshape(-1))
    out = np.empty(max(q8.size, 1), dtype=np.float64)
    lib().oracle_e4m3_decode(_ptr(q8), q8.size, _ptr(out))
    return out[: q8.size]


def e4m3_encode(x):
    """E4M3 codes of binary64 values: nearest even, saturating at +-448."""
    x64 = _f64(x)
    out = np.empty(max(x64.size, 1), dtype=np.uint8)
    lib().oracle_e4m3_encode(_ptr(x64), x64.size, _ptr(out))
    return out[: x64.size]


def fp8_scale_exponent(amax):
    """e of the line scale 2^e: the largest with amax * 2^e <= 448 (0 for amax == 0)."""
    return int(lib().oracle_fp8_scale_exponent(float(amax)))


def quantize_fp8(layout, rows, cols, X, ld, axis, ldq=None):
    """(Q, scales): X (binary32, stored rows x cols) quantized to E4M3 with a power-of-two
    scale per row (axis 0) or per column (axis 1); Q is stored like X with leading dimension
    ldq (default ld)."""
    ldq = ld if ldq is None else ldq
    X32 = np.ascontiguousarray(np.asarray(X, dtype=np.float32).reshape(-1))
    outer = cols if layout == COL else rows
    Q = np.zeros(max(ldq * outer, 1), dtype=np.uint8)
    sc = np.empty(max(rows if axis == 0 else cols, 1), dtype=np.float32)
    lib().oracle_quantize_fp8(layout, rows, cols, _ptr(X32), ld, axis, _ptr(Q), ldq, _ptr(sc))
    return Q[: ldq * outer], sc[: rows if axis == 0 else cols]


def pack_oriented(X, is_b, layout, trans, mn, k, ld, MNT, KT, kmajor):
    """oracle.pack with the block orientation forced (kmajor 1 / 0) or from storage (-1)."""
    Xc = np.ascontiguousarray(np.asarray(X).reshape(-1))
    nt, nk = -(-mn // MNT), -(-k // KT)
    out = np.empty(max(nt * nk * MNT * KT, 1), dtype=Xc.dtype)
    lib().oracle_pack_oriented(Xc.dtype.itemsize, int(bool(is_b)), layout, _t(trans), mn, k,
                               _ptr(Xc), ld, MNT, KT, int(kmajor), _ptr(out))
    return out[: nt * nk * MNT * KT]


MX_KT = {2: 64, 3: 128, 4: 32, 5: 32}     # k-step of each mixed-precision form
MX_PLANES = {2: 1, 3: 1, 4: 3, 5: 2}


def pack_mx(form, X, is_b, layout, trans, mn, k, ld, MNT=128):
    """Reference pack of a mixed-precision operand as bytes: blocks (tile, k-step), each
    holding PLANES planes of MNT*KT elements in the orientation the operand has in storage
    (as oracle.pack).  bfloat16 / E4M3 operands: their bits; the split forms: the bfloat16
    terms of split3, plane t = term t."""
    KT, PL = MX_KT[form], MX_PLANES[form]
    if PL == 1:
        return pack_oriented(X, is_b, layout, trans, mn, k, ld, MNT, KT, -1).view(np.uint8)
    planes = split3(np.asarray(X, dtype=np.float32))
    packs = [pack_oriented(planes[t], is_b, layout, trans, mn, k, ld, MNT, KT, -1)
             .reshape(-1, MNT * KT) for t in range(PL)]
    return np.stack(packs, axis=1).reshape(-1).view(np.uint8)


def mx_values(form, X, scale=None, scale_axis_len=None):
    """binary64 values of a stored mixed-precision operand buffer (decoded bits; E4M3 codes
    are not divided by their scales here)."""
    if form == 2:
        return bf16_decode(X)
    if form == 3:
        return e4m3_decode(X)
    return np.asarray(X, dtype=np.float64)


# ---------------------------------------------------------------------------
# Other level-3 operations (fip_oracle_l3.c)

def syrk(layout, uplo, trans, n, k, alpha, A, lda, beta, C0, ldc):
    """(Cref, D) in C's storage: the uplo triangle of alpha op(A) op(A)^T + beta C0 (op(A)
    n x k); every other entry of Cref is C0's (binary64), of D zero."""
    A64, C64 = _f64(A), _f64(C0)
    Cref = C64.copy()
    D = np.zeros_like(C64)
    lib().oracle_syrk(layout, _t(uplo), _t(trans), n, k, float(alpha), _ptr(A64), lda,
                      float(beta), _ptr(C64), ldc, _ptr(Cref), _ptr(D))
    return Cref, D


def trmm(layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb, beta, C0, ldc):
    """(Cref, D) in C's storage: alpha op(T) B + beta C0 (side 'L') or alpha B op(T) + beta C0
    (side 'R'), T the uplo triangle of A (unit diagonal for diag 'U'); entries of Cref outside
    the m x n result are C0's."""
    A64, B64, C64 = _f64(A), _f64(B), _f64(C0)
    Cref = C64.copy()
    D = np.zeros_like(C64)
    lib().oracle_trmm(layout, _t(side), _t(uplo), _t(transA), _t(diag), m, n, float(alpha),
                      _ptr(A64), lda, _ptr(B64), ldb, float(beta), _ptr(C64), ldc, _ptr(Cref),
                      _ptr(D))
    return Cref, D


def trsm(layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb):
    """X (binary64, in B's storage with B's ld; entries outside m x n are B's) solving
    op(T) X = alpha B (side 'L') or X op(T) = alpha B (side 'R'), T the uplo triangle of A
    (unit diagonal for diag 'U')."""
    A64, B64 = _f64(A), _f64(B)
    X = B64.copy()
    lib().oracle_trsm(layout, _t(side), _t(uplo), _t(transA), _t(diag), m, n, float(alpha),
                      _ptr(A64), lda, _ptr(B64), ldb, _ptr(X), ldb)
    return X


# ---------------------------------------------------------------------------
# Complex GEMM (fip_oracle_cx.c)

def _c128(x):
    """Interleaved (re, im) binary64 buffer of a complex array (or of interleaved reals)."""
    a = np.asarray(x)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.reshape(-1), dtype=np.complex128).view(np.float64)
    return np.ascontiguousarray(a.reshape(-1), dtype=np.float64)


def zgemm(layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C0, ldc):
    """(Cref, D): Cref complex128 in C's storage (entries outside the m x n result are C0's),
    D binary64, one bound per complex entry (zero outside the result)."""
    A64, B64, C64 = _c128(A), _c128(B), _c128(C0)
    Cref = C64.copy()
    D = np.zeros(C64.size // 2, dtype=np.float64)
    al, be = complex(alpha), complex(beta)
    lib().oracle_zgemm(layout, m, n, k, al.real, al.imag, _ptr(A64), lda, _t(transA), _ptr(B64),
                       ldb, _t(transB), be.real, be.imag, _ptr(C64), ldc, _ptr(Cref), _ptr(D))
    return Cref.view(np.complex128), D


def zgemm_entries(layout, k, alpha, A, lda, transA, B, ldb, transB, beta, C0, ldc, rows, cols):
    """Reference values (complex128) and bounds at the entries (rows[t], cols[t])."""
    A64, B64, C64 = _c128(A), _c128(B), _c128(C0)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(2 * max(r.size, 1), dtype=np.float64)
    d = np.empty(max(r.size, 1), dtype=np.float64)
    al, be = complex(alpha), complex(beta)
    lib().oracle_zgemm_entries(layout, k, al.real, al.imag, _ptr(A64), lda, _t(transA), _ptr(B64),
                               ldb, _t(transB), be.real, be.imag, _ptr(C64), ldc, r.size, _ptr(r),
                               _ptr(c), _ptr(out), _ptr(d))
    return out[: 2 * r.size].view(np.complex128), d[: r.size]


def expand_1m(X, is_b, layout, trans, mn, k, ld):
    """The 1m expansion of op(X) as a real binary64 array: A1e (2mn x 2k) for is_b = 0,
    B1r (2k x mn) for is_b = 1."""
    X64 = _c128(X)
    rows, cols = (2 * mn, 2 * k) if not is_b else (2 * k, mn)
    out = np.empty(max(rows * cols, 1), dtype=np.float64)
    lib().oracle_expand_1m(int(bool(is_b)), layout, _t(trans), mn, k, _ptr(X64), ld, _ptr(out))
    return out[: rows * cols].reshape(cols, rows).T.copy()


def pack_1m(X, is_b, layout, trans, mn, k, ld, MNT, KT, dtype=np.float64):
    """Reference pack of a complex operand for the 1m method: the real tile layout of its
    1m expansion (A1e with MN extent 2mn and k extent 2k; B1r with k extent 2k and MN extent
    mn), each block in the orientation the complex operand has in storage.  Elements are
    converted to dtype (binary32 data widened to binary64 and back is exact)."""
    E = expand_1m(X, is_b, layout, trans, mn, k, ld).astype(dtype)
    kmajor = 0 if mn_contiguous(is_b, layout, trans) else 1
    emn, ek = (2 * mn, 2 * k) if not is_b else (mn, 2 * k)
    # E is column-major op(X1m): rows x cols with op 'N'
    return pack_oriented(E.reshape(-1, order="F"), is_b, COL, "N", emn, ek, E.shape[0], MNT, KT,
                         kmajor)
