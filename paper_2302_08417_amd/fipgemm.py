"""Thin Python binding of libfipgemm.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch is used only to own device
memory (tensors' data pointers) and to supply the HIP stream.  If the shared
object is missing this module raises at import time: there is no fallback.

The functions keep the C names and argument order of include/fipgemm.h.
Matrix arguments may be torch tensors (their data_ptr() is passed) or plain
integer device addresses.
"""
import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfipgemm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "fipgemm.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2302_08417_amd.build`")

# The library and PyTorch must share one HIP runtime.  PyTorch ships its own
# libamdhip64; loading it first makes the library's libamdhip64 dependency
# resolve to that copy.  Loaded the other way round, the process ends up with
# two runtimes, and the library's reports no device (hipErrorNoDevice) once
# PyTorch's has opened the GPU.
import torch  # noqa: E402,F401  (load order only)

_lib = ctypes.CDLL(LIB_PATH)

FIP_COL_MAJOR, FIP_ROW_MAJOR = 0, 1
FIP_F64, FIP_F32, FIP_BF16, FIP_E4M3, FIP_BF16X3, FIP_BF16X3_FAST = 0, 1, 2, 3, 4, 5
FIP_C128, FIP_C64 = 6, 7
MX_FORMS = (FIP_BF16, FIP_E4M3, FIP_BF16X3, FIP_BF16X3_FAST)
FIP_ERR_HANDLE, FIP_ERR_WORKSPACE, FIP_ERR_LAUNCH, FIP_ERR_UNSUPPORTED, FIP_ERR_ALLOC = -1, -2, -3, -4, -5
FIP_ATTR_PACK_POLICY, FIP_ATTR_TILE, FIP_ATTR_NO_PUBLISH, FIP_ATTR_STATS, FIP_ATTR_EPOCH = 1, 2, 3, 4, 5
FIP_ATTR_ORDER = 7
FIP_ATTR_VB_SPLIT = 8
FIP_ATTR_VB_GRID = 9
FIP_ATTR_MX_TILE = 10
FIP_ATTR_SPLIT_K = 11
FIP_ATTR_LAST_HIP_ERROR = 12
FIP_ATTR_VB_STATUS = 13
FIP_ATTR_COPIES = 14
FIP_ATTR_DMA = 15
FIP_ATTR_LAST_DMA = 16
FIP_VB_GRAPH = 1
FIP_PACK_AUTO, FIP_PACK_ALL, FIP_PACK_NONE, FIP_PACK_CONSUME_ONLY = 0, 1, 2, 3
COPIES = 8
SCRATCH_BYTES = 64 << 20   # fip_dgemm_noalloc's scratch array per GPU


class fip_plan_t(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
        ("MT", ctypes.c_int32), ("NT", ctypes.c_int32), ("KT", ctypes.c_int32),
        ("tiles_m", ctypes.c_int32), ("tiles_n", ctypes.c_int32), ("ksteps", ctypes.c_int32),
        ("tile_class", ctypes.c_int32),
        ("pack_a", ctypes.c_int32), ("pack_b", ctypes.c_int32),
        ("copies", ctypes.c_int32), ("policy", ctypes.c_int32),
        ("a_kmajor", ctypes.c_int32), ("b_kmajor", ctypes.c_int32),
        ("a_pack_offset", ctypes.c_int64), ("a_copy_bytes", ctypes.c_int64),
        ("b_pack_offset", ctypes.c_int64), ("b_copy_bytes", ctypes.c_int64),
        ("a_flag_offset", ctypes.c_int64), ("b_flag_offset", ctypes.c_int64),
        ("a_claim_offset", ctypes.c_int64), ("b_claim_offset", ctypes.c_int64),
        ("stats_offset", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("split_k", ctypes.c_int32), ("slice_ksteps", ctypes.c_int32),
        ("partial_offset", ctypes.c_int64),
        ("a_pack_first", ctypes.c_int32), ("b_pack_first", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_vp, _i64, _i32, _ch = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_char
_SIGS = {
    "fip_create": [ctypes.POINTER(_vp)],
    "fip_destroy": [_vp],
    "fip_set_stream": [_vp, _vp],
    "fip_set_attr": [_vp, _i32, _i64],
    "fip_get_attr": [_vp, _i32, ctypes.POINTER(_i64)],
    "fip_set_workspace": [_vp, _vp, ctypes.c_size_t],
    "fip_plan": [_vp, _i32, _i32, _i64, _i64, _i64, _ch, _ch, ctypes.POINTER(fip_plan_t)],
    "fip_last_plan": [_vp, ctypes.POINTER(fip_plan_t)],
    "fip_dgemm": [_vp, _i32, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _ch, _vp, _i64, _ch,
                  ctypes.c_double, _vp, _i64],
    "fip_dgemm_noalloc": [_vp, _i32, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _ch, _vp, _i64,
                          _ch, ctypes.c_double, _vp, _i64],
    "fip_sgemm": [_vp, _i32, _i64, _i64, _i64, ctypes.c_float, _vp, _i64, _ch, _vp, _i64, _ch,
                  ctypes.c_float, _vp, _i64],
    "fip_dgemm_tune": [_vp, _i32, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _ch, _vp, _i64,
                       _ch, ctypes.c_double, _vp, _i64, _vp, _vp],
    "fip_sgemm_tune": [_vp, _i32, _i64, _i64, _i64, ctypes.c_float, _vp, _i64, _ch, _vp, _i64,
                       _ch, ctypes.c_float, _vp, _i64, _vp, _vp],
    "fip_tune_save": [_vp, ctypes.c_char_p],
    "fip_tune_load": [_vp, ctypes.c_char_p],
    "fip_zgemm": [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _i64, _ch, _vp, _i64, _ch, _vp, _vp,
                  _i64],
    "fip_cgemm": [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _i64, _ch, _vp, _i64, _ch, _vp, _vp,
                  _i64],
    "fip_pack": [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _ch, _vp, _i64, _ch],
    "fip_xcc_map": [_vp, _vp, _i64],
    "fip_dsyrk": [_vp, _i32, _ch, _ch, _i64, _i64, ctypes.c_double, _vp, _i64, ctypes.c_double,
                  _vp, _i64],
    "fip_ssyrk": [_vp, _i32, _ch, _ch, _i64, _i64, ctypes.c_float, _vp, _i64, ctypes.c_float,
                  _vp, _i64],
    "fip_dtrmm": [_vp, _i32, _ch, _ch, _ch, _ch, _i64, _i64, ctypes.c_double, _vp, _i64, _vp,
                  _i64, ctypes.c_double, _vp, _i64],
    "fip_strmm": [_vp, _i32, _ch, _ch, _ch, _ch, _i64, _i64, ctypes.c_float, _vp, _i64, _vp,
                  _i64, ctypes.c_float, _vp, _i64],
    "fip_dtrsm": [_vp, _i32, _ch, _ch, _ch, _ch, _i64, _i64, ctypes.c_double, _vp, _i64, _vp,
                  _i64],
    "fip_strsm": [_vp, _i32, _ch, _ch, _ch, _ch, _i64, _i64, ctypes.c_float, _vp, _i64, _vp,
                  _i64],
    "fip_plan_l3": [_vp, _i32, _i32, _i32, _ch, _ch, _ch, _ch, _i64, _i64, _i64,
                    ctypes.POINTER(fip_plan_t)],
    "fip_tile_map": [_i64, _i64, _i32, _vp, _vp],
    "fip_gemm_mx": [_vp, _i32, _i32, _i64, _i64, _i64, ctypes.c_float, _vp, _i64, _ch, _vp, _i64,
                    _ch, ctypes.c_float, _vp, _i64, _i32, _vp, _vp],
    "fip_quantize_fp8": [_vp, _i32, _i64, _i64, _vp, _i64, _i32, _vp, _i64, _vp],
    "fip_vbatched_workspace": [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(ctypes.c_size_t)],
    "fip_sgemm_vbatched": [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, _vp, _vp,
                           _vp, _vp, ctypes.c_float, _vp, _vp, _i32],
    "fip_vbatched_tune": [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, _vp, _vp,
                          _vp, _vp, ctypes.c_float, _vp, _vp, ctypes.POINTER(_i32)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int


def header_symbols():
    """Names of the entry points include/fipgemm.h declares."""
    with open(HEADER) as f:
        return re.findall(r"^int\s+(fip_\w+)\s*\(", f.read(), flags=re.M)


class FipError(RuntimeError):
    def __init__(self, func, code, hip_error=None):
        extra = f" (hipError_t {hip_error})" if hip_error else ""
        super().__init__(f"{func} returned {code}{extra}")
        self.func, self.code, self.hip_error = func, code, hip_error


def _addr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _trans(t):
    return t.encode() if isinstance(t, str) else bytes([t]) if isinstance(t, int) else t


# ---- raw entry points (return the C code) ---------------------------------------------

def fip_create():
    h = _vp()
    rc = _lib.fip_create(ctypes.byref(h))
    return rc, h


def fip_destroy(h):
    return _lib.fip_destroy(h)


def fip_set_stream(h, stream):
    return _lib.fip_set_stream(h, _addr(stream))


def fip_set_attr(h, attr, value):
    return _lib.fip_set_attr(h, attr, value)


def fip_get_attr(h, attr):
    v = _i64()
    rc = _lib.fip_get_attr(h, attr, ctypes.byref(v))
    return rc, v.value


def fip_set_workspace(h, ptr, nbytes):
    return _lib.fip_set_workspace(h, _addr(ptr), nbytes)


def fip_plan(h, dtype, layout, m, n, k, transA, transB):
    p = fip_plan_t()
    rc = _lib.fip_plan(h, dtype, layout, m, n, k, _trans(transA), _trans(transB), ctypes.byref(p))
    return rc, p


def fip_last_plan(h):
    p = fip_plan_t()
    rc = _lib.fip_last_plan(h, ctypes.byref(p))
    return rc, p


def fip_dgemm(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    return _lib.fip_dgemm(h, layout, m, n, k, alpha, _addr(A), lda, _trans(transA), _addr(B), ldb,
                          _trans(transB), beta, _addr(C), ldc)


def fip_dgemm_noalloc(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    return _lib.fip_dgemm_noalloc(h, layout, m, n, k, alpha, _addr(A), lda, _trans(transA),
                                  _addr(B), ldb, _trans(transB), beta, _addr(C), ldc)


def fip_sgemm(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    return _lib.fip_sgemm(h, layout, m, n, k, alpha, _addr(A), lda, _trans(transA), _addr(B), ldb,
                          _trans(transB), beta, _addr(C), ldc)


def _tune(fn, h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    tile, split = ctypes.c_int(-2), ctypes.c_int(-2)
    rc = fn(h, layout, m, n, k, alpha, _addr(A), lda, _trans(transA), _addr(B), ldb,
            _trans(transB), beta, _addr(C), ldc, ctypes.byref(tile), ctypes.byref(split))
    return rc, tile.value, split.value


def fip_dgemm_tune(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    """Returns (rc, tile class, split): see the header."""
    return _tune(_lib.fip_dgemm_tune, h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB,
                 beta, C, ldc)


def fip_sgemm_tune(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    return _tune(_lib.fip_sgemm_tune, h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB,
                 beta, C, ldc)


def _path(path):
    return None if path is None else os.fsencode(path)


def fip_tune_save(h, path):
    return _lib.fip_tune_save(h, _path(path))


def fip_tune_load(h, path):
    return _lib.fip_tune_load(h, _path(path))


def _pair(z, ctype):
    """A host (re, im) pair for a complex scalar argument (kept alive by the caller)."""
    z = complex(z)
    return (ctype * 2)(z.real, z.imag)


def fip_zgemm(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    """Complex binary64 GEMM; alpha, beta: Python complex numbers (passed as host pairs)."""
    al, be = _pair(alpha, ctypes.c_double), _pair(beta, ctypes.c_double)
    return _lib.fip_zgemm(h, layout, m, n, k, ctypes.addressof(al), _addr(A), lda, _trans(transA),
                          _addr(B), ldb, _trans(transB), ctypes.addressof(be), _addr(C), ldc)


def fip_cgemm(h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
    al, be = _pair(alpha, ctypes.c_float), _pair(beta, ctypes.c_float)
    return _lib.fip_cgemm(h, layout, m, n, k, ctypes.addressof(al), _addr(A), lda, _trans(transA),
                          _addr(B), ldb, _trans(transB), ctypes.addressof(be), _addr(C), ldc)


def fip_pack(h, dtype, layout, m, n, k, A, lda, transA, B, ldb, transB):
    return _lib.fip_pack(h, dtype, layout, m, n, k, _addr(A), lda, _trans(transA), _addr(B), ldb,
                         _trans(transB))


FIP_OP_SYRK, FIP_OP_TRMM, FIP_OP_TRSM = 1, 2, 3


def fip_dsyrk(h, layout, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    return _lib.fip_dsyrk(h, layout, _trans(uplo), _trans(trans), n, k, alpha, _addr(A), lda,
                          beta, _addr(C), ldc)


def fip_ssyrk(h, layout, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    return _lib.fip_ssyrk(h, layout, _trans(uplo), _trans(trans), n, k, alpha, _addr(A), lda,
                          beta, _addr(C), ldc)


def fip_dtrmm(h, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb, beta, C, ldc):
    return _lib.fip_dtrmm(h, layout, _trans(side), _trans(uplo), _trans(transA), _trans(diag), m,
                          n, alpha, _addr(A), lda, _addr(B), ldb, beta, _addr(C), ldc)


def fip_strmm(h, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb, beta, C, ldc):
    return _lib.fip_strmm(h, layout, _trans(side), _trans(uplo), _trans(transA), _trans(diag), m,
                          n, alpha, _addr(A), lda, _addr(B), ldb, beta, _addr(C), ldc)


def fip_dtrsm(h, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb):
    return _lib.fip_dtrsm(h, layout, _trans(side), _trans(uplo), _trans(transA), _trans(diag), m,
                          n, alpha, _addr(A), lda, _addr(B), ldb)


def fip_strsm(h, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb):
    return _lib.fip_strsm(h, layout, _trans(side), _trans(uplo), _trans(transA), _trans(diag), m,
                          n, alpha, _addr(A), lda, _addr(B), ldb)


def fip_plan_l3(h, op, dtype, layout, side, uplo, trans, diag, m, n, k):
    p = fip_plan_t()
    rc = _lib.fip_plan_l3(h, op, dtype, layout, _trans(side), _trans(uplo), _trans(trans),
                          _trans(diag), m, n, k, ctypes.byref(p))
    return rc, p


def fip_tile_map(tiles_m, tiles_n, order):
    """(rc, tm, tn): the workgroup -> tile map of a launch (host NumPy int32 arrays)."""
    import numpy as np
    T = max(tiles_m * tiles_n, 0)
    tm = np.zeros(max(T, 1), dtype=np.int32)
    tn = np.zeros(max(T, 1), dtype=np.int32)
    rc = _lib.fip_tile_map(tiles_m, tiles_n, order, tm.ctypes.data, tn.ctypes.data)
    return rc, tm[:T], tn[:T]


def fip_xcc_map(h, out, nblocks):
    return _lib.fip_xcc_map(h, _addr(out), nblocks)


def fip_gemm_mx(h, dtype, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc,
                c_type, a_scale=None, b_scale=None):
    return _lib.fip_gemm_mx(h, dtype, layout, m, n, k, alpha, _addr(A), lda, _trans(transA),
                            _addr(B), ldb, _trans(transB), beta, _addr(C), ldc, c_type,
                            _addr(a_scale), _addr(b_scale))


def fip_quantize_fp8(h, layout, rows, cols, X, ldx, axis, Q, ldq, scales):
    return _lib.fip_quantize_fp8(h, layout, rows, cols, _addr(X), ldx, axis, _addr(Q), ldq,
                                 _addr(scales))


def _host_ptr(a):
    """Address of a host NumPy array (or None)."""
    return None if a is None else a.ctypes.data


def fip_vbatched_workspace(h, layout, count, m, n, k, transA, transB):
    nbytes = ctypes.c_size_t()
    rc = _lib.fip_vbatched_workspace(h, layout, count, _host_ptr(m), _host_ptr(n), _host_ptr(k),
                                     _host_ptr(transA), _host_ptr(transB), ctypes.byref(nbytes))
    return rc, nbytes.value


def fip_sgemm_vbatched(h, layout, count, m, n, k, transA, transB, alpha, A, lda, B, ldb, beta,
                       C, ldc, flags=0):
    """m, n, k: host int32 arrays; transA/B: host uint8 arrays of b'N'/b'T'; A, B, C: device
    arrays (tensors) of device pointers (int64); lda, ldb, ldc: device int64 arrays."""
    return _lib.fip_sgemm_vbatched(h, layout, count, _host_ptr(m), _host_ptr(n), _host_ptr(k),
                                   _host_ptr(transA), _host_ptr(transB), alpha, _addr(A),
                                   _addr(lda), _addr(B), _addr(ldb), beta, _addr(C), _addr(ldc),
                                   flags)


def fip_vbatched_tune(h, layout, count, m, n, k, transA, transB, alpha, A, lda, B, ldb, beta,
                      C, ldc):
    split = _i32()
    rc = _lib.fip_vbatched_tune(h, layout, count, _host_ptr(m), _host_ptr(n), _host_ptr(k),
                                _host_ptr(transA), _host_ptr(transB), alpha, _addr(A), _addr(lda),
                                _addr(B), _addr(ldb), beta, _addr(C), _addr(ldc),
                                ctypes.byref(split))
    return rc, split.value


# ---- convenience handle (torch owns the workspace and the stream) ----------------------

class Handle:
    """A library handle bound to the current torch stream, with a growable workspace."""

    def __init__(self, policy=FIP_PACK_AUTO, tile=-1):
        rc, self.h = fip_create()
        if rc:
            raise FipError("fip_create", rc)
        self.workspace = None
        self.set_attr(FIP_ATTR_PACK_POLICY, policy)
        self.set_attr(FIP_ATTR_TILE, tile)

    def close(self):
        if self.h:
            fip_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, name, rc):
        if rc != 0:
            hip = None
            if rc == FIP_ERR_LAUNCH:
                grc, v = fip_get_attr(self.h, FIP_ATTR_LAST_HIP_ERROR)
                if grc == 0:
                    hip = int(v)
            raise FipError(name, rc, hip)

    def set_attr(self, attr, value):
        self._check("fip_set_attr", fip_set_attr(self.h, attr, value))

    def get_attr(self, attr):
        rc, v = fip_get_attr(self.h, attr)
        self._check("fip_get_attr", rc)
        return v

    def plan(self, dtype, layout, m, n, k, transA="N", transB="N"):
        rc, p = fip_plan(self.h, dtype, layout, m, n, k, transA, transB)
        self._check("fip_plan", rc)
        return p

    def last_plan(self):
        rc, p = fip_last_plan(self.h)
        self._check("fip_last_plan", rc)
        return p

    def bind_stream(self):
        import torch
        s = torch.cuda.current_stream()
        self._check("fip_set_stream", fip_set_stream(self.h, s.cuda_stream))
        self.stream = s

    def ensure_workspace(self, nbytes):
        """Make sure a workspace of at least nbytes is attached (grows, never shrinks).  A
        replaced workspace is marked as used by the stream the handle last ran on, so the
        caching allocator does not hand its memory out while queued kernels may still use it."""
        import torch
        if nbytes <= 0:
            return
        if self.workspace is None or self.workspace.numel() < nbytes:
            old, s = self.workspace, getattr(self, "stream", None)
            if old is not None and s is not None:
                old.record_stream(s)
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            self._check("fip_set_workspace",
                        fip_set_workspace(self.h, self.workspace.data_ptr(), self.workspace.numel()))

    def attach_workspace(self, tensor):
        self.workspace = tensor
        self._check("fip_set_workspace", fip_set_workspace(self.h, tensor.data_ptr(), tensor.numel()))

    def gemm(self, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
        """Dispatch on C's dtype (float64 -> fip_dgemm, float32 -> fip_sgemm)."""
        import torch
        dt = FIP_F64 if C.dtype == torch.float64 else FIP_F32
        self.bind_stream()   # first: the plan depends on whether the stream is capturing
        p = self.plan(dt, layout, m, n, k, transA, transB)
        self.ensure_workspace(p.workspace_bytes)
        fn = fip_dgemm if dt == FIP_F64 else fip_sgemm
        rc = fn(self.h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc)
        self._check(fn.__name__, rc)

    def tune(self, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
        """fip_dgemm_tune / fip_sgemm_tune by C's dtype, with a workspace large enough for
        every candidate it times; returns (tile class, split).  C is overwritten."""
        import torch
        dt = FIP_F64 if C.dtype == torch.float64 else FIP_F32
        self.bind_stream()
        keep = (self.get_attr(FIP_ATTR_TILE), self.get_attr(FIP_ATTR_SPLIT_K))
        need = 0
        try:
            for tile in range(3):
                for split in (-1, 1):
                    self.set_attr(FIP_ATTR_TILE, tile)
                    self.set_attr(FIP_ATTR_SPLIT_K, split)
                    need = max(need, self.plan(dt, layout, m, n, k, transA, transB).workspace_bytes)
        finally:
            self.set_attr(FIP_ATTR_TILE, keep[0])
            self.set_attr(FIP_ATTR_SPLIT_K, keep[1])
        self.ensure_workspace(need)
        fn = fip_dgemm_tune if dt == FIP_F64 else fip_sgemm_tune
        rc, tile, split = fn(self.h, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta,
                             C, ldc)
        self._check(fn.__name__, rc)
        return tile, split

    def tune_save(self, path):
        self._check("fip_tune_save", fip_tune_save(self.h, path))

    def tune_load(self, path):
        self._check("fip_tune_load", fip_tune_load(self.h, path))

    def zgemm(self, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc):
        """Complex GEMM by C's dtype (complex128 -> fip_zgemm, complex64 -> fip_cgemm)."""
        import torch
        dt = FIP_C128 if C.dtype == torch.complex128 else FIP_C64
        self.bind_stream()
        p = self.plan(dt, layout, m, n, k, transA, transB)
        self.ensure_workspace(p.workspace_bytes)
        fn = fip_zgemm if dt == FIP_C128 else fip_cgemm
        self._check(fn.__name__, fn(self.h, layout, m, n, k, alpha, A, lda, transA, B, ldb,
                                    transB, beta, C, ldc))

    def gemm_mx(self, dtype, layout, m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C,
                ldc, a_scale=None, b_scale=None):
        """Mixed-precision form dtype (FIP_BF16 .. FIP_BF16X3_FAST); C binary32 or bfloat16."""
        import torch
        c_type = FIP_BF16 if C.dtype == torch.bfloat16 else FIP_F32
        self.bind_stream()   # first: the plan depends on whether the stream is capturing
        p = self.plan(dtype, layout, m, n, k, transA, transB)
        self.ensure_workspace(p.workspace_bytes)
        self._check("fip_gemm_mx", fip_gemm_mx(self.h, dtype, layout, m, n, k, alpha, A, lda,
                                               transA, B, ldb, transB, beta, C, ldc, c_type,
                                               a_scale, b_scale))

    def syrk(self, layout, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
        """fip_dsyrk / fip_ssyrk by C's dtype."""
        import torch
        dt = FIP_F64 if C.dtype == torch.float64 else FIP_F32
        self.bind_stream()
        rc, p = fip_plan_l3(self.h, FIP_OP_SYRK, dt, layout, "L", uplo, trans, "N", n, n, k)
        self._check("fip_plan_l3", rc)
        self.ensure_workspace(p.workspace_bytes)
        fn = fip_dsyrk if dt == FIP_F64 else fip_ssyrk
        self._check(fn.__name__, fn(self.h, layout, uplo, trans, n, k, alpha, A, lda, beta, C, ldc))

    def trmm(self, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb, beta, C, ldc):
        """fip_dtrmm / fip_strmm by C's dtype."""
        import torch
        dt = FIP_F64 if C.dtype == torch.float64 else FIP_F32
        self.bind_stream()
        rc, p = fip_plan_l3(self.h, FIP_OP_TRMM, dt, layout, side, uplo, transA, diag, m, n, 0)
        self._check("fip_plan_l3", rc)
        self.ensure_workspace(p.workspace_bytes)
        fn = fip_dtrmm if dt == FIP_F64 else fip_strmm
        self._check(fn.__name__, fn(self.h, layout, side, uplo, transA, diag, m, n, alpha, A, lda,
                                    B, ldb, beta, C, ldc))

    def trsm(self, layout, side, uplo, transA, diag, m, n, alpha, A, lda, B, ldb):
        """fip_dtrsm / fip_strsm by B's dtype (X overwrites B)."""
        import torch
        dt = FIP_F64 if B.dtype == torch.float64 else FIP_F32
        self.bind_stream()
        rc, p = fip_plan_l3(self.h, FIP_OP_TRSM, dt, layout, side, uplo, transA, diag, m, n, 0)
        self._check("fip_plan_l3", rc)
        self.ensure_workspace(p.workspace_bytes)
        fn = fip_dtrsm if dt == FIP_F64 else fip_strsm
        self._check(fn.__name__, fn(self.h, layout, side, uplo, transA, diag, m, n, alpha, A, lda,
                                    B, ldb))

    def quantize_fp8(self, layout, rows, cols, X, ldx, axis, Q, ldq, scales):
        self.bind_stream()
        self._check("fip_quantize_fp8", fip_quantize_fp8(self.h, layout, rows, cols, X, ldx, axis,
                                                         Q, ldq, scales))

    def pack(self, layout, m, n, k, A, lda, transA, B, ldb, transB, dtype=None):
        import torch
        if dtype is not None:
            dt = dtype
        else:
            dt = {torch.float64: FIP_F64, torch.complex128: FIP_C128,
                  torch.complex64: FIP_C64}.get(A.dtype, FIP_F32)
        old = self.get_attr(FIP_ATTR_PACK_POLICY)
        self.set_attr(FIP_ATTR_PACK_POLICY, FIP_PACK_CONSUME_ONLY)
        p = self.plan(dt, layout, m, n, k, transA, transB)
        self.set_attr(FIP_ATTR_PACK_POLICY, old)
        self.ensure_workspace(p.workspace_bytes)
        self.bind_stream()
        self._check("fip_pack", fip_pack(self.h, dt, layout, m, n, k, A, lda, transA, B, ldb, transB))
