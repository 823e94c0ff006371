"""Python binding of the C-ABI library libsbg.so (include/sbg.h).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the batched GEMM runs in the library's HIP kernels.
There is no CPU or PyTorch fallback -- if the library is missing, load()
raises.

Two call styles:
  * the raw C-ABI names (sbg_sgemm_strided_batched, ...) taking device
    pointers as integers, exposed through `lib()`;
  * tensor helpers (gemm_strided, gemm_batched) that take flat device tensors
    holding column-major batches and pass torch's current stream.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbg.so")

SBG_OK, SBG_INVALID_VALUE, SBG_NOT_SUPPORTED, SBG_HIP_ERROR, SBG_WORKSPACE_TOO_SMALL = range(5)
SCALAR_HOST, SCALAR_DEVICE = 0, 1
R_32F, R_16BF, R_16F, R_8F_E4M3 = range(4)
MODE_PLAIN, MODE_BF16X3 = 0, 1

_PREFIX = {torch.float32: "s", torch.float64: "d", torch.complex64: "c", torch.complex128: "z"}
_REAL = {torch.float32: ctypes.c_float, torch.float64: ctypes.c_double,
         torch.complex64: ctypes.c_float, torch.complex128: ctypes.c_double}

_lib = None

EXPORTS = [
    "sbg_sgemm_strided_batched", "sbg_dgemm_strided_batched",
    "sbg_cgemm_strided_batched", "sbg_zgemm_strided_batched",
    "sbg_sgemm_batched", "sbg_dgemm_batched", "sbg_cgemm_batched", "sbg_zgemm_batched",
    "sbg_set_scalar_mode", "sbg_get_scalar_mode", "sbg_last_invalid_arg",
    "sbg_status_string", "sbg_version", "sbg_describe_strided",
    "sbg_vbatched_workspace_size", "sbg_sgemm_vbatched", "sbg_dgemm_vbatched", "sbg_cgemm_vbatched",
    "sbg_zgemm_vbatched", "sbg_gemm_strided_batched_ex", "sbg_gemm_vbatched_ex",
    "sbg_quantize_e4m3_strided_batched", "sbg_quantize_e4m3_vbatched", "sbg_set_tuning", "sbg_get_tuning",
    "sbg_sgemv_strided_batched", "sbg_dgemv_strided_batched", "sbg_cgemv_strided_batched",
    "sbg_zgemv_strided_batched", "sbg_strsm_strided_batched", "sbg_dtrsm_strided_batched",
    "sbg_ctrsm_strided_batched", "sbg_ztrsm_strided_batched", "sbg_gemm_vbatched_ex_noalloc", "sbg_tuned_table_info",
    "sbg_describe_vbatched", "sbg_sgetrf_strided_batched", "sbg_dgetrf_strided_batched",
]


class SbgError(RuntimeError):
    def __init__(self, status, where, arg=0):
        self.status = status
        self.arg = arg
        msg = f"{where}: status {status} ({_lib.sbg_status_string(status).decode() if _lib else '?'})"
        if status == SBG_INVALID_VALUE:
            msg += f", argument {arg}"
        super().__init__(msg)


def load():
    """Load libsbg.so (built in-tree by the package build step)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_char, i64, vp = ctypes.c_int, ctypes.c_char, ctypes.c_int64, ctypes.c_void_p
    for p in "sdcz":
        f = getattr(lib, f"sbg_{p}gemm_strided_batched")
        f.argtypes = [c_char, c_char, c_int, c_int, c_int, vp, vp, c_int, i64, vp, c_int, i64,
                      vp, vp, c_int, i64, i64, vp]
        f.restype = c_int
        f = getattr(lib, f"sbg_{p}gemm_batched")
        f.argtypes = [c_char, c_char, c_int, c_int, c_int, vp, vp, c_int, vp, c_int, vp, vp, c_int,
                      i64, vp]
        f.restype = c_int
    lib.sbg_set_scalar_mode.argtypes = [c_int]
    lib.sbg_get_scalar_mode.restype = c_int
    lib.sbg_last_invalid_arg.restype = c_int
    lib.sbg_status_string.argtypes = [c_int]
    lib.sbg_status_string.restype = ctypes.c_char_p
    lib.sbg_version.restype = c_int
    lib.sbg_describe_strided.argtypes = [c_char, c_char, c_char, c_int, c_int, c_int, c_int, i64, c_int, i64,
                                         c_int, i64, i64, ctypes.c_char_p, c_int]
    lib.sbg_describe_strided.restype = c_int
    lib.sbg_describe_vbatched.argtypes = [c_char, c_char, c_char, c_int, c_int, c_int, i64, c_int, c_int,
                                          ctypes.c_char_p, c_int]
    lib.sbg_describe_vbatched.restype = c_int
    for p in "sd":
        f = getattr(lib, f"sbg_{p}getrf_strided_batched")
        f.argtypes = [c_int, vp, c_int, i64, vp, i64, vp, i64, vp]
        f.restype = c_int
    for p in "sdcz":
        f = getattr(lib, f"sbg_{p}gemm_vbatched")
        f.argtypes = [c_char, c_char, vp, vp, vp, c_int, c_int, c_int, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp,
                      ctypes.c_size_t, vp]
        f.restype = c_int
    lib.sbg_vbatched_workspace_size.argtypes = [i64]
    lib.sbg_vbatched_workspace_size.restype = ctypes.c_size_t
    lib.sbg_gemm_strided_batched_ex.argtypes = [c_char, c_char, c_int, c_int, c_int, vp, vp, c_int, i64, vp, vp,
                                                c_int, i64, vp, vp, vp, c_int, i64, i64, c_int, c_int, vp]
    lib.sbg_gemm_strided_batched_ex.restype = c_int
    lib.sbg_gemm_vbatched_ex.argtypes = [c_char, c_char, vp, vp, vp, c_int, c_int, c_int, vp, vp, vp, vp, vp, vp,
                                         vp, vp, vp, vp, i64, c_int, c_int, vp, ctypes.c_size_t, vp]
    lib.sbg_gemm_vbatched_ex.restype = c_int
    lib.sbg_gemm_vbatched_ex_noalloc.argtypes = [c_char, c_char, vp, vp, vp, c_int, c_int, c_int, vp, vp, vp, vp,
                                                 vp, vp, vp, vp, vp, vp, i64, c_int, c_int, vp]
    lib.sbg_gemm_vbatched_ex_noalloc.restype = c_int
    lib.sbg_quantize_e4m3_strided_batched.argtypes = [c_int, c_int, vp, c_int, i64, vp, c_int, i64, vp, i64, vp]
    lib.sbg_quantize_e4m3_strided_batched.restype = c_int
    lib.sbg_quantize_e4m3_vbatched.argtypes = [vp, vp, c_int, c_int, vp, vp, vp, vp, vp, i64, vp]
    lib.sbg_quantize_e4m3_vbatched.restype = c_int
    for p in "sdcz":
        f = getattr(lib, f"sbg_{p}gemv_strided_batched")
        f.argtypes = [c_char, c_int, c_int, vp, vp, c_int, i64, vp, c_int, i64, vp, vp, c_int, i64, i64, vp]
        f.restype = c_int
        f = getattr(lib, f"sbg_{p}trsm_strided_batched")
        f.argtypes = [c_char, c_char, c_char, c_char, c_int, c_int, vp, vp, c_int, i64, vp, c_int, i64, i64, vp]
        f.restype = c_int
    lib.sbg_set_tuning.argtypes = [ctypes.c_char_p, c_int]
    lib.sbg_set_tuning.restype = c_int
    lib.sbg_get_tuning.argtypes = [ctypes.c_char_p]
    lib.sbg_get_tuning.restype = c_int
    lib.sbg_tuned_table_info.argtypes = [ctypes.c_char_p, c_int]
    lib.sbg_tuned_table_info.restype = c_int
    _lib = lib
    return lib


def lib():
    return load()


def _scalar_buf(value, dtype):
    """Host buffer holding a scalar in the library's layout (re, im for complex)."""
    rt = _REAL[dtype]
    if dtype.is_complex:
        v = complex(value)
        return (rt * 2)(v.real, v.imag)
    return (rt * 1)(float(value.real if isinstance(value, complex) else value))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _check(status, where):
    if status != SBG_OK:
        raise SbgError(status, where, _lib.sbg_last_invalid_arg())


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def gemm_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                 strideC, batch, stream=None, check=True):
    """C-ABI strided form on flat device tensors (element offsets, column-major).
    alpha/beta are Python scalars (host mode) or 1-element device tensors
    (device mode, switched on for the duration of the call)."""
    L = load()
    dtype = C.dtype
    f = getattr(L, f"sbg_{_PREFIX[dtype]}gemm_strided_batched")
    dev_scalars = isinstance(alpha, torch.Tensor)
    if dev_scalars:
        al, be = ctypes.c_void_p(alpha.data_ptr()), ctypes.c_void_p(beta.data_ptr())
        L.sbg_set_scalar_mode(SCALAR_DEVICE)
    else:
        al, be = _scalar_buf(alpha, dtype), _scalar_buf(beta, dtype)
    try:
        st = f(transa.encode(), transb.encode(), m, n, k, ctypes.cast(al, ctypes.c_void_p) if not dev_scalars else al,
               _dptr(A), lda, strideA, _dptr(B), ldb, strideB,
               ctypes.cast(be, ctypes.c_void_p) if not dev_scalars else be,
               _dptr(C), ldc, strideC, batch, _stream(stream))
    finally:
        if dev_scalars:
            L.sbg_set_scalar_mode(SCALAR_HOST)
    if check:
        _check(st, "gemm_strided")
    return st


def gemm_batched(transa, transb, m, n, k, alpha, Aptrs, lda, Bptrs, ldb, beta, Cptrs, ldc, batch,
                 dtype, stream=None, check=True):
    """C-ABI pointer-array form; Aptrs/Bptrs/Cptrs are int64 device tensors of
    device addresses."""
    L = load()
    f = getattr(L, f"sbg_{_PREFIX[dtype]}gemm_batched")
    al, be = _scalar_buf(alpha, dtype), _scalar_buf(beta, dtype)
    st = f(transa.encode(), transb.encode(), m, n, k, ctypes.cast(al, ctypes.c_void_p),
           _dptr(Aptrs), lda, _dptr(Bptrs), ldb, ctypes.cast(be, ctypes.c_void_p), _dptr(Cptrs), ldc,
           batch, _stream(stream))
    if check:
        _check(st, "gemm_batched")
    return st


def gemv_strided(trans, m, n, alpha, A, lda, strideA, x, incx, stridex, beta, y, incy, stridey, batch,
                 stream=None, check=True):
    """Batched GEMV y_p <- alpha op(A_p) x_p + beta y_p on flat device tensors
    (column-major A, vectors with increments); scalars as in gemm_strided."""
    L = load()
    dtype = y.dtype
    f = getattr(L, f"sbg_{_PREFIX[dtype]}gemv_strided_batched")
    st = _call_scalars(lambda al, be: f(trans.encode(), m, n, al, _dptr(A), lda, strideA, _dptr(x), incx, stridex,
                                        be, _dptr(y), incy, stridey, batch, _stream(stream)),
                       alpha, beta, dtype)
    if check:
        _check(st, "gemv_strided")
    return st


def trsm_strided(side, uplo, transa, diag, m, n, alpha, A, lda, strideA, B, ldb, strideB, batch, stream=None,
                 check=True):
    """Batched TRSM on flat device tensors: side L solves op(A_p) X_p =
    alpha B_p, side R X_p op(A_p) = alpha B_p; X_p overwrites B_p.  alpha is a
    Python scalar (host mode) or a 1-element device tensor (device mode)."""
    L = load()
    dtype = B.dtype
    f = getattr(L, f"sbg_{_PREFIX[dtype]}trsm_strided_batched")
    dev = isinstance(alpha, torch.Tensor)
    if dev:
        al = ctypes.c_void_p(alpha.data_ptr())
        L.sbg_set_scalar_mode(SCALAR_DEVICE)
    else:
        buf = _scalar_buf(alpha, dtype)
        al = ctypes.cast(buf, ctypes.c_void_p)
    try:
        st = f(side.encode(), uplo.encode(), transa.encode(), diag.encode(), m, n, al, _dptr(A), lda, strideA,
               _dptr(B), ldb, strideB, batch, _stream(stream))
    finally:
        if dev:
            L.sbg_set_scalar_mode(SCALAR_HOST)
    if check:
        _check(st, "trsm_strided")
    return st


def _scalars(alpha, beta, dtype):
    """(alpha, beta, device_mode) as ctypes pointers: Python numbers go to host
    buffers, 1-element device tensors are passed as device pointers."""
    if isinstance(alpha, torch.Tensor):
        return ctypes.c_void_p(alpha.data_ptr()), ctypes.c_void_p(beta.data_ptr()), True
    al, be = _scalar_buf(alpha, dtype), _scalar_buf(beta, dtype)
    return al, be, False


def _call_scalars(fn, alpha, beta, dtype, *args):
    """Call fn(alpha_ptr, beta_ptr) with the scalar mode set for the call."""
    L = load()
    al, be, dev = _scalars(alpha, beta, dtype)
    if dev:
        L.sbg_set_scalar_mode(SCALAR_DEVICE)
    try:
        return fn(ctypes.cast(al, ctypes.c_void_p) if not dev else al,
                  ctypes.cast(be, ctypes.c_void_p) if not dev else be)
    finally:
        if dev:
            L.sbg_set_scalar_mode(SCALAR_HOST)


def vbatched_workspace_size(batch):
    return int(load().sbg_vbatched_workspace_size(batch))


def gemm_vbatched(transa, transb, dm, dn, dk, max_m, max_n, max_k, alpha, Aptrs, dlda, Bptrs, dldb, beta, Cptrs,
                  dldc, batch, workspace, dtype, stream=None, check=True):
    """Variable-size form: dm..dldc are int32 device tensors, *ptrs int64
    device tensors of addresses, workspace a device tensor of at least
    vbatched_workspace_size(batch) bytes."""
    L = load()
    f = getattr(L, f"sbg_{_PREFIX[dtype]}gemm_vbatched")
    st = _call_scalars(lambda al, be: f(transa.encode(), transb.encode(), _dptr(dm), _dptr(dn), _dptr(dk), max_m,
                                        max_n, max_k, al, _dptr(Aptrs), _dptr(dlda), _dptr(Bptrs), _dptr(dldb), be,
                                        _dptr(Cptrs), _dptr(dldc), batch, _dptr(workspace),
                                        workspace.numel() * workspace.element_size(), _stream(stream)),
                       alpha, beta, dtype)
    if check:
        _check(st, "gemm_vbatched")
    return st


def gemm_strided_ex(transa, transb, m, n, k, alpha, A, lda, strideA, scaleA, B, ldb, strideB, scaleB, beta, C, ldc,
                    strideC, batch, ab_type, mode=MODE_PLAIN, stream=None, check=True):
    """Mixed-precision strided form (binary32 C); A and B are device tensors of
    the stored type (bf16/fp16 tensors, uint8 for e4m3), scales float32 or None."""
    L = load()
    st = _call_scalars(lambda al, be: L.sbg_gemm_strided_batched_ex(
        transa.encode(), transb.encode(), m, n, k, al, _dptr(A), lda, strideA, _dptr(scaleA), _dptr(B), ldb,
        strideB, _dptr(scaleB), be, _dptr(C), ldc, strideC, batch, ab_type, mode, _stream(stream)),
        alpha, beta, torch.float32)
    if check:
        _check(st, "gemm_strided_ex")
    return st


def gemm_vbatched_ex(transa, transb, dm, dn, dk, max_m, max_n, max_k, alpha, Aptrs, dlda, scaleA, Bptrs, dldb,
                     scaleB, beta, Cptrs, dldc, batch, ab_type, mode, workspace, stream=None, check=True):
    L = load()
    st = _call_scalars(lambda al, be: L.sbg_gemm_vbatched_ex(
        transa.encode(), transb.encode(), _dptr(dm), _dptr(dn), _dptr(dk), max_m, max_n, max_k, al, _dptr(Aptrs),
        _dptr(dlda), _dptr(scaleA), _dptr(Bptrs), _dptr(dldb), _dptr(scaleB), be, _dptr(Cptrs), _dptr(dldc), batch,
        ab_type, mode, _dptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
        alpha, beta, torch.float32)
    if check:
        _check(st, "gemm_vbatched_ex")
    return st


NOALLOC_MAX_BATCH = 262144   # SBG_NOALLOC_MAX_BATCH of include/sbg.h


def gemm_vbatched_ex_noalloc(transa, transb, dm, dn, dk, max_m, max_n, max_k, alpha, Aptrs, dlda, scaleA, Bptrs,
                             dldb, scaleB, beta, Cptrs, dldc, batch, ab_type, mode, stream=None, check=True):
    """sbg_gemm_vbatched_ex without a workspace: the library's own device
    scratch serves as the workspace (no allocation; calls on one GPU must not
    overlap)."""
    L = load()
    st = _call_scalars(lambda al, be: L.sbg_gemm_vbatched_ex_noalloc(
        transa.encode(), transb.encode(), _dptr(dm), _dptr(dn), _dptr(dk), max_m, max_n, max_k, al, _dptr(Aptrs),
        _dptr(dlda), _dptr(scaleA), _dptr(Bptrs), _dptr(dldb), _dptr(scaleB), be, _dptr(Cptrs), _dptr(dldc), batch,
        ab_type, mode, _stream(stream)),
        alpha, beta, torch.float32)
    if check:
        _check(st, "gemm_vbatched_ex_noalloc")
    return st


def quantize_e4m3_strided(rows, cols, X, ldx, strideX, Q, ldq, strideQ, scales, batch, stream=None, check=True):
    st = load().sbg_quantize_e4m3_strided_batched(rows, cols, _dptr(X), ldx, strideX, _dptr(Q), ldq, strideQ,
                                                  _dptr(scales), batch, _stream(stream))
    if check:
        _check(st, "quantize_e4m3_strided")
    return st


def quantize_e4m3_vbatched(drows, dcols, max_rows, max_cols, Xptrs, dldx, Qptrs, dldq, scales, batch, stream=None,
                           check=True):
    st = load().sbg_quantize_e4m3_vbatched(_dptr(drows), _dptr(dcols), max_rows, max_cols, _dptr(Xptrs),
                                           _dptr(dldx), _dptr(Qptrs), _dptr(dldq), _dptr(scales), batch,
                                           _stream(stream))
    if check:
        _check(st, "quantize_e4m3_vbatched")
    return st


def getrf_strided(n, A, lda, strideA, ipiv, strideP, info, batch, stream=None, check=True):
    """Batched LU with partial pivoting of the n x n matrices A_p at
    A + strideA p (float32 or float64 tensor, in place); ipiv and info are
    int32 tensors (1-based interchanges; 0 or the first zero pivot)."""
    p = {torch.float32: "s", torch.float64: "d"}[A.dtype]
    st = getattr(load(), f"sbg_{p}getrf_strided_batched")(n, _dptr(A), lda, strideA, _dptr(ipiv), strideP,
                                                         _dptr(info), batch, _stream(stream))
    if check:
        _check(st, "getrf_strided")
    return st


def describe_vbatched(prefix, transa, transb, max_m, max_n, max_k, batch, ab_type=0, mode=0):
    """What a variable-size call would launch (nothing is launched): a dict
    with "kernel" (demangled symbol), "grid" (work-groups of 4 waves),
    "units" (wave steps; the upper bound for the binned MFMA path, which
    also reports "u16", "u8", "u4"), or None if the call would not launch."""
    buf = ctypes.create_string_buffer(512)
    rc = load().sbg_describe_vbatched(prefix.encode(), transa.encode(), transb.encode(), max_m, max_n, max_k, batch,
                                      ab_type, mode, buf, 512)
    if rc != 0:
        return None
    text = buf.value.decode()
    kernel, _, rest = text.partition(") ")
    out = {"kernel": kernel[len("kernel="):] + ")"}
    for item in rest.split():
        key, _, val = item.partition("=")
        out[key] = int(val)
    return out


def describe_strided(prefix, transa, transb, m, n, k, lda, strideA, ldb, strideB, ldc, strideC, batch):
    """Demangled name of the kernel a strided call with these arguments would
    launch (nothing is launched), or None if the call would not launch."""
    buf = ctypes.create_string_buffer(512)
    rc = load().sbg_describe_strided(prefix.encode(), transa.encode(), transb.encode(), m, n, k, lda, strideA,
                                     ldb, strideB, ldc, strideC, batch, buf, 512)
    return buf.value.decode() if rc == 0 else None


def set_tuning(key, value):
    """Set a launch-tuning knob; returns the previous value."""
    old = load().sbg_set_tuning(key.encode(), int(value))
    if old < 0:
        raise ValueError(f"bad tuning key or value: {key}={value}")
    return old


def get_tuning(key):
    v = load().sbg_get_tuning(key.encode())
    if v < 0:
        raise ValueError(f"unknown tuning key {key}")
    return v


def tuned_table_info():
    """(entry count, description) of the tuned table the library loaded."""
    buf = ctypes.create_string_buffer(1024)
    n = load().sbg_tuned_table_info(buf, len(buf))
    return n, buf.value.decode()


class tuned:
    """Context manager setting tuning knobs for a block: with tuned(staged=1): ..."""

    def __init__(self, **kw):
        self.kw = kw
        self.old = {}

    def __enter__(self):
        for k, v in self.kw.items():
            self.old[k] = set_tuning(k, v)
        return self

    def __exit__(self, *exc):
        for k, v in self.old.items():
            set_tuning(k, v)
        return False


def last_invalid_arg():
    return load().sbg_last_invalid_arg()
