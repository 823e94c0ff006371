"""ctypes front end of the C oracle (gemm_oracle.c) -- TEST INFRASTRUCTURE ONLY.

Argument marshalling only: every number is computed by the C routines, which
follow Eq. (1) of the paper (batched C^p <- alpha op(A^p) op(B^p) + beta C^p)
with the element-offset rule of Sec. 5.  See gemm_oracle.c for the definition.
"""
import ctypes
import os

import numpy as np

from . import build as _build

TYPE_CODES = {"f32": 0, "f64": 1, "c64": 2, "c128": 3, "bf16": 4, "f16": 5, "e4m3": 6}
_NP_CODE = {np.dtype(np.float32): 0, np.dtype(np.float64): 1,
            np.dtype(np.complex64): 2, np.dtype(np.complex128): 3}

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        vp, i64p, i32p, dp = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double))
        common = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char, ctypes.c_char,
                  ctypes.c_int64, i32p, i32p, i32p, dp, dp,
                  vp, i64p, i32p, dp, vp, i64p, i32p, dp, vp, i64p, i32p, i64p]
        lib.oracle_gemm.argtypes = common + [dp, dp, ctypes.c_int]
        lib.oracle_gemm.restype = ctypes.c_int
        lib.oracle_gemm_bound.argtypes = common + [dp]
        lib.oracle_gemm_bound.restype = ctypes.c_int
        lib.oracle_quant_e4m3.argtypes = [ctypes.c_int64, i32p, i32p, vp, i64p, i32p, vp, i64p, vp]
        lib.oracle_quant_e4m3.restype = None
        lib.oracle_gemm_split3.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int64, i32p, i32p, i32p,
                                           ctypes.c_double, ctypes.c_double, vp, i64p, i32p, vp, i64p, i32p,
                                           vp, i64p, i32p, i64p, dp, dp, dp]
        lib.oracle_gemm_split3.restype = ctypes.c_int
        lib.oracle_encode_e4m3.argtypes = [ctypes.c_float]
        lib.oracle_encode_e4m3.restype = ctypes.c_uint8
        lib.oracle_round_bf16.argtypes = [ctypes.c_double]
        lib.oracle_round_bf16.restype = ctypes.c_double
        lib.oracle_decode_e4m3.argtypes = [ctypes.c_uint8]
        lib.oracle_decode_e4m3.restype = ctypes.c_double
        lib.oracle_decode_f16.argtypes = [ctypes.c_uint16]
        lib.oracle_decode_f16.restype = ctypes.c_double
        lib.oracle_decode_bf16.argtypes = [ctypes.c_uint16]
        lib.oracle_decode_bf16.restype = ctypes.c_double
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _vptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _per(x, batch, dtype):
    a = np.asarray(x, dtype=dtype)
    if a.ndim == 0:
        a = np.full(batch, a, dtype=dtype)
    assert a.shape == (batch,), (a.shape, batch)
    return np.ascontiguousarray(a)


def _scal(s):
    s = complex(s)
    return np.array([s.real, s.imag], dtype=np.float64)


def _code(arr, code):
    if code is not None:
        return TYPE_CODES[code] if isinstance(code, str) else int(code)
    return _NP_CODE[arr.dtype]


def _marshal(transa, transb, m, n, k, alpha, beta, A, offA, lda, B, offB, ldb, C, offC, ldc,
             scaleA, scaleB, types, batch):
    tA, tB, tC = types
    cplx = tC in (2, 3)
    m_, n_, k_ = (_per(v, batch, np.int32) for v in (m, n, k))
    lda_, ldb_, ldc_ = (_per(v, batch, np.int32) for v in (lda, ldb, ldc))
    offA_, offB_, offC_ = (_per(v, batch, np.int64) for v in (offA, offB, offC))
    cnt = m_.astype(np.int64) * n_
    offO = np.zeros(batch, dtype=np.int64)
    if batch > 1:
        offO[1:] = np.cumsum(cnt)[:-1] * (2 if cplx else 1)
    total = int(cnt.sum()) * (2 if cplx else 1)
    sA = None if scaleA is None else _per(scaleA, batch, np.float64)
    sB = None if scaleB is None else _per(scaleB, batch, np.float64)
    A = None if A is None else np.ascontiguousarray(A)
    B = None if B is None else np.ascontiguousarray(B)
    C = None if C is None else np.ascontiguousarray(C)
    args = [tA, tB, tC, transa.encode(), transb.encode(), batch,
            _ptr(m_, ctypes.c_int32), _ptr(n_, ctypes.c_int32), _ptr(k_, ctypes.c_int32),
            _ptr(_scal(alpha), ctypes.c_double), _ptr(_scal(beta), ctypes.c_double),
            _vptr(A), _ptr(offA_, ctypes.c_int64), _ptr(lda_, ctypes.c_int32), _ptr(sA, ctypes.c_double),
            _vptr(B), _ptr(offB_, ctypes.c_int64), _ptr(ldb_, ctypes.c_int32), _ptr(sB, ctypes.c_double),
            _vptr(C), _ptr(offC_, ctypes.c_int64), _ptr(ldc_, ctypes.c_int32),
            _ptr(offO, ctypes.c_int64)]
    keep = (m_, n_, k_, lda_, ldb_, ldc_, offA_, offB_, offC_, offO, sA, sB, A, B, C)
    return args, keep, offO, total, cplx, m_, n_


def gemm_general(transa, transb, m, n, k, alpha, A, offA, lda, B, offB, ldb, beta, C, offC, ldc,
                 batch, scaleA=None, scaleB=None, types=None, ext=False):
    """Per-matrix sizes / offsets / leading dimensions (scalars broadcast).

    Returns (hi, lo, offO, m, n): flat float64 arrays holding every result
    matrix column-major at offO[p] (complex as re, im pairs); lo is the
    extended-precision residual (zeros when ext is False)."""
    if types is None:
        ref = C if C is not None else (A if A is not None else B)
        types = (_code(A if A is not None else ref, None), _code(B if B is not None else ref, None),
                 _code(ref, None))
    types = tuple(TYPE_CODES[t] if isinstance(t, str) else int(t) for t in types)
    args, keep, offO, total, cplx, m_, n_ = _marshal(
        transa, transb, m, n, k, alpha, beta, A, offA, lda, B, offB, ldb, C, offC, ldc,
        scaleA, scaleB, types, batch)
    hi = np.empty(max(total, 1), dtype=np.float64)
    lo = np.empty(max(total, 1), dtype=np.float64)
    rc = _load().oracle_gemm(*args, _ptr(hi, ctypes.c_double), _ptr(lo, ctypes.c_double), int(bool(ext)))
    del keep
    if rc != 0:
        raise ValueError("oracle_gemm rejected its arguments")
    return hi, lo, offO, m_, n_


def bound_general(transa, transb, m, n, k, alpha, A, offA, lda, B, offB, ldb, beta, C, offC, ldc,
                  batch, scaleA=None, scaleB=None, types=None):
    """Acceptance-test denominators, one float64 per output entry, packed as in
    gemm_general but with one slot per (complex) entry."""
    if types is None:
        ref = C if C is not None else (A if A is not None else B)
        types = (_code(A if A is not None else ref, None), _code(B if B is not None else ref, None),
                 _code(ref, None))
    types = tuple(TYPE_CODES[t] if isinstance(t, str) else int(t) for t in types)
    # bound packing counts entries, so marshal with a real output type
    args, keep, offO, total, _cplx, m_, n_ = _marshal(
        transa, transb, m, n, k, alpha, beta, A, offA, lda, B, offB, ldb, C, offC, ldc,
        scaleA, scaleB, (types[0], types[1], 0), batch)
    args[2] = types[2]
    out = np.empty(max(total, 1), dtype=np.float64)
    rc = _load().oracle_gemm_bound(*args, _ptr(out, ctypes.c_double))
    del keep
    if rc != 0:
        raise ValueError("oracle_gemm_bound rejected its arguments")
    return out, offO


def _unpack_uniform(flat, batch, m, n, cplx):
    if cplx:
        v = flat[: 2 * batch * m * n].reshape(batch, n, m, 2)
        v = v[..., 0] + 1j * v[..., 1]
    else:
        v = flat[: batch * m * n].reshape(batch, n, m)
    return np.ascontiguousarray(np.swapaxes(v, 1, 2))


def gemm_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                 strideC, batch, ext=False, types=None, scaleA=None, scaleB=None):
    """Strided ("second leading dimension") form.  A, B, C are flat storage
    arrays; returns (hi, lo) shaped (batch, m, n), float64 or complex128."""
    p = np.arange(batch, dtype=np.int64)
    hi, lo, _, _, _ = gemm_general(transa, transb, m, n, k, alpha, A, p * strideA, lda,
                                   B, p * strideB, ldb, beta, C, p * strideC, ldc, batch,
                                   scaleA=scaleA, scaleB=scaleB, types=types, ext=ext)
    if types is None:
        ref = C if C is not None else (A if A is not None else B)
        cplx = _code(ref, None) in (2, 3)
    else:
        tc = types[2]
        cplx = (TYPE_CODES[tc] if isinstance(tc, str) else tc) in (2, 3)
    return _unpack_uniform(hi, batch, m, n, cplx), _unpack_uniform(lo, batch, m, n, cplx)


def bound_strided(transa, transb, m, n, k, alpha, A, lda, strideA, B, ldb, strideB, beta, C, ldc,
                  strideC, batch, types=None, scaleA=None, scaleB=None):
    p = np.arange(batch, dtype=np.int64)
    out, _ = bound_general(transa, transb, m, n, k, alpha, A, p * strideA, lda, B, p * strideB, ldb,
                           beta, C, p * strideC, ldc, batch, scaleA=scaleA, scaleB=scaleB, types=types)
    return _unpack_uniform(out, batch, m, n, False)


def gemm(transa, transb, alpha, A, B, beta, C, ext=False):
    """Convenience form on packed batches: A, B, C are numpy arrays shaped
    (batch, rows, cols) holding the STORED matrices (before op); they are laid
    out column-major with minimal leading dimensions and passed to the strided
    routine.  C may be None when beta == 0.  Returns (hi, lo) (batch, m, n)."""
    A = np.asarray(A)
    B = np.asarray(B)
    batch = A.shape[0]
    ra, ca = A.shape[1:]
    rb, cb = B.shape[1:]
    m, k = (ra, ca) if transa in "NnRr" else (ca, ra)
    k2, n = (rb, cb) if transb in "NnRr" else (cb, rb)
    assert k == k2, "inner dimensions differ"
    dt = np.result_type(A.dtype, B.dtype) if C is None else np.asarray(C).dtype

    def colmajor(X):
        return np.ascontiguousarray(np.swapaxes(X, 1, 2)).reshape(-1)

    Af = colmajor(A.astype(dt))
    Bf = colmajor(B.astype(dt))
    Cf = None if C is None else colmajor(np.asarray(C).astype(dt))
    if Cf is None:
        Cf = np.zeros(batch * m * n, dtype=dt)
    return gemm_strided(transa, transb, m, n, k, alpha, Af, max(ra, 1), ra * ca, Bf, max(rb, 1),
                        rb * cb, beta, Cf, max(m, 1), m * n, batch, ext=ext)


def encode_e4m3(v):
    return int(_load().oracle_encode_e4m3(float(v)))


def round_bf16(x):
    return float(_load().oracle_round_bf16(float(x)))


def decode(code, fmt):
    """Value of one stored code: fmt in {'e4m3', 'f16', 'bf16'}."""
    L = _load()
    return float({"e4m3": L.oracle_decode_e4m3, "f16": L.oracle_decode_f16, "bf16": L.oracle_decode_bf16}[fmt](int(code)))


def quant_e4m3(X, offX, rows, cols, ldx, batch):
    """Per-matrix absmax E4M3 quantisation.  X: flat binary32 storage; returns
    (codes, offQ, scales): codes packed column-major per matrix at offQ[p]."""
    rows_ = _per(rows, batch, np.int32)
    cols_ = _per(cols, batch, np.int32)
    ldx_ = _per(ldx, batch, np.int32)
    offX_ = _per(offX, batch, np.int64)
    cnt = rows_.astype(np.int64) * cols_
    offQ = np.zeros(batch, dtype=np.int64)
    if batch > 1:
        offQ[1:] = np.cumsum(cnt)[:-1]
    Q = np.zeros(max(int(cnt.sum()), 1), dtype=np.uint8)
    scales = np.zeros(max(batch, 1), dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    _load().oracle_quant_e4m3(batch, _ptr(rows_, ctypes.c_int32), _ptr(cols_, ctypes.c_int32), _vptr(X),
                              _ptr(offX_, ctypes.c_int64), _ptr(ldx_, ctypes.c_int32), _vptr(Q),
                              _ptr(offQ, ctypes.c_int64), _vptr(scales))
    return Q, offQ, scales[:batch]


def gemm_split3_general(transa, transb, m, n, k, alpha, A, offA, lda, B, offB, ldb, beta, C, offC, ldc, batch):
    """BF16x3 reference on binary32 storage; returns (hi, lo, bound, offO, m, n)
    flat, packed as gemm_general (real)."""
    m_, n_, k_ = (_per(v, batch, np.int32) for v in (m, n, k))
    lda_, ldb_, ldc_ = (_per(v, batch, np.int32) for v in (lda, ldb, ldc))
    offA_, offB_, offC_ = (_per(v, batch, np.int64) for v in (offA, offB, offC))
    cnt = m_.astype(np.int64) * n_
    offO = np.zeros(batch, dtype=np.int64)
    if batch > 1:
        offO[1:] = np.cumsum(cnt)[:-1]
    total = max(int(cnt.sum()), 1)
    hi = np.empty(total)
    lo = np.empty(total)
    bound = np.empty(total)
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32) if C is not None else None
    rc = _load().oracle_gemm_split3(transa.encode(), transb.encode(), batch, _ptr(m_, ctypes.c_int32),
                                    _ptr(n_, ctypes.c_int32), _ptr(k_, ctypes.c_int32), float(alpha), float(beta),
                                    _vptr(A), _ptr(offA_, ctypes.c_int64), _ptr(lda_, ctypes.c_int32),
                                    _vptr(B), _ptr(offB_, ctypes.c_int64), _ptr(ldb_, ctypes.c_int32),
                                    _vptr(C), _ptr(offC_, ctypes.c_int64), _ptr(ldc_, ctypes.c_int32),
                                    _ptr(offO, ctypes.c_int64), _ptr(hi, ctypes.c_double),
                                    _ptr(lo, ctypes.c_double), _ptr(bound, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_gemm_split3 rejected its arguments")
    return hi, lo, bound, offO, m_, n_
