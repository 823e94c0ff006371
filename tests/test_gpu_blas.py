"""Batched GEMV and TRSM in the strided interface (the paper's proposal to
carry its interface over to other BLAS routines, formulated on batched GEMM):
GPU parity through the C-ABI against oracle/blas.py.

GEMV: |y - yref| / (|alpha| (|op A||x|) + |beta||y_in|) <= 4 max(k,1) u, as
for GEMM (k = length of x).  TRSM: the componentwise backward error
|op(A) X - alpha B| / (|op(A)||X| + |alpha B|) (X op(A) for side R) is at most
4 (s + 1) u for real and 8 (s + 1) u for complex types, s the triangular
order -- substitution's backward error is about s u -- and on the
well-conditioned systems used here the solution also agrees with the
oracle's to 64 (s + 1) u relative to its largest entry."""
import numpy as np
import pytest
import torch

from oracle import blas
from paper_1304_7053_amd import inputs, sbg
from gpu_util import TORCH, from_dev, say, to_dev, unit
import test_gpu_parity as P

pytestmark = pytest.mark.gpu


def _vec_case(g, dtype, trans, m, n, incx, incy, batch, pad=2):
    rows, cols = (m, n) if trans == "N" else (n, m)
    lda = max(m, 1) + 1
    sA = lda * n + pad
    sx = incx * cols + pad
    sy = incy * rows + pad
    A = inputs.uniform(g, (batch * sA,), dtype)
    x = inputs.uniform(g, (batch * sx,), dtype)
    y = inputs.uniform(g, (batch * sy,), dtype)
    return A, lda, sA, x, sx, y, sy, rows, cols


def _run_gemv(dtype, trans, m, n, alpha, A, lda, sA, x, incx, sx, beta, y, incy, sy, batch):
    dA, dx, dy = to_dev(A), to_dev(x), to_dev(y)
    sbg.gemv_strided(trans, m, n, alpha, dA, lda, sA, dx, incx, sx, beta, dy, incy, sy, batch)
    torch.cuda.synchronize()
    return from_dev(dy)


def _check_gemv(dtype, trans, m, n, alpha, A, lda, sA, x, incx, sx, beta, y, incy, sy, batch, got, idx=None):
    rows, cols = (m, n) if trans == "N" else (n, m)
    idx = np.arange(batch) if idx is None else np.asarray(idx)
    worst = 0.0
    for p in idx:
        h, l, b = blas.gemv(trans, m, n, alpha, A[p * sA:], lda, 0, x[p * sx:], incx, 0, beta, y[p * sy:], incy, 0, 1)
        gv = got[p * sy + incy * np.arange(rows)].astype(np.complex128 if np.iscomplexobj(got) else np.float64)
        diff = np.abs((gv - h[0]) - l[0])
        e = np.where(b[0] > 0, diff / np.where(b[0] > 0, b[0], 1), np.where(diff == 0, 0, np.inf))
        worst = max(worst, float(np.max(e)) if e.size else 0.0)
    tol = 4 * max(cols, 1) * unit(dtype)
    assert worst <= tol, f"gemv {np.dtype(dtype).name} {trans} {m}x{n} incx={incx} incy={incy}: " \
                         f"{worst / unit(dtype):.2f} u"
    # entries of y between the vectors are never written
    if batch <= 10_000:
        mask = np.ones(got.shape, dtype=bool)
        for p in range(batch):
            mask[p * sy + incy * np.arange(rows)] = False
        assert np.array_equal(got[mask].view(np.uint8), y[mask].view(np.uint8))
    return worst / unit(dtype)


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_gemv_shapes_ops_increments(gpu_lib, dtype):
    g = inputs.rng(601)
    al, be = P.scalars(dtype)
    worst = 0.0
    for trans in "NTC":
        for (m, n) in [(1, 1), (3, 5), (16, 16), (7, 16), (16, 3), (40, 17), (5, 70)]:
            for incx, incy in [(1, 1), (2, 1), (1, 3), (3, 2)]:
                say(f"gemv {np.dtype(dtype).name} {trans} {m}x{n} incx={incx} incy={incy}")
                A, lda, sA, x, sx, y, sy, rows, cols = _vec_case(g, dtype, trans, m, n, incx, incy, 23)
                got = _run_gemv(dtype, trans, m, n, al, A, lda, sA, x, incx, sx, be, y, incy, sy, 23)
                worst = max(worst, _check_gemv(dtype, trans, m, n, al, A, lda, sA, x, incx, sx, be, y, incy, sy,
                                               23, got))
    say(f"worst {worst:.2f} u")


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_gemv_special_scalars(gpu_lib, dtype):
    """alpha = 0: A and x (NaN) are not read; beta = 0: y (NaN) is not read;
    device scalars give the host-mode result."""
    g = inputs.rng(602)
    m, n, batch = 9, 12, 17
    for trans, incx, incy in (("N", 1, 1), ("T", 2, 3)):
        A, lda, sA, x, sx, y, sy, rows, cols = _vec_case(g, dtype, trans, m, n, incx, incy, batch)
        got = _run_gemv(dtype, trans, m, n, 0.0, np.full_like(A, np.nan), lda, sA, np.full_like(x, np.nan), incx,
                        sx, -0.5, y, incy, sy, batch)
        assert np.all(np.isfinite(got[:batch * sy]))
        _check_gemv(dtype, trans, m, n, 0.0, A, lda, sA, x, incx, sx, -0.5, y, incy, sy, batch, got)
        ynan = np.full_like(y, np.nan)
        got = _run_gemv(dtype, trans, m, n, 1.5, A, lda, sA, x, incx, sx, 0.0, ynan, incy, sy, batch)
        vals = np.concatenate([got[p * sy + incy * np.arange(rows)] for p in range(batch)])
        assert np.all(np.isfinite(vals))
        tdt = TORCH[np.dtype(dtype).type]
        al = torch.tensor([1.5], dtype=tdt, device="cuda")
        be = torch.tensor([-0.5], dtype=tdt, device="cuda")
        dA, dx, dy = to_dev(A), to_dev(x), to_dev(y)
        sbg.gemv_strided(trans, m, n, al, dA, lda, sA, dx, incx, sx, be, dy, incy, sy, batch)
        torch.cuda.synchronize()
        ref = _run_gemv(dtype, trans, m, n, 1.5, A, lda, sA, x, incx, sx, -0.5, y, incy, sy, batch)
        assert np.array_equal(from_dev(dy).view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
def test_gemv_full_size(gpu_lib, dtype):
    """N = 10^6 vectors, A 16 x 16, N and T, packed; sampled against the oracle."""
    g = inputs.rng(603)
    N, m, n = 1_000_000, 16, 16
    A = inputs.uniform(g, (N * m * n,), dtype)
    x = inputs.uniform(g, (N * n,), dtype)
    y = inputs.uniform(g, (N * m,), dtype)
    idx = np.unique(np.concatenate([[0, 1, N - 1], g.choice(N, 300, replace=False)]))
    for trans in "NT":
        say(f"gemv full {np.dtype(dtype).name} {trans}")
        got = _run_gemv(dtype, trans, m, n, 1.5, A, m, m * n, x, 1, n, -0.5, y, 1, m, N)
        _check_gemv(dtype, trans, m, n, 1.5, A, m, m * n, x, 1, n, -0.5, y, 1, m, N, got, idx=idx)


def _tri_batch(g, dtype, size, batch, pad=3, diag_nan=False, other_nan=False, uplo="L"):
    """Well-conditioned triangular factors: off-diagonal U[-1, 1] / size,
    diagonal magnitude in [1.5, 2.5]."""
    lda = size + 2
    sA = lda * size + pad
    A = np.zeros(batch * sA, dtype=dtype)
    for p in range(batch):
        T = inputs.uniform(g, (size, size), dtype) / max(size, 1)
        d = 2.0 + 0.5 * inputs.uniform(g, (size,), np.float64)
        T[np.arange(size), np.arange(size)] = d.astype(dtype)
        if diag_nan:
            T[np.arange(size), np.arange(size)] = np.nan
        if other_nan:
            iu = np.triu_indices(size, 1) if uplo == "L" else np.tril_indices(size, -1)
            T[iu] = np.nan
        for j in range(size):
            A[p * sA + lda * j: p * sA + lda * j + size] = T[:, j]
    return A, lda, sA


def _run_trsm(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, batch):
    dA, dB = to_dev(A), to_dev(B)
    sbg.trsm_strided(side, uplo, trans, diag, m, n, alpha, dA, lda, sA, dB, ldb, sB, batch)
    torch.cuda.synchronize()
    return from_dev(dB)


def _check_trsm(dtype, side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, batch, got, idx=None,
                Aref=None):
    idx = np.arange(batch) if idx is None else np.asarray(idx)
    s = m if side == "L" else n
    Aref = A if Aref is None else Aref
    X = np.stack([got[p * sB + np.arange(m)[:, None] + ldb * np.arange(n)[None, :]] for p in idx])
    Asub = np.concatenate([Aref[p * sA:p * sA + sA] for p in idx])
    Bsub = np.concatenate([B[p * sB:p * sB + sB] for p in idx])
    cnt = len(idx)
    r = blas.trsm_residual(side, uplo, trans, diag, m, n, alpha, Asub, lda, sA, Bsub, ldb, sB, X, cnt)
    cplx = np.dtype(dtype).kind == "c"
    tol = (8 if cplx else 4) * (s + 1) * unit(dtype)
    lbl = f"trsm {np.dtype(dtype).name} {side}{uplo}{trans}{diag} {m}x{n}"
    assert np.all(np.isfinite(X)), lbl
    assert float(np.max(r)) <= tol, f"{lbl}: backward error {float(np.max(r)) / unit(dtype):.2f} u"
    hi, lo, _ = blas.trsm(side, uplo, trans, diag, m, n, alpha, Asub, lda, sA, Bsub, ldb, sB, cnt)
    ref = hi + lo
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    fwd = float(np.max(np.abs(X - ref))) / scale if scale > 0 else float(np.max(np.abs(X)))
    assert fwd <= 64 * (s + 1) * unit(dtype), f"{lbl}: forward error {fwd / unit(dtype):.1f} u"
    # entries of B outside the m x n matrices are never written
    if batch <= 10_000:
        mask = np.ones(got.shape, dtype=bool)
        for p in range(batch):
            mask[p * sB + np.arange(m)[:, None] + ldb * np.arange(n)[None, :]] = False
        assert np.array_equal(got[mask].view(np.uint8), B[mask].view(np.uint8))
    return float(np.max(r)) / unit(dtype)


def _b_batch(g, dtype, m, n, batch, pad=2):
    ldb = m + 1
    sB = ldb * n + pad
    return inputs.uniform(g, (batch * sB,), dtype), ldb, sB


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("side", "LR")
def test_trsm_all_variants_small(gpu_lib, dtype, side):
    g = inputs.rng(604)
    alpha = complex(0.5, -1.0) if np.dtype(dtype).kind == "c" else -1.25
    worst = 0.0
    for uplo in "UL":
        for trans in "NTC":
            for diag in "NU":
                for (s, o) in [(1, 3), (5, 7), (16, 16), (9, 1), (16, 20)]:
                    m, n = (s, o) if side == "L" else (o, s)
                    A, lda, sA = _tri_batch(g, dtype, s, 9)
                    B, ldb, sB = _b_batch(g, dtype, m, n, 9)
                    say(f"trsm {np.dtype(dtype).name} {side}{uplo}{trans}{diag} {m}x{n}")
                    got = _run_trsm(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, 9)
                    worst = max(worst, _check_trsm(dtype, side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb,
                                                   sB, 9, got))
    say(f"worst backward error {worst:.2f} u")


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("side", "LR")
def test_trsm_blocked_above_16(gpu_lib, dtype, side):
    """Triangular order above 16: diagonal blocks by the substitution kernel,
    updates by batched GEMM."""
    g = inputs.rng(605)
    alpha = complex(1.0, 0.5) if np.dtype(dtype).kind == "c" else 0.75
    for uplo in "UL":
        for trans in "NTC":
            for diag in "NU":
                for (s, o) in [(17, 5), (40, 3)]:
                    m, n = (s, o) if side == "L" else (o, s)
                    A, lda, sA = _tri_batch(g, dtype, s, 5)
                    B, ldb, sB = _b_batch(g, dtype, m, n, 5)
                    say(f"trsm blocked {np.dtype(dtype).name} {side}{uplo}{trans}{diag} {m}x{n}")
                    got = _run_trsm(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, 5)
                    _check_trsm(dtype, side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, 5, got)


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_trsm_unread_entries_and_alpha(gpu_lib, dtype):
    """diag U: a NaN diagonal is never read; the other triangle (NaN) is never
    read; alpha = 0 gives zeros without reading A or B (NaN); device alpha
    gives the host-mode result."""
    g = inputs.rng(606)
    for s in (7, 16, 33):
        m, n = s, 4
        A, lda, sA = _tri_batch(g, dtype, s, 6, diag_nan=True, other_nan=True, uplo="L")
        Aclean, _, _ = _tri_batch(inputs.rng(606 + s), dtype, s, 6)
        B, ldb, sB = _b_batch(g, dtype, m, n, 6)
        say(f"trsm unread {np.dtype(dtype).name} s={s}")
        got = _run_trsm("L", "L", "N", "U", m, n, 1.0, A, lda, sA, B, ldb, sB, 6)
        # reference: the same strictly-lower part with ones on the diagonal
        Aref = np.where(np.isnan(A), 0, A).astype(dtype)
        _check_trsm(dtype, "L", "L", "N", "U", m, n, 1.0, A, lda, sA, B, ldb, sB, 6, got, Aref=Aref)
        Bn = np.full((6 * (n + 1) * s + 12,), np.nan, dtype=dtype)
        dA, dB = to_dev(np.full_like(A, np.nan)), to_dev(Bn)
        sbg.trsm_strided("R", "U", "T", "N", n, s, 0.0, dA, lda, sA, dB, n + 1, (n + 1) * s + 2, 6)
        torch.cuda.synchronize()
        out = from_dev(dB)
        for p in range(6):
            blk = out[p * ((n + 1) * s + 2) + np.arange(n)[:, None] + (n + 1) * np.arange(s)[None, :]]
            assert np.all(blk == 0)
        tdt = TORCH[np.dtype(dtype).type]
        al = torch.tensor([-0.5], dtype=tdt, device="cuda")
        dA, dB = to_dev(Aclean), to_dev(B)
        sbg.trsm_strided("L", "U", "C", "N", m, n, al, dA, lda, sA, dB, ldb, sB, 6)
        torch.cuda.synchronize()
        ref = _run_trsm("L", "U", "C", "N", m, n, -0.5, Aclean, lda, sA, B, ldb, sB, 6)
        assert np.array_equal(from_dev(dB).view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
def test_trsm_full_size(gpu_lib, dtype):
    """N = 100,000 systems of order 16 with 16 right-hand sides, LLNN and
    RUTN, packed; sampled systems checked."""
    g = inputs.rng(607)
    N, s = 100_000, 16
    A = inputs.uniform(g, (N * s * s,), dtype) / s
    d = np.arange(N * s * s).reshape(N, s, s)
    diag = d[:, np.arange(s), np.arange(s)].ravel()
    A[diag] = (2.0 + 0.5 * inputs.uniform(g, (N * s,), np.float64)).astype(dtype)
    B = inputs.uniform(g, (N * s * s,), dtype)
    idx = np.unique(np.concatenate([[0, 1, N - 1], g.choice(N, 200, replace=False)]))
    for side, uplo, trans in (("L", "L", "N"), ("R", "U", "T")):
        say(f"trsm full {np.dtype(dtype).name} {side}{uplo}{trans}N")
        got = _run_trsm(side, uplo, trans, "N", s, s, 1.5, A, s, s * s, B, s, s * s, N)
        _check_trsm(dtype, side, uplo, trans, "N", s, s, 1.5, A, s, s * s, B, s, s * s, N, got, idx=idx)
