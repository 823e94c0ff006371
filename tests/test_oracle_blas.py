"""Pins of the batched GEMV / TRSM oracle (oracle/blas.py) against things
other than itself: exact rational arithmetic on small inputs (GEMV), a
library triangular solver and the defining residual (TRSM), and closed forms
(identity and diagonal matrices, unit diagonals that must not be read)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import blas
from paper_1304_7053_amd import inputs


def _frac(v):
    v = complex(v)
    return (Fraction(v.real), Fraction(v.imag))


def _cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.complex64, np.complex128])
@pytest.mark.parametrize("trans", "NTC")
def test_gemv_exact_rationals(dtype, trans):
    """Every entry matches the exact rational result to within 2^-58 of the
    error bound's denominator (extended precision: far below the binary64
    unit the GPU is judged by), with non-unit increments, padding between
    matrices and vectors, and a ragged batch."""
    g = inputs.rng(501)
    m, n, lda, incx, incy, batch = 3, 4, 5, 2, 3, 3
    cplx = np.dtype(dtype).kind == "c"
    sA = lda * n + 2
    rows, cols = (m, n) if trans == "N" else (n, m)
    sx, sy = incx * cols + 1, incy * rows + 2
    A = inputs.uniform(g, (batch * sA,), dtype)
    x = inputs.uniform(g, (batch * sx,), dtype)
    y = inputs.uniform(g, (batch * sy,), dtype)
    alpha, beta = (complex(1.5, -0.25), complex(-0.5, 0.75)) if cplx else (1.5, -0.5)
    hi, lo, bnd = blas.gemv(trans, m, n, alpha, A, lda, sA, x, incx, sx, beta, y, incy, sy, batch)
    for p in range(batch):
        for i in range(rows):
            acc = (Fraction(0), Fraction(0))
            for l in range(cols):
                a = A[p * sA + (i + lda * l if trans == "N" else l + lda * i)]
                a = np.conj(a) if trans == "C" else a
                t = _cmul(_frac(a), _frac(x[p * sx + incx * l]))
                acc = (acc[0] + t[0], acc[1] + t[1])
            ref = _cmul(_frac(alpha), acc)
            t = _cmul(_frac(beta), _frac(y[p * sy + incy * i]))
            ref = (ref[0] + t[0], ref[1] + t[1])
            gh, gl = complex(hi[p, i]), complex(lo[p, i])
            got = (Fraction(gh.real) + Fraction(gl.real), Fraction(gh.imag) + Fraction(gl.imag))
            err = abs(got[0] - ref[0]) + abs(got[1] - ref[1])
            assert bnd[p, i] > 0
            assert err <= Fraction(1, 2 ** 58) * Fraction(float(bnd[p, i]))


def test_gemv_identity_and_special_scalars():
    """A = I gives y = alpha x + beta y; alpha = 0 never reads A or x (NaN),
    beta = 0 never reads y (NaN)."""
    g = inputs.rng(502)
    n = 6
    A = np.eye(n).ravel(order="F").astype(np.float64)
    x = inputs.uniform(g, (n,), np.float64)
    y = inputs.uniform(g, (n,), np.float64)
    hi, lo, _ = blas.gemv("N", n, n, 2.0, A, n, 0, x, 1, 0, 3.0, y, 1, 0, 1)
    assert np.array_equal(hi[0] + lo[0], 2.0 * x + 3.0 * y)
    nanA = np.full_like(A, np.nan)
    hi, _, _ = blas.gemv("T", n, n, 0.0, nanA, n, 0, np.full_like(x, np.nan), 1, 0, -1.0, y, 1, 0, 1)
    assert np.array_equal(hi[0], -y)
    hi, _, _ = blas.gemv("N", n, n, 1.0, A, n, 0, x, 1, 0, 0.0, np.full_like(y, np.nan), 1, 0, 1)
    assert np.array_equal(hi[0], x)


def _tri_case(g, dtype, side, m, n, batch, pad=3):
    size = m if side == "L" else n
    lda = size + 2
    sA = lda * size + pad
    A = np.zeros(batch * sA, dtype=dtype)
    for p in range(batch):
        T = inputs.uniform(g, (size, size), dtype) / size
        T[np.arange(size), np.arange(size)] += np.asarray(1.5, dtype=dtype) + 0.5 * inputs.uniform(g, (size,), dtype).real.astype(dtype)
        for j in range(size):
            A[p * sA + lda * j: p * sA + lda * j + size] = T[:, j]
    ldb = m + 1
    sB = ldb * n + pad
    B = inputs.uniform(g, (batch * sB,), dtype)
    return A, lda, sA, B, ldb, sB


@pytest.mark.parametrize("dtype", [np.float64, np.complex128])
@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("uplo", "UL")
@pytest.mark.parametrize("trans", "NTC")
@pytest.mark.parametrize("diag", "NU")
def test_trsm_against_library_solver(dtype, side, uplo, trans, diag):
    """scipy's triangular solver on the same systems (side R recast as
    op(A)^T X^T = alpha B^T), and the defining residual op(A) X = alpha B."""
    g = inputs.rng(503)
    m, n, batch = 5, 4, 3
    A, lda, sA, B, ldb, sB = _tri_case(g, dtype, side, m, n, batch)
    alpha = complex(0.5, 1.0) if np.dtype(dtype).kind == "c" else -1.25
    hi, lo, X = blas.trsm(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, batch)
    size = m if side == "L" else n
    for p in range(batch):
        T = blas.triangle(A, p * sA, lda, size, uplo, diag, np.longdouble if dtype == np.float64
                          else np.clongdouble)
        T = np.asarray(T, dtype=np.complex128 if np.dtype(dtype).kind == "c" else np.float64)
        opT = {"N": T, "T": T.T, "C": np.conj(T).T}[trans]
        rhs = alpha * np.asarray(B[p * sB + np.arange(m)[:, None] + ldb * np.arange(n)[None, :]])
        if side == "L":
            ref = scipy.linalg.solve_triangular(opT, rhs, lower=bool(np.allclose(np.triu(opT, 1), 0)))
        else:
            M = opT.T
            ref = scipy.linalg.solve_triangular(M, rhs.T, lower=bool(np.allclose(np.triu(M, 1), 0))).T
        assert np.allclose(hi[p] + lo[p], ref, rtol=1e-12, atol=1e-13)
    r = blas.trsm_residual(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, hi + lo, batch)
    assert np.all(r < 1e-15)


def test_trsm_closed_forms():
    """Diagonal A: X = alpha B / diag; unit diagonal: a NaN stored on the
    diagonal is never read, and the other triangle (NaN) never either."""
    g = inputs.rng(504)
    m, n = 4, 3
    d = np.array([2.0, -4.0, 0.5, 8.0])
    A = np.diag(d).ravel(order="F")
    B = inputs.uniform(g, (m * n,), np.float64)
    hi, lo, _ = blas.trsm("L", "U", "N", "N", m, n, 3.0, A, m, 0, B, m, 0, 1)
    assert np.array_equal(hi[0], 3.0 * B.reshape(n, m).T / d[:, None])
    L = np.tril(inputs.uniform(g, (m, m), np.float64), -1)
    stored = L.copy()
    stored[np.arange(m), np.arange(m)] = np.nan
    stored[np.triu_indices(m, 1)] = np.nan
    ref_A = L + np.eye(m)
    hi, lo, _ = blas.trsm("L", "L", "N", "U", m, n, 1.0, stored.ravel(order="F"), m, 0, B, m, 0, 1)
    assert np.allclose(ref_A @ (hi[0] + lo[0]), B.reshape(n, m).T, rtol=1e-14, atol=1e-15)
    # alpha = 0: X = 0 and A (NaN) is not read
    hi, _, _ = blas.trsm("R", "U", "T", "N", m, n, 0.0, np.full(n * n, np.nan), n, 0, B, m, 0, 1)
    assert np.all(hi == 0)


def test_trsm_order_and_triangle_mistakes_fail():
    """The pins above fail on plausible mistakes: solving with the wrong
    triangle or in the wrong order changes the result."""
    g = inputs.rng(505)
    m, n = 5, 2
    A, lda, sA, B, ldb, sB = _tri_case(g, np.float64, "L", m, n, 1)
    good, _, _ = blas.trsm("L", "L", "N", "N", m, n, 1.0, A, lda, sA, B, ldb, sB, 1)
    other, _, _ = blas.trsm("L", "U", "N", "N", m, n, 1.0, A, lda, sA, B, ldb, sB, 1)
    trans, _, _ = blas.trsm("L", "L", "T", "N", m, n, 1.0, A, lda, sA, B, ldb, sB, 1)
    assert not np.allclose(good, other) and not np.allclose(good, trans)


@pytest.mark.parametrize("dtype", [np.float64, np.complex128])
@pytest.mark.parametrize("side", "LR")
def test_trsm_residual_rejects_wrong_solutions(dtype, side):
    """The backward-error check that accepts GPU TRSM results must reject
    what a broken solver would return: B itself (nothing solved), the
    solution of the other triangle, the solution of the other op, and a
    solution with one entry off by a relative 1e-6 -- each ratio far above
    the acceptance level 4 (s + 1) u, while the true solution sits below it."""
    g = inputs.rng(506)
    m, n, batch = 6, 5, 4
    A, lda, sA, B, ldb, sB = _tri_case(g, dtype, side, m, n, batch)
    alpha = complex(0.75, -0.5) if np.dtype(dtype).kind == "c" else 1.25
    size = m if side == "L" else n
    accept = 4 * (size + 1) * 2.0 ** -53 * (2 if np.dtype(dtype).kind == "c" else 1)
    args = (side, "L", "N", "N", m, n, alpha, A, lda, sA, B, ldb, sB)
    hi, lo, _ = blas.trsm(*args, batch)
    good = hi + lo
    assert np.all(blas.trsm_residual(*args, good, batch) <= accept)
    unsolved = np.stack([B[p * sB + np.arange(m)[:, None] + ldb * np.arange(n)[None, :]] for p in range(batch)])
    assert np.all(blas.trsm_residual(*args, unsolved, batch) > 1e-3)
    h2, l2, _ = blas.trsm(side, "U", "N", "N", m, n, alpha, A, lda, sA, B, ldb, sB, batch)
    assert np.all(blas.trsm_residual(*args, h2 + l2, batch) > 1e-3)
    h3, l3, _ = blas.trsm(side, "L", "T", "N", m, n, alpha, A, lda, sA, B, ldb, sB, batch)
    assert np.all(blas.trsm_residual(*args, h3 + l3, batch) > 1e-3)
    nudged = good.copy()
    nudged[:, 2, 1] *= 1 + 1e-6
    assert np.all(blas.trsm_residual(*args, nudged, batch) > 1e3 * accept)
