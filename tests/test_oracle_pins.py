"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

Each test ties the oracle to something other than its own formula:
  * a library routine the definition reduces to (numpy.matmul in float64 /
    complex128, for every op pair of Sec. 2 and every scalar type);
  * exact special cases (identity / permutation operands, alpha = 0,
    beta = 0, rank-1 closed forms, integer data, conjugate-transpose
    identities), compared bit for bit;
  * exact rational brute force on tiny batches, against which the two
    accumulation modes must sit within their rounding bounds;
  * the storage-layout rule of Sec. 5 (leading dimensions and matrix offsets
    in elements, gaps never read).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1304_7053_amd import inputs

U53 = 2.0 ** -53
OPS = "NTCR"
DTYPES = [np.float32, np.float64, np.complex64, np.complex128]


def np_op(X, op):
    """op(X) on a (batch, rows, cols) stack, written with numpy primitives."""
    if op == "N":
        return X
    if op == "T":
        return np.swapaxes(X, 1, 2)
    if op == "C":
        return np.conj(np.swapaxes(X, 1, 2))
    if op == "R":
        return np.conj(X)
    raise ValueError(op)


def stored_shape(op, rows, cols):
    return (rows, cols) if op == "N" or op == "R" else (cols, rows)


def random_case(g, dtype, ta, tb, m, n, k, batch=7, dist="uniform"):
    A = inputs.DISTS[dist](g, (batch,) + stored_shape(ta, m, k), dtype)
    B = inputs.DISTS[dist](g, (batch,) + stored_shape(tb, k, n), dtype)
    C = inputs.DISTS[dist](g, (batch, m, n), dtype)
    return A, B, C


def hp(x):
    """float64 / complex128 copy."""
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("ta", OPS)
@pytest.mark.parametrize("tb", OPS)
def test_matches_numpy_matmul(dtype, ta, tb):
    g = inputs.rng(101, salt=OPS.index(ta) * 4 + OPS.index(tb))
    cplx = np.dtype(dtype).kind == "c"
    for (m, n, k) in [(1, 1, 1), (3, 5, 2), (16, 16, 16), (7, 1, 13), (16, 9, 4)]:
        A, B, C = random_case(g, dtype, ta, tb, m, n, k)
        alpha = complex(1.25, -0.5) if cplx else 1.25
        beta = complex(-0.75, 0.25) if cplx else -0.75
        ref = alpha * (np_op(hp(A), ta) @ np_op(hp(B), tb)) + beta * hp(C)
        absref = abs(alpha) * (np.abs(np_op(hp(A), ta)) @ np.abs(np_op(hp(B), tb))) + abs(beta) * np.abs(hp(C))
        for ext in (False, True):
            hi, lo = oracle.gemm(ta, tb, alpha, A, B, beta, C, ext=ext)
            err = np.abs((hi - ref) + lo)
            assert np.all(err <= (2 * k + 6) * U53 * absref), (m, n, k, ext, float(np.max(err / absref)))


@pytest.mark.parametrize("dtype", DTYPES)
def test_identity_and_permutation_are_exact(dtype):
    g = inputs.rng(102)
    for (ta, tb) in [("N", "N"), ("T", "N"), ("C", "T"), ("R", "C")]:
        for k in (1, 5, 16):
            n = 11
            perm = g.permutation(k)
            P = np.zeros((k, k), dtype=dtype)
            P[np.arange(k), perm] = 1
            # stored A such that op(A) = P (conj and transpose of a 0/1 matrix)
            A_op = np.broadcast_to(P, (3, k, k))
            # P is real 0/1, so conjugation leaves it alone: only the transpose matters
            A = np.ascontiguousarray(np.swapaxes(A_op, 1, 2) if ta in "TC" else A_op)
            B = inputs.uniform(g, (3,) + stored_shape(tb, k, n), dtype)
            hi, lo = oracle.gemm(ta, tb, 1.0, A, B, 0.0, None)
            expect = hp(np_op(B, tb))[:, perm, :]
            assert np.array_equal(hi, expect)
            assert not np.any(lo)


@pytest.mark.parametrize("dtype", DTYPES)
def test_alpha_zero_returns_beta_c_and_never_reads_a_b(dtype):
    g = inputs.rng(103)
    cplx = np.dtype(dtype).kind == "c"
    m, n, k, batch = 5, 7, 3, 4
    C = inputs.uniform(g, (batch, m, n), dtype)
    A = np.full((batch, m, k), np.nan, dtype=dtype)
    B = np.full((batch, k, n), np.nan, dtype=dtype)
    beta = complex(0.3, -1.7) if cplx else -0.3
    hi, _ = oracle.gemm("N", "N", 0.0, A, B, beta, C)
    assert np.all(np.isfinite(hi))
    if cplx:
        # a complex product rounds each part of two products and a sum
        ref = np.asarray(beta, dtype=np.complex128) * hp(C)
        assert np.all(np.abs(hi - ref) <= 4 * U53 * abs(beta) * np.abs(hp(C)))
    else:
        assert np.array_equal(hi, np.float64(beta) * hp(C))
    # beta = 0 as well: exact zeros, C not read either
    hi0, _ = oracle.gemm("N", "N", 0.0, A, B, 0.0, np.full_like(C, np.nan))
    assert np.array_equal(hi0, np.zeros_like(hi0))


@pytest.mark.parametrize("dtype", DTYPES)
def test_beta_zero_never_reads_c(dtype):
    g = inputs.rng(104)
    A, B, _ = random_case(g, dtype, "N", "T", 6, 4, 9)
    Cnan = np.full((7, 6, 4), np.nan, dtype=dtype)
    hi, _ = oracle.gemm("N", "T", 2.0, A, B, 0.0, Cnan)
    ref = 2.0 * (hp(A) @ np.swapaxes(hp(B), 1, 2))
    assert np.all(np.isfinite(hi))
    assert np.allclose(hi, ref, rtol=1e-14, atol=1e-14)


def dyadic(g, shape, cplx):
    v = g.integers(-64, 65, size=shape) / 32.0
    if cplx:
        v = v + 1j * g.integers(-64, 65, size=shape) / 16.0
    return v


@pytest.mark.parametrize("dtype", DTYPES)
def test_rank1_closed_form(dtype):
    """op(A) = x s^T, op(B) = t z^T  =>  C = alpha (s.t) x z^T + beta C exactly
    (all entries dyadic with few bits, so every step is exact)."""
    g = inputs.rng(105)
    cplx = np.dtype(dtype).kind == "c"
    for (ta, tb, m, n, k) in [("N", "N", 4, 6, 3), ("T", "C", 16, 16, 16), ("C", "R", 2, 9, 7)]:
        x, s = dyadic(g, m, cplx), dyadic(g, k, cplx)
        t, z = dyadic(g, k, cplx), dyadic(g, n, cplx)
        opA = np.outer(x, s)
        opB = np.outer(t, z)
        # undo the op to get the stored operands
        def stored(opX, op):
            if op == "N":
                return opX
            if op == "T":
                return opX.T
            if op == "C":
                return np.conj(opX).T
            return np.conj(opX)
        A = stored(opA, ta)[None].astype(dtype)
        B = stored(opB, tb)[None].astype(dtype)
        C = dyadic(g, (1, m, n), cplx).astype(dtype)
        alpha = (0.5 + 0.25j) if cplx else 0.5
        beta = (-2.0 + 1.0j) if cplx else -2.0
        st = np.dot(s, t)  # exact: a handful of few-bit dyadic products
        expect = alpha * st * np.outer(x, z) + beta * C[0].astype(np.complex128 if cplx else np.float64)
        hi, lo = oracle.gemm(ta, tb, alpha, A, B, beta, C)
        assert np.array_equal(hi[0], expect), (ta, tb)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_conjugate_transpose_identities(dtype):
    g = inputs.rng(106)
    m, n, k = 5, 7, 6
    A = inputs.uniform(g, (4, m, k), dtype)
    B = inputs.uniform(g, (4, k, n), dtype)
    AB, _ = oracle.gemm("N", "N", 1.0, A, B, 0.0, None)
    # (AB)^H = B^H A^H
    BhAh, _ = oracle.gemm("C", "C", 1.0, B, A, 0.0, None)
    assert np.array_equal(BhAh, np.conj(np.swapaxes(AB, 1, 2)))
    # (AB)^T = B^T A^T
    BtAt, _ = oracle.gemm("T", "T", 1.0, B, A, 0.0, None)
    assert np.array_equal(BtAt, np.swapaxes(AB, 1, 2))
    # op 'C' on A equals 'N' on the materialised A^H
    Ah = np.ascontiguousarray(np.conj(np.swapaxes(A, 1, 2)))
    X1, _ = oracle.gemm("C", "N", 1.0, Ah, B, 0.0, None)
    assert np.array_equal(X1, AB)
    # op 'R' (conjugate, no transpose) equals 'N' on conj(A); conj(A)B = conj(A conj(B))
    X2, _ = oracle.gemm("R", "N", 1.0, A, B, 0.0, None)
    X3, _ = oracle.gemm("N", "R", 1.0, A, B, 0.0, None)
    assert np.array_equal(X2, oracle.gemm("N", "N", 1.0, np.conj(A), B, 0.0, None)[0])
    assert np.array_equal(X2, np.conj(X3))


@pytest.mark.parametrize("dtype", DTYPES)
def test_real_conj_equals_transpose(dtype):
    if np.dtype(dtype).kind == "c":
        pytest.skip("real types only")
    g = inputs.rng(107)
    A, B, C = random_case(g, dtype, "T", "T", 6, 5, 4)
    x1, _ = oracle.gemm("T", "T", 1.5, A, B, -0.5, C)
    x2, _ = oracle.gemm("C", "C", 1.5, A, B, -0.5, C)
    assert np.array_equal(x1, x2)


def exact_gemm(ta, tb, alpha, A, B, beta, C):
    """Exact rational evaluation of Eq. (1) on a tiny batch (Fractions for the
    real and imaginary parts separately)."""
    def fr(x):
        return (Fraction(float(np.real(x))), Fraction(float(np.imag(x))))

    def mul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    def add(a, b):
        return (a[0] + b[0], a[1] + b[1])

    oA = np_op(A, ta)
    oB = np_op(B, tb)
    batch, m, k = oA.shape
    n = oB.shape[2]
    al, be = fr(alpha), fr(beta)
    out = np.empty((batch, m, n), dtype=object)
    for p in range(batch):
        for i in range(m):
            for j in range(n):
                s = (Fraction(0), Fraction(0))
                for l in range(k):
                    s = add(s, mul(fr(oA[p, i, l]), fr(oB[p, l, j])))
                out[p, i, j] = add(mul(al, s), mul(be, fr(C[p, i, j])))
    return out


@pytest.mark.parametrize("dtype", DTYPES)
def test_exact_rational_brute_force(dtype):
    g = inputs.rng(108)
    cplx = np.dtype(dtype).kind == "c"
    alpha = complex(1.5, -0.25) if cplx else 1.5
    beta = complex(0.25, -1.0) if cplx else -0.5
    for (ta, tb) in [("N", "N"), ("T", "C"), ("C", "R"), ("R", "T")]:
        for (m, n, k) in [(2, 3, 4), (4, 1, 9), (3, 3, 16)]:
            A, B, C = random_case(g, dtype, ta, tb, m, n, k, batch=2)
            ex = exact_gemm(ta, tb, alpha, A, B, beta, C)
            absA = np.abs(hp(np_op(A, ta)))
            absB = np.abs(hp(np_op(B, tb)))
            den = abs(alpha) * (absA @ absB) + abs(beta) * np.abs(hp(C))
            for ext, lim in ((False, (2 * k + 8) * U53), (True, 4.0 * U53)):
                hi, lo = oracle.gemm(ta, tb, alpha, A, B, beta, C, ext=ext)
                for idx in np.ndindex(ex.shape):
                    er, ei = ex[idx]
                    dr = abs(Fraction(float(np.real(hi[idx]))) + Fraction(float(np.real(lo[idx]))) - er)
                    di = abs(Fraction(float(np.imag(hi[idx]))) + Fraction(float(np.imag(lo[idx]))) - ei)
                    assert float(dr) <= lim * den[idx] and float(di) <= lim * den[idx], (ta, tb, m, n, k, ext, idx)


@pytest.mark.parametrize("dtype", [np.float32, np.complex64])
def test_integer_data_exact(dtype):
    """Integer entries in {-3..3} with dyadic alpha, beta: every partial result
    is a small dyadic number, so the oracle must be exact (checked against
    exact rational evaluation)."""
    g = inputs.rng(109)
    cplx = np.dtype(dtype).kind == "c"
    alpha = complex(1.0, 0.5) if cplx else 1.5
    beta = complex(0.25, -1.0) if cplx else -0.5
    A, B, C = random_case(g, dtype, "T", "N", 16, 16, 16, batch=2, dist="int")
    ex = exact_gemm("T", "N", alpha, A, B, beta, C)
    hi, lo = oracle.gemm("T", "N", alpha, A, B, beta, C)
    for idx in np.ndindex(ex.shape):
        assert Fraction(float(np.real(hi[idx]))) == ex[idx][0]
        assert Fraction(float(np.imag(hi[idx]))) == ex[idx][1]
    assert not np.any(lo)


@pytest.mark.parametrize("dtype", DTYPES)
def test_layout_rule_padding_never_read(dtype):
    """Element (i, j) of matrix p sits at p*ld2 + i + ld*j (units: elements).
    Padding filled with NaN must not reach the result, and the result must
    equal the packed-layout result bit for bit."""
    g = inputs.rng(110)
    m, n, k, batch = 5, 3, 4, 6
    lda, ldb, ldc = 9, 6, 7
    sA, sB, sC = lda * k + 5, ldb * n + 1, ldc * n + 3
    A = inputs.strided_batch(g, batch, m, k, lda, sA, dtype)
    B = inputs.strided_batch(g, batch, k, n, ldb, sB, dtype)
    C = inputs.strided_batch(g, batch, m, n, ldc, sC, dtype)
    hi, _ = oracle.gemm_strided("N", "N", m, n, k, 0.75, A, lda, sA, B, ldb, sB, -1.25, C, ldc, sC, batch)
    assert np.all(np.isfinite(hi))

    def pack(X, rows, cols, ld, st):
        p = np.arange(batch)[:, None, None]
        c = np.arange(cols)[None, :, None]
        r = np.arange(rows)[None, None, :]
        return np.swapaxes(X[p * st + c * ld + r], 1, 2)  # (batch, rows, cols)

    hp_, _ = oracle.gemm("N", "N", 0.75, pack(A, m, k, lda, sA), pack(B, k, n, ldb, sB), -1.25,
                         pack(C, m, n, ldc, sC))
    assert np.array_equal(hi, hp_)


@pytest.mark.parametrize("dtype", DTYPES)
def test_bound_matches_abs_matmul(dtype):
    g = inputs.rng(111)
    cplx = np.dtype(dtype).kind == "c"
    m, n, k = 6, 5, 7
    A, B, C = random_case(g, dtype, "C", "N", m, n, k, batch=3)
    alpha = complex(0.6, 0.8) if cplx else -2.0
    beta = complex(0.0, 0.5) if cplx else 0.5
    Af = np.ascontiguousarray(np.swapaxes(A, 1, 2)).reshape(-1)
    Bf = np.ascontiguousarray(np.swapaxes(B, 1, 2)).reshape(-1)
    Cf = np.ascontiguousarray(np.swapaxes(C, 1, 2)).reshape(-1)
    out = oracle.bound_strided("C", "N", m, n, k, alpha, Af, k, k * m, Bf, k, k * n, beta, Cf, m, m * n, 3)
    ref = abs(alpha) * (np.abs(hp(np_op(A, "C"))) @ np.abs(hp(B))) + abs(beta) * np.abs(hp(C))
    assert np.allclose(out, ref, rtol=1e-14, atol=0)
