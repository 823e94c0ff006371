"""Pins of the batched LU oracle (oracle/lu.py) against what mathematics and
an independent implementation fix: a factorisation worked by hand, exact
rational elimination, LAPACK's dgetrf (scipy), singular and tie cases, and
the backward-error check rejecting wrong factors."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import lu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lu_3x3.json")


def frac(x):
    return Fraction(x) if isinstance(x, str) else Fraction(int(x))


def test_worked_example():
    g = json.load(open(GOLDEN))
    A = np.array(g["A_rows"], dtype=np.float64)
    F, ipiv, info, _ = lu.getrf_one(A)
    assert list(ipiv) == g["ipiv0"] and info == 0
    L = [[frac(x) for x in r] for r in g["L_rows"]]
    U = [[frac(x) for x in r] for r in g["U_rows"]]
    for i in range(3):
        for j in range(3):
            want = L[i][j] if j < i else U[i][j]
            assert abs(float(F[i, j]) - float(want)) <= 1e-18 * max(1.0, abs(float(want))), (i, j)


def exact_lu(rows):
    """Partial-pivoting elimination in rational arithmetic (largest
    magnitude, first on ties)."""
    A = [[Fraction(int(x)) for x in r] for r in rows]
    n = len(A)
    piv = []
    info = 0
    for k in range(n):
        p = max(range(k, n), key=lambda i: (abs(A[i][k]), -i))
        piv.append(p)
        A[k], A[p] = A[p], A[k]
        if A[k][k] != 0:
            for i in range(k + 1, n):
                A[i][k] = A[i][k] / A[k][k]
        elif info == 0:
            info = k + 1
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                A[i][j] -= A[i][k] * A[k][j]
    return A, piv, info


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_matches_exact_rational_elimination(n):
    g = np.random.default_rng(100 + n)
    for _ in range(20):
        M = g.integers(-9, 10, size=(n, n))
        E, piv, info = exact_lu(M.tolist())
        F, ipiv, inf, _ = lu.getrf_one(M.astype(np.float64))
        assert list(ipiv) == piv and inf == info
        for i in range(n):
            for j in range(n):
                e = float(E[i][j])
                assert abs(float(F[i, j]) - e) <= 1e-15 * max(1.0, abs(e)), (i, j, float(F[i, j]), e)


@pytest.mark.parametrize("n", [1, 4, 9, 16, 32])
def test_matches_lapack_dgetrf(n):
    g = np.random.default_rng(7 + n)
    for _ in range(10):
        M = g.uniform(-1, 1, size=(n, n))
        ref, piv, info = lapack.dgetrf(M)
        F, ipiv, inf, _ = lu.getrf_one(M)
        assert info == inf == 0
        assert np.array_equal(piv, ipiv)              # scipy's piv is 0-based
        assert np.max(np.abs(F.astype(np.float64) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_singular_and_ties_follow_lapack():
    # a zero column at step 1 (after the first elimination), ties in column 0
    cases = [
        np.array([[2.0, 4.0, 1.0], [1.0, 2.0, 3.0], [-2.0, -4.0, 5.0]]),   # column 1 vanishes below the pivot
        np.array([[1.0, 2.0], [-1.0, 3.0]]),                               # |1| == |-1|: the first row stays
        np.zeros((4, 4)),                                                  # every pivot zero
        np.array([[0.0, 1.0], [0.0, 2.0]]),
    ]
    for M in cases:
        ref, piv, info = lapack.dgetrf(M)
        F, ipiv, inf, _ = lu.getrf_one(M)
        assert inf == info, (M, inf, info)
        assert np.array_equal(piv, ipiv), (M, ipiv, piv)
        assert np.allclose(F.astype(np.float64), ref, atol=0, rtol=1e-15)


def test_residual_accepts_factors_and_rejects_wrong_ones():
    g = np.random.default_rng(5)
    n = 12
    M = g.uniform(-1, 1, size=(n, n))
    F, ipiv, _, _ = lu.getrf_one(M)
    F64 = F.astype(np.float64)
    u = 2.0 ** -53
    accept = 2 * n * u
    assert lu.getrf_residual(M, F64, ipiv) <= accept
    bad = F64.copy()
    bad[5, 3] *= 1 + 1e-9                                   # a perturbed multiplier
    assert lu.getrf_residual(M, bad, ipiv) > 1e3 * accept
    wrong = ipiv.copy()
    wrong[0] = (wrong[0] + 1) % n                           # a wrong interchange
    assert lu.getrf_residual(M, F64, wrong) > 1e-3
    flipped = F64.copy()
    flipped[2, 7] = -flipped[2, 7]                          # a sign error in U
    assert lu.getrf_residual(M, flipped, ipiv) > 1e-3


def test_batched_layout():
    g = np.random.default_rng(9)
    n, lda, batch = 5, 7, 6
    stride = lda * n + 3
    X = g.uniform(-1, 1, size=stride * batch)
    F, piv, info, _ = lu.getrf(n, X, lda, stride, batch)
    for p in range(batch):
        M = X[p * stride + np.arange(n)[:, None] + lda * np.arange(n)[None, :]]
        ref, pv, inf = lapack.dgetrf(M)
        assert np.array_equal(pv, piv[p]) and inf == info[p]
        assert np.allclose(F[p], ref, rtol=1e-13, atol=1e-15)
