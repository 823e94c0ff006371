"""GPU parity of the batched LU factorisation (sbg_?getrf_strided_batched)
against the LU oracle (oracle/lu.py).

Partial pivoting makes the factors unique only where every pivot choice is
clear-cut, so the checks are:
  * exact data -- A = P^T L U with L's multipliers in {0, +-1/2, +-1/4} and
    small integer U: every operation is exact in binary32, the pivots are
    forced, and factors, interchanges and info must equal the oracle's bit
    for bit (also with a zero last pivot: info = n);
  * random data -- the backward error |P A - L U| <= 4 n u |L| |U| elementwise
    with the GPU's own interchanges, every multiplier of magnitude <= 1, and
    the interchanges equal to the oracle's wherever the oracle's choice has a
    margin above 1e-3 at every step (elsewhere: only valid interchanges)."""
import numpy as np
import pytest
import torch

from oracle import lu
from paper_1304_7053_amd import inputs, sbg
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

UNIT = {np.float32: 2.0 ** -24, np.float64: 2.0 ** -53}


def run(dtype, n, X, lda, stride, batch, sP=None):
    sP = sP if sP is not None else max(n, 1)
    dA = to_dev(X)
    ipiv = torch.full((max(batch * sP, 1),), -5, dtype=torch.int32, device="cuda")
    info = torch.full((max(batch, 1),), -5, dtype=torch.int32, device="cuda")
    sbg.getrf_strided(n, dA, lda, stride, ipiv, sP, info, batch)
    torch.cuda.synchronize()
    return from_dev(dA), from_dev(ipiv), from_dev(info)


def mat(X, off, lda, n):
    return X[off + np.arange(n)[:, None] + lda * np.arange(n)[None, :]]


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 11, 16, 17, 24, 32])
def test_getrf_random_backward_error(gpu_lib, dtype, n):
    g = inputs.rng(6, salt=n)
    batch = 3001 if n <= 16 else 1001
    lda = n + 1
    stride = lda * n + 2
    X = g.uniform(-1, 1, size=stride * batch).astype(dtype)
    say(f"getrf {np.dtype(dtype).name} n={n} N={batch}")
    out, ipiv, info = run(dtype, n, X, lda, stride, batch)
    assert np.all(info[:batch] == 0)
    _, opiv, oinfo, marg = lu.getrf(n, X, lda, stride, batch)
    u = UNIT[dtype]
    clear = 0
    for p in range(batch):
        F = mat(out, p * stride, lda, n).astype(np.float64)
        piv0 = ipiv[p * n:(p + 1) * n].astype(np.int64) - 1
        assert np.all(piv0 >= np.arange(n)) and np.all(piv0 < n), (p, piv0)
        assert np.all(np.abs(np.tril(F, -1)) <= 1.0), p
        r = lu.getrf_residual(mat(X, p * stride, lda, n), F, piv0)
        assert r <= 4 * n * u, (p, r / u)
        if np.all(marg[p] > 1 + 1e-3):
            clear += 1
            assert np.array_equal(piv0, opiv[p]), (p, piv0, opiv[p])
    assert clear >= batch // 2
    # padding between the matrices keeps its values
    keep = np.ones(X.size, dtype=bool)
    for p in range(batch):
        keep[p * stride + np.arange(n)[:, None] + lda * np.arange(n)[None, :]] = False
    assert np.array_equal(out[keep], X[keep])


def exact_batch(g, n, batch, singular=False):
    """A_p = P_p^T L_p U_p with multipliers in {0, +-1/2, +-1/4} and integer U
    (|u| <= 4): every partial-pivoting step is exact and forced.  (A zero
    pivot earlier than the last would leave ties, and the tie-broken choice
    can bring non-dyadic quotients, rounded differently in each precision.)"""
    mats = []
    for _ in range(batch):
        L = np.tril(g.choice([0.0, 0.5, -0.5, 0.25, -0.25], size=(n, n)), -1) + np.eye(n)
        U = np.triu(g.integers(-4, 5, size=(n, n)).astype(np.float64))
        d = g.integers(1, 5, size=n) * g.choice([-1, 1], size=n)
        U[np.arange(n), np.arange(n)] = d
        if singular:
            U[n - 1, n - 1] = 0.0        # the last pivot: earlier ones stay forced and exact
        perm = g.permutation(n)
        A = np.empty((n, n))
        A[perm] = L @ U                  # row i of P A is row perm[i] of A
        mats.append(A)
    return mats


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("n", [3, 7, 12, 16, 20, 32])
@pytest.mark.parametrize("singular", [False, True], ids=["full", "singular"])
def test_getrf_exact_data_bit_exact(gpu_lib, dtype, n, singular):
    g = inputs.rng(6, salt=100 + n + (50 if singular else 0))
    batch = 257
    mats = exact_batch(g, n, batch, singular)
    lda, stride = n, n * n
    X = np.concatenate([M.T.reshape(-1) for M in mats]).astype(dtype)
    say(f"getrf exact {np.dtype(dtype).name} n={n} singular={singular}")
    out, ipiv, info = run(dtype, n, X, lda, stride, batch)
    F, opiv, oinfo, _ = lu.getrf(n, X, lda, stride, batch)
    assert np.array_equal(info[:batch], oinfo)
    if singular:
        assert np.all(oinfo == n)
    assert np.array_equal(ipiv[:batch * n].reshape(batch, n) - 1, opiv)
    got = np.stack([mat(out, p * stride, lda, n) for p in range(batch)]).astype(np.float64)
    assert np.array_equal(got, F)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_getrf_edges(gpu_lib, dtype):
    g = inputs.rng(6, salt=7)
    # n = 0: every info is set to 0
    out, ipiv, info = run(dtype, 0, np.zeros(4, dtype=dtype), 1, 0, 3, sP=0)
    assert np.all(info[:3] == 0)
    # zero matrices: all pivots zero, info = 1, no interchanges, factors zero
    n, batch = 6, 65
    X = np.zeros(n * n * batch, dtype=dtype)
    out, ipiv, info = run(dtype, n, X, n, n * n, batch)
    assert np.all(info[:batch] == 1)
    assert np.array_equal(ipiv[:batch * n].reshape(batch, n), np.tile(np.arange(1, n + 1), (batch, 1)))
    assert np.all(out == 0)
    # ties: |1| == |-1| in column 0 keeps the first row (LAPACK's first maximum)
    M = np.array([[1.0, 2.0], [-1.0, 3.0]])
    out, ipiv, info = run(dtype, 2, M.T.reshape(-1).astype(dtype), 2, 4, 1)
    assert list(ipiv[:2]) == [1, 2] and info[0] == 0
    # a batch whose size is not a multiple of the matrices per wave
    n, batch = 5, 37
    X = g.uniform(-1, 1, size=n * n * batch).astype(dtype)
    out, ipiv, info = run(dtype, n, X, n, n * n, batch)
    for p in range(batch):
        r = lu.getrf_residual(mat(X, p * n * n, n, n), mat(out, p * n * n, n, n).astype(np.float64),
                              ipiv[p * n:(p + 1) * n].astype(np.int64) - 1)
        assert r <= 4 * n * UNIT[dtype]
