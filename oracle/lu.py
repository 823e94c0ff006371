"""Oracle for batched LU factorisation with partial pivoting -- TEST
INFRASTRUCTURE ONLY.

The paper proposes formulating other batched BLAS/LAPACK kernels on its
batched interface (Sec. 9, Discussion); LU is the first of them.  What it
computes is fixed by the LAPACK definition of GETRF: P A = L U, with L unit
lower triangular, U upper triangular, and the row interchanges chosen column
by column as the entry of largest magnitude on and below the diagonal (the
first such entry on ties).  This module writes out right-looking elimination
in that order, one matrix at a time, in extended precision (numpy's
longdouble, a 64-bit significand on x86-64):

  for k = 0 .. n-1:
      p = first index of max |A[k:, k]| (+ k);  ipiv[k] = p (0-based here)
      swap rows k and p (whole rows)
      if A[k, k] != 0:  A[k+1:, k] /= A[k, k]          (the multipliers)
      else:             info = k + 1 if no earlier zero pivot
      A[k+1:, k+1:] -= A[k+1:, k] A[k, k+1:]

The factors overwrite A (L strictly below the diagonal, U on and above).
Storage is column-major: element (i, j) of matrix p is X[off_p + i + ld j].

getrf_residual gives the backward error of computed factors: the elementwise
ratio |P A - L U| / (|L| |U|), evaluated in extended precision; a backward
stable elimination keeps it below gamma_n = n u / (1 - n u) (Higham,
Accuracy and Stability of Numerical Algorithms, Thm. 9.3).
"""
import numpy as np

LD = np.longdouble


def _mat(X, off, ld, n):
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return np.asarray(X)[off + i + ld * j].astype(LD)


def getrf_one(M):
    """In-place LU with partial pivoting of one square wide matrix; returns
    (factors, ipiv 0-based, info, margins) -- margins[k] is the ratio of the
    largest to the second largest candidate magnitude at step k (inf when
    there is a single candidate or the second is zero), for callers that
    need to know whether a pivot choice was clear-cut."""
    A = np.array(M, dtype=LD)
    n = A.shape[0]
    ipiv = np.zeros(n, dtype=np.int64)
    margins = np.full(n, np.inf)
    info = 0
    for k in range(n):
        col = np.abs(A[k:, k])
        p = int(np.argmax(col)) + k            # argmax returns the first maximum
        ipiv[k] = p
        if len(col) > 1:
            srt = np.sort(col)[::-1]
            margins[k] = float(srt[0] / srt[1]) if srt[1] != 0 else np.inf
        if p != k:
            A[[k, p], :] = A[[p, k], :]
        if A[k, k] != 0:
            A[k + 1:, k] /= A[k, k]
        elif info == 0:
            info = k + 1
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A, ipiv, info, margins


def getrf(n, A, lda, sA, batch):
    """Batched LU of the n x n matrices A_p at offsets sA p.  Returns
    (factors as a (batch, n, n) float64 array of the extended-precision
    result, ipiv (batch, n) 0-based, info (batch,), margins (batch, n))."""
    F = np.zeros((batch, n, n))
    piv = np.zeros((batch, n), dtype=np.int64)
    info = np.zeros(batch, dtype=np.int64)
    marg = np.zeros((batch, n))
    for p in range(batch):
        f, ip, inf, mg = getrf_one(_mat(A, sA * p, lda, n))
        F[p] = f.astype(np.float64)
        piv[p] = ip
        info[p] = inf
        marg[p] = mg
    return F, piv, info, marg


def permutation(ipiv):
    """Row order produced by applying the interchanges ipiv (0-based) in
    sequence: row i of P A is row perm[i] of A."""
    perm = np.arange(len(ipiv))
    for k, p in enumerate(ipiv):
        perm[[k, p]] = perm[[p, k]]
    return perm


def getrf_residual(A0, F, ipiv):
    """Elementwise backward error of factors F (n x n, L unit lower below the
    diagonal, U on and above) with interchanges ipiv (0-based) for the
    original matrix A0: max over entries of |P A0 - L U| / (|L| |U|)
    (0/0 counts as 0, x/0 as inf)."""
    A0 = np.asarray(A0, dtype=LD)
    F = np.asarray(F, dtype=LD)
    n = A0.shape[0]
    L = np.tril(F, -1) + np.eye(n, dtype=LD)
    U = np.triu(F)
    PA = A0[permutation(ipiv)]
    R = np.abs(PA - L @ U)
    D = np.abs(L) @ np.abs(U)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(R == 0, 0, R / D)
    return float(np.max(ratio)) if ratio.size else 0.0
