"""Oracle for batched GEMV and TRSM in the paper's second-leading-dimension
interface -- TEST INFRASTRUCTURE ONLY.

The paper proposes carrying its batched interface over to other BLAS routines
and formulating them in terms of batched GEMM (Sec. 9).  What those routines
compute is fixed by their BLAS definitions; this module writes the
definitions out, one matrix at a time, in extended precision (numpy's
longdouble: 64-bit significand on x86-64), and returns each result as a
binary64 pair hi + lo.

Storage (column-major, sizes in elements): element (i, j) of matrix p is
X[offX_p + i + ld j] with offX_p = strideX p; element i of vector p is
x[stridex p + inc i].

  gemv:  y_p <- alpha op(A_p) x_p + beta y_p        A_p m x n, op in N, T, C;
         op(A_p) has rows m (N) or n (T, C).
  trsm:  side L: op(A_p) X_p = alpha B_p,  side R: X_p op(A_p) = alpha B_p;
         A_p triangular: uplo U uses only the upper triangle, L only the
         lower; diag U takes the diagonal as ones and never reads it; the
         solution X_p (m x n) replaces B_p.

trsm is substitution on the triangular system: for side L the columns of B
are solved one by one, forward when op(A) is lower triangular, backward when
it is upper; side R solves op(A)^T X^T = alpha B^T the same way (rows of B).
"""
import numpy as np

LD = np.longdouble
CLD = np.clongdouble


def _wide(dtype):
    return CLD if np.dtype(dtype).kind == "c" else LD


def _mat(X, off, ld, rows, cols, wide):
    """Stored rows x cols matrix at offset off, as a wide array."""
    i = np.arange(rows)[:, None]
    j = np.arange(cols)[None, :]
    return np.asarray(X)[off + i + ld * j].astype(wide)


def _op(M, op):
    if op in "Nn":
        return M
    if op in "Tt":
        return M.T
    if op in "Cc":
        return np.conj(M).T
    raise ValueError(op)


def _split(v):
    """Wide values as a binary64 pair (hi, lo), complex kept as complex128."""
    if np.iscomplexobj(v):
        hr, hi_ = v.real.astype(np.float64), v.imag.astype(np.float64)
        lr = (v.real - hr.astype(LD)).astype(np.float64)
        li = (v.imag - hi_.astype(LD)).astype(np.float64)
        return hr + 1j * hi_, lr + 1j * li
    h = v.astype(np.float64)
    return h, (v - h.astype(LD)).astype(np.float64)


def gemv(trans, m, n, alpha, A, lda, sA, x, incx, sx, beta, y, incy, sy, batch):
    """Reference y for every matrix of the batch: returns (hi, lo, bound),
    each (batch, len_y); bound = |alpha| (|op A| |x|) + |beta| |y_in|, the
    denominator of the normalised error."""
    wide = _wide(np.asarray(A).dtype)
    rows, cols = (m, n) if trans in "Nn" else (n, m)
    al, be = wide(alpha), wide(beta)
    out = np.zeros((batch, rows), dtype=wide)
    bnd = np.zeros((batch, rows), dtype=np.float64)
    for p in range(batch):
        opA = _op(_mat(A, p * sA, lda, m, n, wide), trans)
        xv = np.asarray(x)[p * sx + incx * np.arange(cols)].astype(wide)
        yv = np.asarray(y)[p * sy + incy * np.arange(rows)].astype(wide)
        acc = np.zeros(rows, dtype=wide)
        mag = np.zeros(rows, dtype=LD)
        if alpha != 0:                 # alpha = 0: A and x are not referenced
            for l in range(cols):      # the sum over l, in index order
                acc += opA[:, l] * xv[l]
                mag += np.abs(opA[:, l]) * np.abs(xv[l])
        tot = al * acc
        b = abs(al) * mag
        if beta != 0:                  # beta = 0: y is not referenced
            tot = tot + be * yv
            b = b + abs(be) * np.abs(yv)
        out[p] = tot
        bnd[p] = b.astype(np.float64)
    hi, lo = _split(out)
    return hi, lo, bnd


def triangle(A, off, lda, size, uplo, diag, wide):
    """The triangular matrix the routine uses: the uplo triangle of the
    stored size x size matrix, ones on the diagonal for diag = U (the stored
    diagonal is not read)."""
    i = np.arange(size)[:, None]
    j = np.arange(size)[None, :]
    keep = (i <= j) if uplo in "Uu" else (i >= j)
    if diag in "Uu":
        keep = keep & (i != j)
    idx = off + i + lda * j
    T = np.zeros((size, size), dtype=wide)
    T[keep] = np.asarray(A)[idx[keep]].astype(wide)
    if diag in "Uu":
        T[np.arange(size), np.arange(size)] = 1
    return T


def _substitute(M, rhs, lower):
    """Solve M x = rhs for a triangular M, one right-hand side per column of
    rhs: forward substitution if M is lower triangular, backward if upper."""
    size = M.shape[0]
    X = np.array(rhs, dtype=M.dtype)
    order = range(size) if lower else range(size - 1, -1, -1)
    for i in order:
        others = range(i) if lower else range(i + 1, size)
        for l in others:
            X[i] -= M[i, l] * X[l]
        X[i] = X[i] / M[i, i]
    return X


def trsm(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, batch):
    """Reference X for every matrix: returns (hi, lo) of shape (batch, m, n)
    and the wide solutions themselves (for residual checks)."""
    wide = _wide(np.asarray(B).dtype)
    size = m if side in "Ll" else n
    al = wide(alpha)
    X = np.zeros((batch, m, n), dtype=wide)
    if alpha == 0:                     # X = 0; A and B are not referenced
        hi, lo = _split(X)
        return hi, lo, X
    for p in range(batch):
        T = triangle(A, p * sA, lda, size, uplo, diag, wide)
        opT = _op(T, trans)
        rhs = al * _mat(B, p * sB, ldb, m, n, wide)
        # op(A) is lower triangular for (L, N) and (U, T/C)
        op_lower = (uplo in "Ll") == (trans in "Nn")
        if side in "Ll":
            X[p] = _substitute(opT, rhs, op_lower)
        else:
            X[p] = _substitute(opT.T, rhs.T, not op_lower).T
    hi, lo = _split(X)
    return hi, lo, X


def trsm_residual(side, uplo, trans, diag, m, n, alpha, A, lda, sA, B, ldb, sB, Xgot, batch):
    """Componentwise backward-error ratio of a computed solution Xgot
    (batch, m, n): |op(A) X - alpha B| / (|op(A)| |X| + |alpha B|) for side
    L (X op(A) for side R), evaluated in extended precision.  Substitution
    has a backward error of about size * u relative to |op(A)| |X|."""
    wide = _wide(np.asarray(B).dtype)
    size = m if side in "Ll" else n
    al = wide(alpha)
    worst = np.zeros(batch)
    for p in range(batch):
        opT = _op(triangle(A, p * sA, lda, size, uplo, diag, wide), trans)
        Xw = np.asarray(Xgot[p]).astype(wide)
        rhs = al * _mat(B, p * sB, ldb, m, n, wide)
        if side in "Ll":
            r = opT @ Xw - rhs
            d = np.abs(opT) @ np.abs(Xw) + np.abs(rhs)
        else:
            r = Xw @ opT - rhs
            d = np.abs(Xw) @ np.abs(opT) + np.abs(rhs)
        with np.errstate(divide="ignore", invalid="ignore"):
            e = np.where(d > 0, np.abs(r) / np.where(d > 0, d, 1), np.where(np.abs(r) == 0, 0, np.inf))
        worst[p] = float(np.max(e)) if e.size else 0.0
    return worst
