"""Helpers for the GPU parity tests: build seeded batches on the host, run the
library through its C-ABI binding, and score the result against the CPU
oracle with the acceptance test

    max |C - Cref| / (|alpha| (|op A| |op B|) + |beta| |C_in|)  <=  4 max(k, 1) u

(u = 2^-24 for S/C, 2^-53 for D/Z; entries whose denominator is 0 must match
exactly).  The oracle runs in long-double mode so that its own rounding does
not blur the D/Z comparison."""
import sys

import numpy as np
import torch

import oracle
from paper_1304_7053_amd import inputs, sbg

UNIT = {np.float32: 2.0 ** -24, np.complex64: 2.0 ** -24, np.float64: 2.0 ** -53, np.complex128: 2.0 ** -53}
TORCH = {np.float32: torch.float32, np.float64: torch.float64, np.complex64: torch.complex64,
         np.complex128: torch.complex128}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def unit(dtype):
    return UNIT[np.dtype(dtype).type]


def stored_dims(op, rows, cols):
    return (rows, cols) if op in "NnRr" else (cols, rows)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def from_dev(t):
    return t.cpu().numpy()


class Case:
    """One strided batched GEMM with host copies of every input."""

    def __init__(self, dtype, ta, tb, m, n, k, batch, alpha, beta, g, lda=None, ldb=None, ldc=None,
                 pad_stride=0, dist="uniform", fill=np.nan):
        self.dtype, self.ta, self.tb = dtype, ta, tb
        self.m, self.n, self.k, self.batch = m, n, k, batch
        self.alpha, self.beta = alpha, beta
        ra, ca = stored_dims(ta, m, k)
        rb, cb = stored_dims(tb, k, n)
        self.lda = lda if lda is not None else max(ra, 1)
        self.ldb = ldb if ldb is not None else max(rb, 1)
        self.ldc = ldc if ldc is not None else max(m, 1)
        self.sA = self.lda * ca + pad_stride
        self.sB = self.ldb * cb + pad_stride
        self.sC = self.ldc * n + pad_stride
        self.A = inputs.strided_batch(g, batch, ra, ca, self.lda, self.sA, dtype, dist, fill)
        self.B = inputs.strided_batch(g, batch, rb, cb, self.ldb, self.sB, dtype, dist, fill)
        self.C = inputs.strided_batch(g, batch, m, n, self.ldc, self.sC, dtype, dist, fill)

    def run_gpu(self, A=None, B=None, C=None):
        dA = to_dev(self.A if A is None else A) if self.A.size else torch.empty(1, dtype=TORCH[np.dtype(self.dtype).type], device="cuda")
        dB = to_dev(self.B if B is None else B) if self.B.size else torch.empty(1, dtype=dA.dtype, device="cuda")
        dC = to_dev(self.C if C is None else C) if self.C.size else torch.empty(1, dtype=dA.dtype, device="cuda")
        sbg.gemm_strided(self.ta, self.tb, self.m, self.n, self.k, self.alpha, dA, self.lda, self.sA,
                         dB, self.ldb, self.sB, self.beta, dC, self.ldc, self.sC, self.batch)
        torch.cuda.synchronize()
        return from_dev(dC)

    def unpack(self, flat, idx=None):
        """(len(idx), m, n) view of matrices idx of a flat C-layout array."""
        idx = np.arange(self.batch) if idx is None else np.asarray(idx)
        p = idx[:, None, None].astype(np.int64)
        i = np.arange(self.m)[None, :, None]
        j = np.arange(self.n)[None, None, :]
        return flat[p * self.sC + i + j * self.ldc]

    def oracle(self, idx=None, A=None, B=None, C=None):
        idx = np.arange(self.batch) if idx is None else np.asarray(idx, dtype=np.int64)
        A = self.A if A is None else A
        B = self.B if B is None else B
        C = self.C if C is None else C
        args = (self.ta, self.tb, self.m, self.n, self.k, self.alpha, A, idx * self.sA, self.lda,
                B, idx * self.sB, self.ldb, self.beta, C, idx * self.sC, self.ldc, len(idx))
        hi, lo, offO, _, _ = oracle.gemm_general(*args, ext=True)
        bnd, _ = oracle.bound_general(*args)
        cplx = np.dtype(self.dtype).kind == "c"
        cnt = len(idx)
        if cplx:
            ref = (hi[0::2] + 1j * hi[1::2])[: cnt * self.m * self.n]
            rlo = (lo[0::2] + 1j * lo[1::2])[: cnt * self.m * self.n]
        else:
            ref, rlo = hi[: cnt * self.m * self.n], lo[: cnt * self.m * self.n]
        shape = (cnt, self.n, self.m)
        tr = lambda v: np.swapaxes(v.reshape(shape), 1, 2)  # noqa: E731
        return tr(ref), tr(rlo), tr(bnd[: cnt * self.m * self.n])


def normalised_error(got, ref, lo, bound):
    """Per-entry |got - ref| / bound; entries with bound 0 must be exact
    (returns +inf where they are not)."""
    wide = got.astype(np.complex128 if np.iscomplexobj(got) else np.float64)
    diff = np.abs((wide - ref) - lo)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(bound > 0, diff / np.where(bound > 0, bound, 1.0), np.where(diff == 0, 0.0, np.inf))
    e = np.where(np.isnan(diff), np.inf, e)
    return e


def check(case, got_flat, idx=None, label=""):
    idx = np.arange(case.batch) if idx is None else np.asarray(idx)
    got = case.unpack(got_flat, idx)
    ref, lo, bnd = case.oracle(idx)
    e = normalised_error(got, ref, lo, bnd)
    tol = 4 * max(case.k, 1) * unit(case.dtype)
    worst = float(np.max(e)) if e.size else 0.0
    assert worst <= tol, (f"{label} {np.dtype(case.dtype).name} {case.ta}{case.tb} m={case.m} n={case.n} "
                          f"k={case.k} batch={case.batch}: max normalised error {worst:.3e} > {tol:.3e} "
                          f"(= {worst / unit(case.dtype):.2f} u)")
    return worst / unit(case.dtype)
