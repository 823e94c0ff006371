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

    def describe(self):
        """Name of the kernel the library picks for this case's strided call."""
        prefix = {np.float32: "s", np.float64: "d", np.complex64: "c", np.complex128: "z"}[np.dtype(self.dtype).type]
        return sbg.describe_strided(prefix, self.ta, self.tb, self.m, self.n, self.k,
                                    self.lda, self.sA, self.ldb, self.sB, self.ldc, self.sC, self.batch)

    def unpack(self, flat, idx=None):
        """(len(idx), m, n) view of matrices idx of a flat C-layout array."""
        idx = np.arange(self.batch) if idx is None else np.asarray(idx)
        p = idx[:, None, None].astype(np.int64)
        i = np.arange(self.m)[None, :, None]
        j = np.arange(self.n)[None, None, :]
        return flat[p * self.sC + i + j * self.ldc]

    def oracle(self, idx=None, A=None, B=None, C=None, ext=True):
        idx = np.arange(self.batch) if idx is None else np.asarray(idx, dtype=np.int64)
        A = self.A if A is None else A
        B = self.B if B is None else B
        C = self.C if C is None else C
        args = (self.ta, self.tb, self.m, self.n, self.k, self.alpha, A, idx * self.sA, self.lda,
                B, idx * self.sB, self.ldb, self.beta, C, idx * self.sC, self.ldc, len(idx))
        hi, lo, offO, _, _ = oracle.gemm_general(*args, ext=ext)
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


class VarCase:
    """A variable-size batch: matrix p has sizes (m_p, n_p, k_p) and its own
    leading dimensions; all matrices of one operand live in one flat buffer at
    host-chosen element offsets (gaps filled with NaN), addressed through
    device pointer arrays."""

    def __init__(self, dtype, ta, tb, dims, alpha, beta, g, pad=True, dist="uniform", store=None):
        self.dtype, self.ta, self.tb = dtype, ta, tb
        self.m, self.n, self.k = (np.asarray(d, dtype=np.int32) for d in dims)
        self.batch = len(self.m)
        self.alpha, self.beta = alpha, beta
        self.store = store or dtype       # storage dtype of A and B (numpy)
        ra = np.where(ta in "NnRr", self.m, self.k)
        ca = np.where(ta in "NnRr", self.k, self.m)
        rb = np.where(tb in "NnRr", self.k, self.n)
        cb = np.where(tb in "NnRr", self.n, self.k)
        extra = (g.integers(0, 3, size=(3, self.batch)) if pad else np.zeros((3, self.batch), dtype=np.int64))
        self.lda = (np.maximum(ra, 1) + extra[0]).astype(np.int32)
        self.ldb = (np.maximum(rb, 1) + extra[1]).astype(np.int32)
        self.ldc = (np.maximum(self.m, 1) + extra[2]).astype(np.int32)
        self.A, self.offA = self._fill(g, ra, ca, self.lda, dist, pad)
        self.B, self.offB = self._fill(g, rb, cb, self.ldb, dist, pad)
        self.C, self.offC = self._fill(g, self.m, self.n, self.ldc, dist, pad)

    def _fill(self, g, rows, cols, ld, dist, pad):
        sizes = np.where(cols > 0, ld.astype(np.int64) * np.maximum(cols, 0), 0) + (g.integers(0, 5, self.batch)
                                                                                    if pad else 0)
        sizes = np.maximum(sizes, 1)
        off = np.zeros(self.batch, dtype=np.int64)
        off[1:] = np.cumsum(sizes)[:-1]
        buf = np.full(int(sizes.sum()), np.nan, dtype=self.dtype)
        for p in range(self.batch):
            r, c = int(rows[p]), int(cols[p])
            if r > 0 and c > 0:
                vals = inputs.DISTS[dist](g, (c, r), self.dtype)
                idx = off[p] + np.arange(c)[:, None] * ld[p] + np.arange(r)[None, :]
                buf[idx] = vals
        return buf, off

    def device(self, A=None, B=None, C=None):
        """Device buffers, pointer arrays and size arrays (dict)."""
        esz = np.dtype(self.dtype).itemsize
        dA = to_dev(self.A if A is None else A)
        dB = to_dev(self.B if B is None else B)
        dC = to_dev(self.C if C is None else C)
        aesz = dA.element_size()
        d = dict(A=dA, B=dB, C=dC,
                 pA=torch.tensor(dA.data_ptr() + self.offA * aesz, dtype=torch.int64, device="cuda"),
                 pB=torch.tensor(dB.data_ptr() + self.offB * dB.element_size(), dtype=torch.int64, device="cuda"),
                 pC=torch.tensor(dC.data_ptr() + self.offC * esz, dtype=torch.int64, device="cuda"))
        for name in ("m", "n", "k", "lda", "ldb", "ldc"):
            d[name] = torch.from_numpy(getattr(self, name).astype(np.int32)).to("cuda")
        d["ws"] = torch.zeros(sbg.vbatched_workspace_size(self.batch) // 4 + 1, dtype=torch.int32, device="cuda")
        return d

    def run_gpu(self, maxes=(16, 16, 16), d=None):
        d = d or self.device()
        sbg.gemm_vbatched(self.ta, self.tb, d["m"], d["n"], d["k"], maxes[0], maxes[1], maxes[2], self.alpha,
                          d["pA"], d["lda"], d["pB"], d["ldb"], self.beta, d["pC"], d["ldc"], self.batch, d["ws"],
                          d["C"].dtype)
        torch.cuda.synchronize()
        return from_dev(d["C"]), d

    def oracle(self, idx=None, types=None, scaleA=None, scaleB=None, A=None, B=None):
        idx = np.arange(self.batch) if idx is None else np.asarray(idx)
        sl = lambda v: v[idx]  # noqa: E731
        A = self.A if A is None else A
        B = self.B if B is None else B
        args = (self.ta, self.tb, sl(self.m), sl(self.n), sl(self.k), self.alpha, A, sl(self.offA), sl(self.lda),
                B, sl(self.offB), sl(self.ldb), self.beta, self.C, sl(self.offC), sl(self.ldc), len(idx))
        kw = dict(types=types, scaleA=None if scaleA is None else scaleA[idx],
                  scaleB=None if scaleB is None else scaleB[idx])
        hi, lo, offO, mm, nn = oracle.gemm_general(*args, ext=True, **kw)
        bnd, _ = oracle.bound_general(*args, **kw)
        return hi, lo, bnd, offO, mm, nn

    def got(self, Cflat, p):
        m, n, ld = int(self.m[p]), int(self.n[p]), int(self.ldc[p])
        return Cflat[self.offC[p] + np.arange(m)[:, None] + np.arange(n)[None, :] * ld]


def check_var(case, Cflat, idx=None, unit_=None, kmul=1, label="", types=None, scaleA=None, scaleB=None, A=None,
              B=None):
    """Every matrix of a VarCase (or the subset idx) against the oracle:
    max normalised error <= 4 * kmul * max(k_p, 1) * u."""
    idx = np.arange(case.batch) if idx is None else np.asarray(idx)
    hi, lo, bnd, offO, mm, nn = case.oracle(idx, types=types, scaleA=scaleA, scaleB=scaleB, A=A, B=B)
    cplx = np.dtype(case.dtype).kind == "c"
    u = unit(case.dtype) if unit_ is None else unit_
    worst = 0.0
    bstart = np.concatenate([[0], np.cumsum(mm.astype(np.int64) * nn)])   # bound: one slot per entry
    for q, p in enumerate(idx):
        m, n = int(mm[q]), int(nn[q])
        if m == 0 or n == 0:
            continue
        o = int(offO[q])
        if cplx:
            ref = (hi[o:o + 2 * m * n:2] + 1j * hi[o + 1:o + 2 * m * n:2]).reshape(n, m).T
            rlo = (lo[o:o + 2 * m * n:2] + 1j * lo[o + 1:o + 2 * m * n:2]).reshape(n, m).T
        else:
            ref = hi[o:o + m * n].reshape(n, m).T
            rlo = lo[o:o + m * n].reshape(n, m).T
        b = bnd[bstart[q]:bstart[q] + m * n].reshape(n, m).T
        e = normalised_error(case.got(Cflat, p), ref, rlo, b)
        tol = 4 * kmul * max(int(case.k[p]), 1) * u
        w = float(np.max(e))
        assert w <= tol, (f"{label} matrix {p} ({m}x{n}x{int(case.k[p])}) {case.ta}{case.tb}: "
                          f"{w:.3e} > {tol:.3e} ({w / u:.2f} u)")
        worst = max(worst, w / u)
    return worst
