"""64-bit addressing: element offsets beyond 2^31 in every place an offset
is formed -- the batch stride (the paper's int `lda2` would overflow here),
the run offset of the LDS-staged kernel over a packed batch larger than 2^31
elements, and the column offset of a large leading dimension.  The buffers
(tens of GB) are left uninitialised except where the matrices live; the
matrices are checked against the oracle through the 4 max(k,1) u test."""
import numpy as np
import pytest
import torch

import oracle
from paper_1304_7053_amd import inputs, sbg
from gpu_util import normalised_error, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BIG = (1 << 31) + 11


def _check(got, A, B, C, ta, tb, m, n, k, alpha, beta):
    """got, A, B, C: host arrays of packed matrices (batch, flat)."""
    ra, ca = (m, k) if ta == "N" else (k, m)
    rb, cb = (k, n) if tb == "N" else (n, k)
    N = A.shape[0]
    args = (ta, tb, m, n, k, alpha, A.ravel(), ra, ra * ca, B.ravel(), rb, rb * cb, beta, C.ravel(), m, m * n, N)
    hi, lo = oracle.gemm_strided(*args, ext=True)
    bnd = oracle.bound_strided(*args)
    got_mn = np.swapaxes(got.reshape(N, n, m), 1, 2).astype(np.float64)   # column-major -> (batch, m, n)
    e = normalised_error(got_mn, hi, lo, bnd)
    assert np.max(e) <= 4 * max(k, 1) * U32, np.max(e) / U32


def test_batch_stride_beyond_int32():
    """strideA = strideB = strideC = 2^31 + 11 elements, three matrices
    (48 GiB of f32 buffers)."""
    g = inputs.rng(301)
    m = n = k = 5
    N = 3
    say(f"stride {BIG} elements, allocating {3 * (2 * BIG + 25) * 4 / 2**30:.1f} GiB")
    dA = torch.empty(2 * BIG + 25, dtype=torch.float32, device="cuda")
    dB = torch.empty_like(dA)
    dC = torch.empty_like(dA)
    A = inputs.uniform(g, (N, 25), np.float32)
    B = inputs.uniform(g, (N, 25), np.float32)
    C = inputs.uniform(g, (N, 25), np.float32)
    for p in range(N):
        dA[p * BIG:p * BIG + 25] = torch.from_numpy(A[p]).cuda()
        dB[p * BIG:p * BIG + 25] = torch.from_numpy(B[p]).cuda()
        dC[p * BIG:p * BIG + 25] = torch.from_numpy(C[p]).cuda()
    sbg.gemm_strided("N", "T", m, n, k, 1.5, dA, m, BIG, dB, n, BIG, -0.5, dC, m, BIG, N)
    torch.cuda.synchronize()
    got = np.stack([dC[p * BIG:p * BIG + 25].cpu().numpy() for p in range(N)])
    del dA, dB, dC
    torch.cuda.empty_cache()
    _check(got, A, B, C, "N", "T", m, n, k, 1.5, -0.5)


def test_packed_batch_beyond_int32_elements_staged():
    """A packed f32 batch of 12x12 matrices with more than 2^31 elements per
    operand (staged kernel, 24 GiB); the first, last and sampled matrices are
    checked."""
    m = n = k = 12
    N = (1 << 31) // (m * k) + 4097
    with sbg.tuned(staged=1):
        name = sbg.describe_strided("s", "N", "N", m, n, k, m, m * k, k, k * n, m, m * n, N)
    assert "gemm_staged_kernel" in name
    say(f"packed N={N}, {N * m * k} elements per operand")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 302)
    dA = torch.rand(N * m * k, generator=gen, device="cuda") * 2 - 1
    dB = torch.rand(N * k * n, generator=gen, device="cuda") * 2 - 1
    dC = torch.rand(N * m * n, generator=gen, device="cuda") * 2 - 1
    rs = np.random.default_rng(302)
    idx = np.unique(np.concatenate([[0, 1, N - 2, N - 1], rs.choice(N, 60, replace=False),
                                    [(1 << 31) // (m * k) + d for d in (-1, 0, 1)]]))
    take = lambda t, e: np.stack([t[int(p) * e:(int(p) + 1) * e].cpu().numpy() for p in idx])  # noqa: E731
    A, B, C = take(dA, m * k), take(dB, k * n), take(dC, m * n)
    with sbg.tuned(staged=1):
        sbg.gemm_strided("N", "N", m, n, k, 1.5, dA, m, m * k, dB, k, k * n, -0.5, dC, m, m * n, N)
    torch.cuda.synchronize()
    got = take(dC, m * n)
    del dA, dB, dC
    torch.cuda.empty_cache()
    _check(got, A, B, C, "N", "N", m, n, k, 1.5, -0.5)


def test_leading_dimension_offsets_beyond_int32():
    """lda = ldb = ldc = 2^30 + 5 with three columns: column offsets reach
    2^31 + 10 elements (24 GiB); one matrix, all four op pairs."""
    g = inputs.rng(303)
    ld = (1 << 30) + 5
    m = n = k = 3
    size = 2 * ld + 3
    say(f"ld {ld}, allocating {3 * size * 4 / 2**30:.1f} GiB")
    dA = torch.empty(size, dtype=torch.float32, device="cuda")
    dB = torch.empty_like(dA)
    dC = torch.empty_like(dA)
    for ta in "NT":
        for tb in "NT":
            A = inputs.uniform(g, (3, 3), np.float32)   # (column, row) of the stored 3x3
            B = inputs.uniform(g, (3, 3), np.float32)
            C = inputs.uniform(g, (3, 3), np.float32)
            for j in range(3):
                dA[j * ld:j * ld + 3] = torch.from_numpy(A[j]).cuda()
                dB[j * ld:j * ld + 3] = torch.from_numpy(B[j]).cuda()
                dC[j * ld:j * ld + 3] = torch.from_numpy(C[j]).cuda()
            sbg.gemm_strided(ta, tb, m, n, k, 1.5, dA, ld, 0, dB, ld, 0, -0.5, dC, ld, 0, 1)
            torch.cuda.synchronize()
            got = np.stack([dC[j * ld:j * ld + 3].cpu().numpy() for j in range(3)])
            say(f"large ld {ta}{tb}")
            _check(got.reshape(1, 9), A.reshape(1, 9), B.reshape(1, 9), C.reshape(1, 9), ta, tb, m, n, k, 1.5, -0.5)
    del dA, dB, dC
    torch.cuda.empty_cache()
