"""Sizes above 16 (the sub-blocked kernel): parity with the oracle through the
C-ABI, same acceptance test as the small sizes,
|C - Cref| / (|alpha| (|op A||op B|) + |beta||C_in|) <= 4 max(k,1) u.

Shapes cover one and several 16 x 16 output blocks, ragged last blocks in
every dimension, k-chunk groups of 1, 2 and 4 chunks plus a second group
(k > 64), every op pair, padded layouts, the pointer-array form, the alpha /
beta special cases, device scalars, and a full-size batch checked on sampled
matrices."""
import numpy as np
import pytest
import torch

from paper_1304_7053_amd import inputs, sbg
from gpu_util import Case, TORCH, check, from_dev, say, to_dev
import test_gpu_parity as P

pytestmark = pytest.mark.gpu

SHAPES = [(17, 17, 17), (32, 32, 32), (20, 5, 40), (5, 33, 7), (16, 16, 17), (17, 1, 1), (1, 1, 70),
          (48, 16, 64), (33, 31, 65), (64, 64, 64), (24, 40, 100)]


def _kernel(t, m, n, k, ta="N", tb="N"):
    ra, ca = (m, k) if ta == "N" else (k, m)
    rb, cb = (k, n) if tb == "N" else (n, k)
    return sbg.describe_strided(t, ta, tb, m, n, k, ra, ra * ca, rb, rb * cb, m, m * n, 10)


def test_blocked_kernel_selected(gpu_lib):
    for t in "sdcz":
        assert "gemm_blocked_kernel" in _kernel(t, 17, 4, 4)      # one block-column: nothing to share
        assert "gemm_blocked_kernel" in _kernel(t, 4, 4, 100)     # k above 64
        assert "gemm_blocked" not in _kernel(t, 16, 16, 16)
    for t in "sd":
        # the built-in rule: A and B reused, from size 32 on, for s with op(A) N from 48
        assert "gemm_blocked_lds_kernel" in _kernel(t, 64, 64, 64)
        assert "gemm_blocked_lds_kernel" in _kernel(t, 48, 48, 48)
        assert "gemm_blocked_lds_kernel" in _kernel(t, 32, 48, 24, "T", "T")
        assert "gemm_blocked_kernel" in _kernel(t, 24, 24, 24)
        assert "gemm_blocked_kernel" in _kernel(t, 64, 16, 64)
        assert ("gemm_blocked_lds_kernel" in _kernel(t, 32, 32, 32)) == (t == "d")
        with sbg.tuned(blocked=1):
            assert "gemm_blocked_kernel" in _kernel(t, 64, 64, 64)
        with sbg.tuned(blocked=2):
            assert "gemm_blocked_lds_kernel" in _kernel(t, 24, 24, 24)
            assert "gemm_blocked_lds_kernel" in _kernel(t, 20, 4, 8)
            assert "gemm_blocked_kernel" in _kernel(t, 17, 4, 4)  # lda * s not a multiple of 16
    for t in "cz":
        assert "gemm_blocked_kernel" in _kernel(t, 64, 64, 64)


# shapes the LDS-staged kernel takes for every op pair (every size a multiple
# of 4, so every stored leading dimension is a whole number of 16 bytes)
LDS_SHAPES = [(20, 20, 20), (32, 32, 32), (36, 44, 28), (64, 48, 40), (24, 64, 60), (4, 40, 12), (64, 64, 64),
              (52, 8, 64), (16, 16, 20)]


@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
def test_blocked_lds_matches_register_kernel_bitwise(gpu_lib, dtype):
    """The LDS-staged kernel feeds the same chunks to the same MFMA steps in
    the same order as the register kernel: results equal bit for bit, for
    every op pair, ragged blocks, a C leading dimension of its own and
    matrices at every 16-byte offset (odd batch strides)."""
    al, be = P.scalars(dtype)
    g = inputs.rng(408)
    for ops in P.op_pairs(dtype):
        for (m, n, k) in LDS_SHAPES:
            for pad in (0, 1, 3):
                c = Case(dtype, ops[0], ops[1], m, n, k, 17, al, be, g, ldc=m + 1, pad_stride=pad)
                say(f"blocked lds {np.dtype(dtype).name} {ops} {m}x{n}x{k} pad={pad}")
                with sbg.tuned(blocked=2):
                    assert "gemm_blocked_lds_kernel" in c.describe(), (ops, m, n, k)
                    out = c.run_gpu()
                with sbg.tuned(blocked=1):
                    assert "gemm_blocked_kernel" in c.describe()
                    ref = c.run_gpu()
                assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), (ops, m, n, k, pad)
                check(c, out, label="blocked lds")


@pytest.fixture
def lds_forced():
    with sbg.tuned(blocked=2):
        yield


@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
def test_blocked_lds_special_cases_and_pointer_form(gpu_lib, dtype, lds_forced):
    g = inputs.rng(409)
    m, n, k = 36, 20, 44
    # alpha = 0: A and B (NaN) never read, C = beta C exactly
    c = Case(dtype, "T", "N", m, n, k, 9, 0.0, -0.75, g)
    assert "gemm_blocked_lds_kernel" in c.describe()
    out = c.run_gpu(A=np.full_like(c.A, np.nan), B=np.full_like(c.B, np.nan))
    assert np.array_equal(c.unpack(out), (np.asarray(c.beta, dtype=dtype) * c.unpack(c.C)).astype(dtype))
    # beta = 0: C (NaN) never read
    c2 = Case(dtype, "N", "T", m, n, k, 9, 1.25, 0.0, g)
    out2 = c2.run_gpu(C=np.full_like(c2.C, np.nan))
    assert np.all(np.isfinite(c2.unpack(out2)))
    check(c2, out2, label="blocked lds beta0")
    # padded layout: gaps keep their bytes
    c3 = Case(dtype, "N", "N", m, n, k, 11, 1.5, -0.5, g, lda=m + 8, ldb=k + 4, ldc=m + 3, pad_stride=2)
    assert "gemm_blocked_lds_kernel" in c3.describe()
    out3 = c3.run_gpu()
    check(c3, out3, label="blocked lds padded")
    inside = np.zeros(c3.C.shape, dtype=bool)
    p = np.arange(c3.batch)[:, None, None]
    inside[p * c3.sC + np.arange(m)[None, :, None] + np.arange(n)[None, None, :] * c3.ldc] = True
    assert np.array_equal(out3[~inside].view(np.uint8), c3.C[~inside].view(np.uint8))
    # pointer arrays in reverse order equal the strided form bit for bit
    c4 = Case(dtype, "T", "T", m, n, k, 21, 1.5, -0.5, g)
    ref = c4.run_gpu()
    dA, dB, dC = to_dev(c4.A), to_dev(c4.B), to_dev(c4.C)
    order = np.arange(c4.batch)[::-1].copy()
    esz = dA.element_size()
    pa = torch.tensor([dA.data_ptr() + int(q) * c4.sA * esz for q in order], dtype=torch.int64, device="cuda")
    pb = torch.tensor([dB.data_ptr() + int(q) * c4.sB * esz for q in order], dtype=torch.int64, device="cuda")
    pc = torch.tensor([dC.data_ptr() + int(q) * c4.sC * esz for q in order], dtype=torch.int64, device="cuda")
    say(f"blocked lds pointer form {np.dtype(dtype).name}")
    sbg.gemm_batched("T", "T", m, n, k, 1.5, pa, c4.lda, pb, c4.ldb, -0.5, pc, c4.ldc, c4.batch, dC.dtype)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(dC).view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_shapes_all_op_pairs(gpu_lib, dtype):
    al, be = P.scalars(dtype)
    g = inputs.rng(401)
    worst = 0.0
    for ops in P.op_pairs(dtype):
        for (m, n, k) in SHAPES:
            say(f"blocked {np.dtype(dtype).name} {ops} {m}x{n}x{k}")
            c = Case(dtype, ops[0], ops[1], m, n, k, 13, al, be, g)
            worst = max(worst, check(c, c.run_gpu(), label="blocked"))
    say(f"worst {worst:.2f} u")


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_random_shapes(gpu_lib, dtype):
    g = inputs.rng(402)
    al, be = P.scalars(dtype)
    ops = "NTCR" if np.dtype(dtype).kind == "c" else "NTC"
    for t in range(40):
        m, n, k = (int(v) for v in g.integers(1, 80, size=3))
        if max(m, n, k) <= 16:
            m = 17
        ta, tb = ops[g.integers(len(ops))], ops[g.integers(len(ops))]
        batch = int(g.integers(1, 20))
        say(f"blocked rect {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k} batch={batch}")
        c = Case(dtype, ta, tb, m, n, k, batch, al, be, g)
        check(c, c.run_gpu(), label="blocked rect")


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_padded_layout_gaps_untouched(gpu_lib, dtype):
    g = inputs.rng(403)
    al, be = P.scalars(dtype)
    for (ta, tb, m, n, k, lda, ldb, ldc, pad) in [("N", "N", 21, 18, 35, 23, 40, 22, 3),
                                                  ("T", "C", 32, 17, 20, 33, 19, 40, 5),
                                                  ("C", "T", 5, 40, 50, 51, 41, 9, 1)]:
        say(f"blocked padded {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k}")
        c = Case(dtype, ta, tb, m, n, k, 11, al, be, g, lda=lda, ldb=ldb, ldc=ldc, pad_stride=pad)
        out = c.run_gpu()
        check(c, out, label="blocked padded")
        inside = np.zeros(c.C.shape, dtype=bool)
        p = np.arange(c.batch)[:, None, None]
        inside[p * c.sC + np.arange(m)[None, :, None] + np.arange(n)[None, None, :] * c.ldc] = True
        assert np.array_equal(out[~inside].view(np.uint8), c.C[~inside].view(np.uint8))


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_alpha_beta_special_cases(gpu_lib, dtype):
    g = inputs.rng(404)
    cplx = np.dtype(dtype).kind == "c"
    for (m, n, k) in [(20, 17, 33), (40, 8, 80)]:
        c = Case(dtype, "N", "T", m, n, k, 9, 0.0, complex(0.5, 2.0) if cplx else -0.75, g)
        say(f"blocked alpha=0 {np.dtype(dtype).name} {m}x{n}x{k}")
        out = c.run_gpu(A=np.full_like(c.A, np.nan), B=np.full_like(c.B, np.nan))
        got = c.unpack(out)
        assert np.all(np.isfinite(got))
        if not cplx:
            assert np.array_equal(got, (np.asarray(c.beta, dtype=dtype) * c.unpack(c.C)).astype(dtype))
        else:
            check(c, out, label="blocked alpha0")
        c2 = Case(dtype, "T", "N", m, n, k, 9, complex(1.0, -1.0) if cplx else 2.0, 0.0, g)
        say(f"blocked beta=0 {np.dtype(dtype).name} {m}x{n}x{k}")
        out2 = c2.run_gpu(C=np.full_like(c2.C, np.nan))
        assert np.all(np.isfinite(c2.unpack(out2)))
        check(c2, out2, label="blocked beta0")
        c3 = Case(dtype, "N", "N", m, n, k, 9, 0.0, 0.0, g)
        say(f"blocked alpha=beta=0 {np.dtype(dtype).name} {m}x{n}x{k}")
        out3 = c3.run_gpu(A=np.full_like(c3.A, np.nan), B=np.full_like(c3.B, np.nan),
                          C=np.full_like(c3.C, np.nan))
        assert np.all(c3.unpack(out3) == 0)
        # k = 0 with beta != 1: C = beta C, A and B never read
        c4 = Case(dtype, "N", "N", m, n, 0, 9, 1.5, -0.5, g)
        say(f"blocked k=0 {np.dtype(dtype).name} {m}x{n}")
        check(c4, c4.run_gpu(), label="blocked k0")


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_pointer_form_matches_strided_form(gpu_lib, dtype):
    g = inputs.rng(405)
    al, be = P.scalars(dtype)
    for (m, n, k) in [(17, 30, 45), (64, 20, 3)]:
        c = Case(dtype, "T", "N", m, n, k, 21, al, be, g)
        ref = c.run_gpu()
        dA, dB, dC = to_dev(c.A), to_dev(c.B), to_dev(c.C)
        # matrices in reverse order through the pointer arrays
        order = np.arange(c.batch)[::-1].copy()
        esz = dA.element_size()
        pa = torch.tensor([dA.data_ptr() + int(p) * c.sA * esz for p in order], dtype=torch.int64, device="cuda")
        pb = torch.tensor([dB.data_ptr() + int(p) * c.sB * esz for p in order], dtype=torch.int64, device="cuda")
        pc = torch.tensor([dC.data_ptr() + int(p) * c.sC * esz for p in order], dtype=torch.int64, device="cuda")
        say(f"blocked pointer form {np.dtype(dtype).name} {m}x{n}x{k}")
        sbg.gemm_batched(c.ta, c.tb, m, n, k, c.alpha, pa, c.lda, pb, c.ldb, c.beta, pc, c.ldc, c.batch, dC.dtype)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(dC).view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_blocked_device_scalar_mode(gpu_lib, dtype):
    g = inputs.rng(406)
    al, be = P.scalars(dtype)
    c = Case(dtype, "N", "N", 33, 17, 50, 7, al, be, g)
    dA, dB, dC = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    tdt = TORCH[np.dtype(dtype).type]
    alpha = torch.tensor([al], dtype=tdt, device="cuda")
    beta = torch.tensor([be], dtype=tdt, device="cuda")
    say(f"blocked device scalars {np.dtype(dtype).name}")
    sbg.gemm_strided("N", "N", 33, 17, 50, alpha, dA, c.lda, c.sA, dB, c.ldb, c.sB, beta, dC, c.ldc, c.sC, c.batch)
    torch.cuda.synchronize()
    check(c, from_dev(dC), label="blocked devscalar")
    # beta == 0 read on the device: C (NaN) must not be read
    beta.zero_()
    dC2 = to_dev(np.full_like(c.C, np.nan))
    sbg.gemm_strided("N", "N", 33, 17, 50, alpha, dA, c.lda, c.sA, dB, c.ldb, c.sB, beta, dC2, c.ldc, c.sC, c.batch)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(c.unpack(from_dev(dC2))))


@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("s", [24, 32, 48, 64])
@pytest.mark.parametrize("kernel", [2, 1], ids=["lds", "register"])
def test_blocked_full_size(gpu_lib, dtype, s, kernel):
    """N = 50,000 (s = 24, 32) or 10,000 (s = 48, 64) square matrices, NN and
    TN, through the LDS-staged and the register kernel; the first, last and
    300 sampled matrices against the oracle."""
    g = inputs.rng(407)
    N = 50_000 if s < 48 else 10_000
    c = Case(dtype, "N", "N", s, s, s, N, 1.5, -0.5, g)
    idx = np.unique(np.concatenate([[0, 1, N - 1], g.choice(N, 300, replace=False)]))
    with sbg.tuned(blocked=kernel):
        for ops in ("NN", "TN"):
            c.ta, c.tb = ops[0], ops[1]
            assert ("gemm_blocked_lds_kernel" in c.describe()) == (kernel == 2)
            say(f"blocked full {np.dtype(dtype).name} n={s} {ops} N={N} kernel={kernel}")
            check(c, c.run_gpu(), idx=idx, label="blocked full")
