"""GPU parity of the strided and pointer-array batched GEMM against the CPU
oracle, through the C-ABI (include/sbg.h).  Acceptance test of every entry:
|C - Cref| / (|alpha| (|op A||op B|) + |beta||C_in|) <= 4 max(k,1) u."""
import numpy as np
import pytest
import torch

from paper_1304_7053_amd import inputs, sbg
from gpu_util import Case, TORCH, check, from_dev, say, to_dev, unit

pytestmark = pytest.mark.gpu

REAL = [np.float32, np.float64]
CPLX = [np.complex64, np.complex128]
ALL = REAL + CPLX


def scalars(dtype):
    if np.dtype(dtype).kind == "c":
        return complex(1.0, 0.5), complex(0.25, -1.0)
    return 1.5, -0.5


def op_pairs(dtype):
    ops = "NTCR" if np.dtype(dtype).kind == "c" else "NTC"
    return [a + b for a in ops for b in ops]


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_square_sizes_all_op_pairs(gpu_lib, dtype):
    """Every square size 1..16 and every op pair, ragged batch (several tiles)."""
    al, be = scalars(dtype)
    g = inputs.rng(201)
    worst = 0.0
    for ops in op_pairs(dtype):
        for s in range(1, 17):
            say(f"square {np.dtype(dtype).name} {ops} n={s}")
            c = Case(dtype, ops[0], ops[1], s, s, s, 37, al, be, g)
            worst = max(worst, check(c, c.run_gpu(), label="square"))
    say(f"worst {worst:.2f} u")


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_rectangular_random_shapes(gpu_lib, dtype):
    """Random (m, n, k) in 1..16 with random ops, ragged batch sizes."""
    g = inputs.rng(202)
    al, be = scalars(dtype)
    ops = "NTCR" if np.dtype(dtype).kind == "c" else "NTC"
    for t in range(120):
        m, n, k = (int(v) for v in g.integers(1, 17, size=3))
        ta, tb = ops[g.integers(len(ops))], ops[g.integers(len(ops))]
        batch = int(g.integers(1, 70))
        say(f"rect {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k} batch={batch}")
        c = Case(dtype, ta, tb, m, n, k, batch, al, be, g)
        check(c, c.run_gpu(), label="rect")


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_padded_layout_gaps_untouched(gpu_lib, dtype):
    """Leading dimensions above the minimum and gaps between matrices: the gaps
    hold NaN, must never be read (results finite and correct) and must never
    be written (C's gaps keep their bit pattern)."""
    g = inputs.rng(203)
    al, be = scalars(dtype)
    for (ta, tb, m, n, k, lda, ldb, ldc, pad) in [("N", "N", 5, 7, 3, 9, 4, 6, 3),
                                                  ("T", "C", 16, 16, 16, 17, 19, 16, 5),
                                                  ("C", "T", 3, 12, 9, 11, 13, 8, 1),
                                                  ("N", "T", 8, 8, 8, 8, 8, 9, 64)]:
        say(f"padded {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k}")
        c = Case(dtype, ta, tb, m, n, k, 53, al, be, g, lda=lda, ldb=ldb, ldc=ldc, pad_stride=pad)
        out = c.run_gpu()
        check(c, out, label="padded")
        inside = np.zeros(c.C.shape, dtype=bool)
        p = np.arange(c.batch)[:, None, None]
        inside[p * c.sC + np.arange(m)[None, :, None] + np.arange(n)[None, None, :] * c.ldc] = True
        assert np.array_equal(out[~inside].view(np.uint8), c.C[~inside].view(np.uint8))


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_alpha_zero_and_beta_zero_special_cases(gpu_lib, dtype):
    g = inputs.rng(204)
    cplx = np.dtype(dtype).kind == "c"
    for s in (3, 8, 16):
        # alpha = 0: A, B full of NaN are never read; real types give fl(beta*C) exactly
        c = Case(dtype, "N", "T", s, s, s, 29, 0.0, complex(0.5, 2.0) if cplx else -0.75, g)
        nanA = np.full_like(c.A, np.nan)
        nanB = np.full_like(c.B, np.nan)
        say(f"alpha=0 {np.dtype(dtype).name} n={s}")
        out = c.run_gpu(A=nanA, B=nanB)
        got = c.unpack(out)
        assert np.all(np.isfinite(got))
        if not cplx:
            assert np.array_equal(got, (np.asarray(c.beta, dtype=dtype) * c.unpack(c.C)).astype(dtype))
        else:
            check(c, out, label="alpha0")
        # beta = 0: C full of NaN is never read
        c2 = Case(dtype, "T", "N", s, s, s, 29, complex(1.0, -1.0) if cplx else 2.0, 0.0, g)
        say(f"beta=0 {np.dtype(dtype).name} n={s}")
        out2 = c2.run_gpu(C=np.full_like(c2.C, np.nan))
        assert np.all(np.isfinite(c2.unpack(out2)))
        check(c2, out2, label="beta0")
        # both zero: exact zeros, nothing read
        c3 = Case(dtype, "N", "N", s, s, s, 29, 0.0, 0.0, g)
        say(f"alpha=beta=0 {np.dtype(dtype).name} n={s}")
        out3 = c3.run_gpu(A=nanA[: c3.A.size], B=nanB[: c3.B.size], C=np.full_like(c3.C, np.nan))
        assert np.all(c3.unpack(out3) == 0)


def _pointer_run(c, g):
    """Run a Case through the pointer-array form (matrix pointers of its
    strided buffers, in a shuffled order); returns the flat C buffer."""
    esz = np.dtype(c.dtype).itemsize
    dA, dB, dC = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    perm = g.permutation(c.batch)
    pa = torch.tensor(dA.data_ptr() + perm * c.sA * esz, dtype=torch.int64, device="cuda")
    pb = torch.tensor(dB.data_ptr() + perm * c.sB * esz, dtype=torch.int64, device="cuda")
    pc = torch.tensor(dC.data_ptr() + perm * c.sC * esz, dtype=torch.int64, device="cuda")
    sbg.gemm_batched(c.ta, c.tb, c.m, c.n, c.k, c.alpha, pa, c.lda, pb, c.ldb, c.beta, pc, c.ldc, c.batch, dC.dtype)
    torch.cuda.synchronize()
    return from_dev(dC)


@pytest.mark.parametrize("form", ["strided", "pointer"])
@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_integer_data_bit_exact(gpu_lib, dtype, form):
    """Entries in {-3..3}, dyadic alpha and beta: every partial result is exact
    in the working precision, so GPU and oracle agree bit for bit (-0 == +0),
    for the four real op pairs of the size sweep, in both batch forms."""
    g = inputs.rng(205)
    al, be = scalars(dtype)
    for s in (2, 5, 8, 11, 16):
        for ops in ("NN", "NT", "TN", "TT"):
            say(f"integer {form} {np.dtype(dtype).name} {ops} n={s}")
            c = Case(dtype, ops[0], ops[1], s, s, s, 3001, al, be, g, dist="int")
            got = c.unpack(c.run_gpu() if form == "strided" else _pointer_run(c, g))
            ref, lo, _ = c.oracle()
            assert not np.any(lo)
            assert np.array_equal(got.astype(ref.dtype), ref)


@pytest.mark.parametrize("dtype", REAL, ids=lambda d: np.dtype(d).name)
def test_integer_data_full_size_bit_exact(gpu_lib, dtype):
    """The integer variant of the size sweep at its full size: N = 100,000,
    square n = 2..16, NN/NT/TN/TT, alpha = 1.5, beta = -0.5, entries in
    {-3..3}; every matrix of every call equals the oracle bit for bit (its
    binary64 evaluation of integer data is exact)."""
    N = 100_000
    g = inputs.rng(2, salt=7)
    for s in range(2, 17):
        c = Case(dtype, "N", "N", s, s, s, N, 1.5, -0.5, g, dist="int")
        for ops in ("NN", "NT", "TN", "TT"):
            c.ta, c.tb = ops[0], ops[1]
            say(f"integer full-size {np.dtype(dtype).name} {ops} n={s} N={N}")
            got = c.unpack(c.run_gpu())
            ref, lo, _ = c.oracle(ext=False)
            assert not np.any(lo)
            assert np.array_equal(got.astype(np.float64), ref), (ops, s)


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_pointer_form_matches_strided_form(gpu_lib, dtype):
    """The pointer-array form runs the same arithmetic as the strided form when
    the same kernel serves both (built-in rules, tuned table off): with the
    pointers of a strided batch (shuffled) it must reproduce the strided
    result bit for bit."""
    g = inputs.rng(206)
    al, be = scalars(dtype)
    esz = np.dtype(dtype).itemsize
    for (ta, tb, m, n, k) in [("N", "N", 16, 16, 16), ("T", "N", 7, 5, 9), ("C", "T", 4, 4, 4), ("N", "C", 1, 13, 8)]:
        c = Case(dtype, ta, tb, m, n, k, 203, al, be, g)
        table = sbg.set_tuning("table", 0)
        say(f"pointer form {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k}")
        ref = c.run_gpu()
        dA, dB, dC = to_dev(c.A), to_dev(c.B), to_dev(c.C)
        perm = g.permutation(c.batch)
        pa = torch.tensor(dA.data_ptr() + perm * c.sA * esz, dtype=torch.int64, device="cuda")
        pb = torch.tensor(dB.data_ptr() + perm * c.sB * esz, dtype=torch.int64, device="cuda")
        pc = torch.tensor(dC.data_ptr() + perm * c.sC * esz, dtype=torch.int64, device="cuda")
        sbg.gemm_batched(ta, tb, m, n, k, al, pa, c.lda, pb, c.ldb, be, pc, c.ldc, c.batch, dC.dtype)
        torch.cuda.synchronize()
        sbg.set_tuning("table", table)
        assert np.array_equal(from_dev(dC).view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_shared_operand_and_k_zero(gpu_lib, dtype):
    g = inputs.rng(207)
    al, be = scalars(dtype)
    # strideA = 0: one A for the whole batch
    c = Case(dtype, "N", "N", 9, 6, 12, 77, al, be, g)
    c.sA = 0
    say(f"shared A {np.dtype(dtype).name}")
    check(c, c.run_gpu(), label="sharedA")
    # k = 0: C <- beta C
    c0 = Case(dtype, "N", "N", 5, 5, 0, 40, al, be, g)
    say(f"k=0 {np.dtype(dtype).name}")
    check(c0, c0.run_gpu(), label="k0")


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_device_scalar_mode(gpu_lib, dtype):
    g = inputs.rng(208)
    al, be = scalars(dtype)
    c = Case(dtype, "T", "N", 12, 10, 7, 91, al, be, g)
    tdt = TORCH[np.dtype(dtype).type]
    dA, dB, dC = to_dev(c.A), to_dev(c.B), to_dev(c.C)
    alpha = torch.tensor([al], dtype=tdt, device="cuda")
    beta = torch.tensor([be], dtype=tdt, device="cuda")
    say(f"device scalars {np.dtype(dtype).name}")
    sbg.gemm_strided("T", "N", 12, 10, 7, alpha, dA, c.lda, c.sA, dB, c.ldb, c.sB, beta, dC, c.ldc, c.sC, c.batch)
    torch.cuda.synchronize()
    check(c, from_dev(dC), label="devscalar")
    # beta == 0 read on the device: C (NaN) must not be read
    beta.zero_()
    dC2 = to_dev(np.full_like(c.C, np.nan))
    sbg.gemm_strided("T", "N", 12, 10, 7, alpha, dA, c.lda, c.sA, dB, c.ldb, c.sB, beta, dC2, c.ldc, c.sC, c.batch)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(c.unpack(from_dev(dC2))))


def _sample(batch, g, count=600):
    idx = np.concatenate([np.arange(40), np.arange(batch - 40, batch), g.choice(batch, count, replace=False)])
    return np.unique(idx)


@pytest.mark.parametrize("dtype", REAL, ids=lambda d: np.dtype(d).name)
def test_full_size_square_sweep(gpu_lib, dtype):
    """The size sweep workload: N = 100,000, square n = 2..16, ops NN/NT/TN/TT,
    alpha = 1.5, beta = -0.5; sampled matrices (first and last tiles plus a
    random set) against the oracle."""
    N = 100_000
    g = inputs.rng(2)
    for s in range(2, 17):
        c = Case(dtype, "N", "N", s, s, s, N, 1.5, -0.5, g)
        idx = _sample(N, g)
        for ops in ("NN", "NT", "TN", "TT"):
            c.ta, c.tb = ops[0], ops[1]
            say(f"full-size {np.dtype(dtype).name} {ops} n={s} N={N}")
            check(c, c.run_gpu(), idx=idx, label="fullsize")


@pytest.mark.parametrize("dtype", CPLX, ids=lambda d: np.dtype(d).name)
def test_full_size_complex(gpu_lib, dtype):
    """N = 100,000 complex, n in {4, 8, 12, 16}, all 9 op pairs over {N, T, C},
    alpha = (1, 0.5), beta = (0.25, -1); sampled against the oracle."""
    N = 100_000
    g = inputs.rng(3)
    for s in (4, 8, 12, 16):
        c = Case(dtype, "N", "N", s, s, s, N, complex(1, 0.5), complex(0.25, -1), g)
        idx = _sample(N, g, 300)
        for ta in "NTC":
            for tb in "NTC":
                c.ta, c.tb = ta, tb
                say(f"full-size {np.dtype(dtype).name} {ta}{tb} n={s} N={N}")
                check(c, c.run_gpu(), idx=idx, label="fullsize-c")


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_shared_operand_every_class(gpu_lib, dtype):
    """One A or one B for the whole batch (stride 0): every size class, op
    pair and shared side, batches long enough that every wave runs several
    tiles, through whatever kernel the library picks."""
    g = inputs.rng(208)
    al, be = scalars(dtype)
    ops = "NTC" if np.dtype(dtype).kind == "c" else "NT"
    for (m, n, k) in ((3, 4, 2), (8, 8, 8), (7, 5, 6), (16, 16, 16), (13, 5, 11)):
        for ta in ops:
            for tb in ops:
                for shared in "AB":
                    c = Case(dtype, ta, tb, m, n, k, 5003, al, be, g)
                    if shared == "A":
                        c.sA = 0
                    else:
                        c.sB = 0
                    say(f"shared {shared} {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k}")
                    check(c, c.run_gpu(), label=f"shared{shared}")


@pytest.mark.parametrize("dtype", REAL, ids=lambda d: np.dtype(d).name)
def test_full_size_fixed_operand(gpu_lib, dtype):
    """The fixed-operand case (Sec. 9 outlook): one A (strideA = 0) or one B
    (strideB = 0) for the whole N = 100,000 batch, sampled against the
    oracle, n in {8, 13, 16} (direct and staged sizes)."""
    N = 100_000
    g = inputs.rng(209)
    for s in (8, 13, 16):
        for shared in ("A", "B"):
            c = Case(dtype, "N", "N", s, s, s, N, 1.5, -0.5, g)
            if shared == "A":
                c.sA = 0
            else:
                c.sB = 0
            idx = _sample(N, g, 300)
            say(f"fixed operand {np.dtype(dtype).name} n={s} shared {shared}")
            check(c, c.run_gpu(), idx=idx, label="fixed")
