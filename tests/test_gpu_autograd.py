"""GPU checks of the differentiable batched GEMM and of the FEM element chain.

* torch.autograd.gradcheck (binary64 / complex128, finite differences) on the
  library-backed backward for every op pair: pins the flipped-op gradient
  formulas, Wirtinger convention included;
* binary32 gradients, one backward GEMM each, against the oracle evaluating
  the gradient definition on explicitly transposed / conjugated operands,
  within 4 max(k,1) u;
* the FEM batch K = B^T (D B) at N = 1,000,000: forward and both gradients on
  64 sampled elements against the binary64 oracle and against central finite
  differences of the oracle's forward (h = 1e-3)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import fem as ofem
from paper_1304_7053_amd import inputs
from paper_1304_7053_amd.autograd import gemm
from paper_1304_7053_amd.fem import element_stiffness
from gpu_util import normalised_error, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def np_op(X, op):
    if op == "N":
        return X
    if op == "T":
        return np.swapaxes(X, 1, 2)
    if op == "C":
        return np.conj(np.swapaxes(X, 1, 2))
    return np.conj(X)


def stored(op, rows, cols):
    return (rows, cols) if op in "NR" else (cols, rows)


@pytest.mark.parametrize("dtype", [torch.float64, torch.complex128], ids=["f64", "c128"])
def test_gradcheck_all_op_pairs(gpu_lib, dtype):
    g = torch.Generator(device="cpu").manual_seed(13047053 + 5)
    cplx = dtype.is_complex
    ops = "NTCR" if cplx else "NTC"
    alpha = complex(0.7, -1.2) if cplx else 0.7
    beta = complex(-0.4, 0.3) if cplx else -0.4
    m, n, k, N = 3, 4, 5, 2
    for ta in ops:
        for tb in ops:
            A = torch.randn((N,) + stored(ta, m, k), generator=g, dtype=dtype).cuda().requires_grad_()
            B = torch.randn((N,) + stored(tb, k, n), generator=g, dtype=dtype).cuda().requires_grad_()
            C = torch.randn((N, m, n), generator=g, dtype=dtype).cuda().requires_grad_()
            say(f"gradcheck {dtype} {ta}{tb}")
            f = lambda a, b, c: gemm(a, b, c, ta, tb, alpha, beta)  # noqa: E731
            assert torch.autograd.gradcheck(f, (A, B, C), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64], ids=["f32", "c64"])
def test_fp32_backward_gemms_against_oracle(gpu_lib, dtype):
    gen = inputs.rng(5, salt=7)
    npdt = np.float32 if dtype == torch.float32 else np.complex64
    cplx = dtype.is_complex
    ops = "NTCR" if cplx else "NTC"
    alpha = complex(1.0, 0.5) if cplx else 1.5
    m, n, k, N = 7, 5, 9, 64
    for ta in ops:
        for tb in ops:
            A = inputs.uniform(gen, (N,) + stored(ta, m, k), npdt)
            B = inputs.uniform(gen, (N,) + stored(tb, k, n), npdt)
            G = inputs.uniform(gen, (N, m, n), npdt)
            tA = torch.from_numpy(A).cuda().requires_grad_()
            tB = torch.from_numpy(B).cuda().requires_grad_()
            say(f"fp32 backward {dtype} {ta}{tb}")
            out = gemm(tA, tB, None, ta, tb, alpha, 0.0)
            out.backward(torch.from_numpy(G).cuda())
            torch.cuda.synchronize()
            X, Y = np_op(A, ta), np_op(B, tb)
            ca = np.conj(alpha)
            # dX = conj(a) G Y^H, dY = conj(a) X^H G, mapped back through the ops
            YH = np.ascontiguousarray(np.conj(np.swapaxes(Y, 1, 2)))
            XH = np.ascontiguousarray(np.conj(np.swapaxes(X, 1, 2)))
            for (name, grad, lhs, rhs, inv, kk) in (("dA", tA.grad, G, YH, ta, n), ("dB", tB.grad, XH, G, tb, m)):
                hi, lo = oracle.gemm("N", "N", ca, lhs, rhs, 0.0, None, ext=True)
                absl = np.abs(lhs.astype(np.complex128 if cplx else np.float64))
                absr = np.abs(rhs.astype(np.complex128 if cplx else np.float64))
                bnd = abs(ca) * (absl @ absr)
                ref, rlo, b = (np_op(x, inv) for x in (hi, lo, bnd))
                # op C / R conjugate the gradient; the bound is real
                b = np.abs(b)
                e = normalised_error(grad.cpu().numpy(), ref, rlo, b)
                assert np.max(e) <= 4 * kk * U32, (name, ta, tb, np.max(e) / U32)


def test_fem_element_batch_full_size(gpu_lib):
    """N = 1,000,000 FEM elements; 64 sampled elements checked."""
    N = 1_000_000
    g = inputs.rng(5)
    say("generating FEM batch")
    B, D, dK = inputs.fem_element_batch(g, N)
    tB = torch.from_numpy(B).cuda().requires_grad_()
    tD = torch.from_numpy(D).cuda().requires_grad_()
    say("forward + backward")
    K = element_stiffness(tB, tD)
    K.backward(torch.from_numpy(dK).cuda())
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([[0, N - 1], g.choice(N, 62, replace=False)]))
    Kg = K.detach()[idx].cpu().numpy()
    dBg = tB.grad[idx].cpu().numpy().astype(np.float64)
    dDg = tD.grad[idx].cpu().numpy().astype(np.float64)
    Bs, Ds, dKs = B[idx].astype(np.float64), D[idx].astype(np.float64), dK[idx].astype(np.float64)
    Kref, Tref = ofem.forward(Bs, Ds)
    dBref, dDref, dTref, _ = ofem.backward(Bs, Ds, dKs)
    aB, aD, adK = np.abs(Bs), np.abs(Ds), np.abs(dKs)
    # chained error bounds (each GEMM within 4 k u of its own |.| products)
    aT = aD @ aB
    bK = 4 * 6 * U32 * (np.swapaxes(aB, 1, 2) @ aT) * 2
    assert np.all(np.abs(Kg - Kref) <= bK)
    adT = aB @ adK
    bdB = 4 * 12 * U32 * (aT @ np.swapaxes(adK, 1, 2)) * 2 + 4 * 12 * U32 * (np.swapaxes(aD, 1, 2) @ adT) * 2
    bdD = 4 * 12 * U32 * (adT @ np.swapaxes(aB, 1, 2)) * 2
    assert np.all(np.abs(dBg - dBref) <= bdB)
    assert np.all(np.abs(dDg - dDref) <= bdD)

    # central finite differences of the oracle forward on the sampled elements
    def loss(Bx, Dx):
        Kx, _ = ofem.forward(Bx, Dx)
        return np.sum(dKs * Kx, axis=(1, 2))

    h = 1e-3
    say("finite differences")
    for i in range(6):
        for j in range(12):
            e = np.zeros_like(Bs)
            e[:, i, j] = h
            fd = (loss(Bs + e, Ds) - loss(Bs - e, Ds)) / (2 * h)
            assert np.all(np.abs(fd - dBg[:, i, j]) <= bdB[:, i, j] + 1e-9 * np.abs(fd))
    for i in range(6):
        for j in range(6):
            e = np.zeros_like(Ds)
            e[:, i, j] = h
            fd = (loss(Bs, Ds + e) - loss(Bs, Ds - e)) / (2 * h)
            assert np.all(np.abs(fd - dDg[:, i, j]) <= bdD[:, i, j] + 1e-9 * np.abs(fd))
