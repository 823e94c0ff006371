"""Pins of the FEM oracle (no GPU): its forward against numpy's matmul, and
its gradients of L = <dK, K> against central finite differences, which are
exact up to rounding for this loss (quadratic in B, linear in D)."""
import numpy as np

from oracle import fem
from paper_1304_7053_amd import inputs


def test_forward_matches_numpy():
    g = inputs.rng(5)
    B, D, _ = inputs.fem_element_batch(g, 20)
    K, T = fem.forward(B, D)
    Bd, Dd = B.astype(np.float64), D.astype(np.float64)
    ref = np.swapaxes(Bd, 1, 2) @ (Dd @ Bd)
    assert np.allclose(K, ref, rtol=1e-13, atol=1e-13)
    assert np.allclose(T, Dd @ Bd, rtol=1e-13, atol=1e-13)
    # K is symmetric because D is
    assert np.allclose(K, np.swapaxes(K, 1, 2), rtol=1e-12, atol=1e-12)


def test_gradients_match_central_differences():
    g = inputs.rng(5, salt=1)
    B, D, dK = inputs.fem_element_batch(g, 64)
    B, D, dK = (x.astype(np.float64) for x in (B, D, dK))
    dB, dD, _, _ = fem.backward(B, D, dK)

    def loss(Bx, Dx):
        K, _ = fem.forward(Bx, Dx)
        return np.sum(dK * K, axis=(1, 2))      # one loss per element

    h = 1e-3
    fdB = np.zeros_like(B)
    for i in range(6):
        for j in range(12):
            e = np.zeros_like(B)
            e[:, i, j] = h
            fdB[:, i, j] = (loss(B + e, D) - loss(B - e, D)) / (2 * h)
    fdD = np.zeros_like(D)
    for i in range(6):
        for j in range(6):
            e = np.zeros_like(D)
            e[:, i, j] = h
            fdD[:, i, j] = (loss(B, D + e) - loss(B, D - e)) / (2 * h)
    scaleB = np.max(np.abs(dB))
    scaleD = np.max(np.abs(dD))
    assert np.max(np.abs(fdB - dB)) <= 1e-10 * scaleB
    assert np.max(np.abs(fdD - dD)) <= 1e-10 * scaleD
