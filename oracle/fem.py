"""Oracle for the finite-element chain K = B^T (D B) and its gradients --
TEST INFRASTRUCTURE ONLY.

Forward and backward are written as compositions of the oracle GEMM
(oracle.gemm, long-double accumulation): T = D B, K = B^T T; for the loss
L = <dK, K> the gradients follow from the product rule,
    dT = B dK,  dB = T dK^T + D^T dT,  dD = dT B^T.
tests/test_oracle_fem.py pins these formulas with central finite
differences (exact up to rounding because L is quadratic in B and linear in D).
"""
import numpy as np

from .oracle import gemm


def _g(ta, tb, A, B):
    hi, lo = gemm(ta, tb, 1.0, A, B, 0.0, None, ext=True)
    return hi + lo


def forward(B, D):
    """K (batch, 12, 12) and T (batch, 6, 12) in binary64 from B, D of any
    real dtype (promoted exactly)."""
    B = np.asarray(B, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    T = _g("N", "N", D, B)
    K = _g("T", "N", B, T)
    return K, T


def backward(B, D, dK):
    B = np.asarray(B, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    dK = np.asarray(dK, dtype=np.float64)
    T = _g("N", "N", D, B)
    dT = _g("N", "N", B, dK)
    dB = _g("N", "T", T, dK) + _g("T", "N", D, dT)
    dD = _g("N", "T", dT, B)
    return dB, dD, dT, T
