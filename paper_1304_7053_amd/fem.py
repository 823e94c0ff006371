"""Finite-element stiffness batch K_e = B_e^T (D_e B_e), differentiable.

The paper motivates batched small GEMM with finite-element computations
(abstract; Sec. 1).  Per element, the strain-displacement matrix B_e (6 x 12)
and the material matrix D_e (6 x 6) give the element stiffness as two chained
batched GEMMs:
    T = D B          (m = 6,  n = 12, k = 6,  NN)
    K = B^T T        (m = 12, n = 12, k = 6,  TN)
Backward from dK (L = <dK, K>), four batched GEMMs, the B-gradient of the two
uses accumulated by the second call with beta = 1 (no separate add):
    dT = B dK        dB = T dK^T        dB += D^T dT        dD = dT B^T
All products run in the library's kernels; D is treated as a general matrix
(its symmetry is not imposed on the gradient).
"""
import torch

from .autograd import gemm_rm


class ElementStiffness(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, D):
        T = gemm_rm("N", "N", 1.0, D, B)
        K = gemm_rm("T", "N", 1.0, B, T)
        ctx.save_for_backward(B, D, T)
        return K

    @staticmethod
    def backward(ctx, dK):
        B, D, T = ctx.saved_tensors
        dK = dK.contiguous()
        dT = gemm_rm("N", "N", 1.0, B, dK)
        dB = gemm_rm("N", "T", 1.0, T, dK)
        gemm_rm("T", "N", 1.0, D, dT, beta=1.0, C=dB)
        dD = gemm_rm("N", "T", 1.0, dT, B)
        return dB, dD


def element_stiffness(B, D):
    """K_e = B_e^T D_e B_e for a batch: B (N, 6, 12), D (N, 6, 6) on the GPU."""
    return ElementStiffness.apply(B, D)
