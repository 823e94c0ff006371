"""Batched small GEMM on torch tensors, differentiable.

`gemm(A, B, C, transa, transb, alpha, beta)` returns alpha op(A) op(B) + beta C
for batches of row-major torch matrices shaped (N, rows, cols) on the GPU
(Eq. (1) of the paper, Sec. 2, with op in {N, T, C} and the extension R =
conjugate without transpose).  Every product -- forward and backward -- is
one call of the C-ABI strided batched GEMM; torch provides memory, streams
and the autograd graph.

Layout: a contiguous row-major (N, r, c) tensor is, column-major, the batch
of transposes (c x r, leading dimension c, stride r c).  So
    C^T = op(B)^T op(A)^T
is computed with the library's operands swapped, sizes (n, m, k) and the op
letters unchanged (op(X)^T of the row-major X is op applied to the stored
column-major transpose).

Backward (PyTorch's convention for complex tensors: the gradient of
y = a x is conj(a) times the incoming gradient).  With X = op(A), Y = op(B),
G = dL/dC:  dX = conj(alpha) G Y^H,  dY = conj(alpha) X^H G,  dC0 = conj(beta) G,
and dA = op_A(dX), dB = op_B(dY), each realised as ONE batched GEMM whose op
letters are derived from (transa, transb) in `_grad_a` / `_grad_b`.
"""
import torch

from . import sbg

_OPS = ("N", "T", "C", "R")
# op(X)^H as an op on X; conj(op(X)) as an op on X; op(X)^T as an op on X
_H_FLIP = {"N": "C", "T": "R", "C": "N", "R": "T"}
_CONJ_FLIP = {"N": "R", "T": "C", "C": "T", "R": "N"}
_T_FLIP = {"N": "T", "T": "N", "C": "R", "R": "C"}


def _check_batch(X, name):
    if X.dim() != 3:
        raise ValueError(f"{name} must be a batch of matrices shaped (N, rows, cols)")
    if not X.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")


def _op_shape(X, op):
    _, r, c = X.shape
    return (r, c) if op in "NR" else (c, r)


def gemm_rm(opA, opB, alpha, A, B, beta=0.0, C=None):
    """alpha op(A) op(B) + beta C on row-major batches through the C-ABI
    (no autograd).  Returns a new tensor unless C is given (then C is updated
    in place and returned)."""
    _check_batch(A, "A")
    _check_batch(B, "B")
    if opA not in _OPS or opB not in _OPS:
        raise ValueError("op must be one of N, T, C, R")
    dtype = torch.promote_types(A.dtype, B.dtype)
    if dtype not in (torch.float32, torch.float64, torch.complex64, torch.complex128):
        raise TypeError(f"unsupported dtype {dtype}")
    A = A.to(dtype).contiguous()
    B = B.to(dtype).contiguous()
    N = A.shape[0]
    if B.shape[0] != N:
        raise ValueError("batch sizes differ")
    m, k = _op_shape(A, opA)
    k2, n = _op_shape(B, opB)
    if k != k2:
        raise ValueError(f"inner sizes differ: {k} vs {k2}")
    if C is None:
        C = torch.empty((N, m, n), dtype=dtype, device=A.device)
        beta = 0.0
    else:
        if C.shape != (N, m, n) or C.dtype != dtype or not C.is_contiguous():
            raise ValueError("C must be a contiguous (N, m, n) tensor of the product's dtype")
    ra, ca = A.shape[1:]
    rb, cb = B.shape[1:]
    # column-major call: C^T (n x m) = op_B(B_cm) op_A(A_cm), B_cm = B^T (cb x rb), A_cm = A^T (ca x ra)
    sbg.gemm_strided(opB, opA, n, m, k, alpha, B.view(-1), max(cb, 1), rb * cb, A.view(-1), max(ca, 1), ra * ca,
                     beta, C.view(-1), max(n, 1), m * n, N)
    return C


def _grad_a(opA, opB, alpha, G, A, B):
    """dA for C = alpha op_A(A) op_B(B) + beta C0."""
    ca = complex(alpha).conjugate() if isinstance(alpha, complex) else alpha
    if opA == "N":       # dA = conj(a) G op(B)^H
        return gemm_rm("N", _H_FLIP[opB], ca, G, B)
    if opA == "T":       # dA = conj(a) conj(op(B)) G^T
        return gemm_rm(_CONJ_FLIP[opB], "T", ca, B, G)
    if opA == "C":       # dA = a op(B) G^H
        return gemm_rm(opB, "C", alpha, B, G)
    return gemm_rm("R", _T_FLIP[opB], alpha, G, B)   # 'R': dA = a conj(G) op(B)^T


def _grad_b(opA, opB, alpha, G, A, B):
    """dB for C = alpha op_A(A) op_B(B) + beta C0."""
    ca = complex(alpha).conjugate() if isinstance(alpha, complex) else alpha
    if opB == "N":       # dB = conj(a) op(A)^H G
        return gemm_rm(_H_FLIP[opA], "N", ca, A, G)
    if opB == "T":       # dB = conj(a) G^T conj(op(A))
        return gemm_rm("T", _CONJ_FLIP[opA], ca, G, A)
    if opB == "C":       # dB = a G^H op(A)
        return gemm_rm("C", opA, alpha, G, A)
    return gemm_rm(_T_FLIP[opA], "R", alpha, A, G)   # 'R': dB = a op(A)^T conj(G)


def _scale(G, s):
    """s * G through the library (alpha = 0 call: A and B are not read)."""
    out = torch.empty_like(G)
    out.copy_(G)
    N, r, c = G.shape
    sbg.gemm_strided("N", "N", c, r, 0, 0.0, out.view(-1), max(c, 1), 0, out.view(-1), 1, 0, s, out.view(-1),
                     max(c, 1), r * c, N)
    return out


class GemmFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, C0, transa, transb, alpha, beta):
        ctx.transa, ctx.transb, ctx.alpha, ctx.beta = transa, transb, alpha, beta
        ctx.has_c = C0 is not None
        ctx.save_for_backward(A, B)
        if C0 is None or beta == 0:
            return gemm_rm(transa, transb, alpha, A, B)
        out = C0.detach().to(torch.promote_types(A.dtype, B.dtype)).contiguous().clone()
        return gemm_rm(transa, transb, alpha, A, B, beta, out)

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        G = G.contiguous()
        dA = dB = dC = None
        if ctx.needs_input_grad[0]:
            dA = _grad_a(ctx.transa, ctx.transb, ctx.alpha, G, A, B)
        if ctx.needs_input_grad[1]:
            dB = _grad_b(ctx.transa, ctx.transb, ctx.alpha, G, A, B)
        if ctx.has_c and ctx.needs_input_grad[2]:
            cb = complex(ctx.beta).conjugate() if isinstance(ctx.beta, complex) else ctx.beta
            dC = _scale(G, cb)
        return dA, dB, dC, None, None, None, None


def gemm(A, B, C=None, transa="N", transb="N", alpha=1.0, beta=0.0):
    """Differentiable alpha op(A) op(B) + beta C on (N, rows, cols) GPU batches."""
    return GemmFn.apply(A, B, C, transa, transb, alpha, beta)
