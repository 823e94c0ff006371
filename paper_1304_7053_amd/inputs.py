"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws numbers; it holds none of the GEMM arithmetic, so both
the GPU path's tests and the CPU oracle's tests can use it.  All draws use
numpy's PCG64 with seed 13047053 + config id (+ an optional salt), in the
order A, B, C; complex values draw (re, im) pairs.

Workloads (the paper times N = 100,000 independent square pairs with minimal
leading dimensions, Sec. 8; the variable-size, precision and FEM batches
extend it):
  cfg 1: N = 1000, 8x8x8, U[-1,1], fp32
  cfg 2: N = 100,000, square n = 2..16, U[-1,1] fp32/fp64, plus integers in {-3..3}
  cfg 3: N = 100,000, n in {4,8,12,16}, complex U[-1,1] parts
  cfg 4: N = 200,000 variable (m, n, k): 40% mass at 8, 30% at 16, the rest
         uniform over the other 14 values; U[-1,1] and +-10^U(-3,3)
  cfg 5: N = 1,000,000 FEM elements, B_e 6x12 U[-1,1], D_e = L L^T + 6 I with
         L 6x6 U[-0.5,0.5], upstream gradient dK_e U[-1,1]
"""
import numpy as np

SEED_BASE = 13047053


def rng(cfg_id: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(cfg_id) + 1000003 * int(salt)))


def _is_complex(dtype) -> bool:
    return np.dtype(dtype).kind == "c"


def _real_of(dtype):
    return np.float32 if np.dtype(dtype) in (np.float32, np.complex64) else np.float64


def uniform(g, shape, dtype, lo=-1.0, hi=1.0):
    rt = _real_of(dtype)
    if _is_complex(dtype):
        v = g.uniform(lo, hi, size=tuple(shape) + (2,)).astype(rt)
        return (v[..., 0] + 1j * v[..., 1]).astype(dtype)
    return g.uniform(lo, hi, size=shape).astype(dtype)


def integers(g, shape, dtype, lo=-3, hi=3):
    if _is_complex(dtype):
        v = g.integers(lo, hi + 1, size=tuple(shape) + (2,)).astype(np.float64)
        return (v[..., 0] + 1j * v[..., 1]).astype(dtype)
    return g.integers(lo, hi + 1, size=shape).astype(dtype)


def log_uniform(g, shape, dtype, lo_exp=-3.0, hi_exp=3.0):
    """Entries +-10^U(lo_exp, hi_exp) with a random sign."""
    def one(sh):
        mag = 10.0 ** g.uniform(lo_exp, hi_exp, size=sh)
        sign = np.where(g.integers(0, 2, size=sh) == 0, -1.0, 1.0)
        return mag * sign
    if _is_complex(dtype):
        v = one(tuple(shape) + (2,))
        return (v[..., 0] + 1j * v[..., 1]).astype(dtype)
    return one(shape).astype(dtype)


DISTS = {"uniform": uniform, "int": integers, "logu": log_uniform}


def span(batch, rows, cols, ld, stride):
    """Number of elements a strided batch occupies (0 when empty)."""
    if batch == 0 or rows == 0 or cols == 0:
        return 0
    return (batch - 1) * stride + (cols - 1) * ld + rows


def strided_batch(g, batch, rows, cols, ld, stride, dtype, dist="uniform", fill=np.nan):
    """Flat column-major storage for `batch` rows x cols matrices, matrix p at
    element offset p*stride, leading dimension ld.  Entries outside the
    matrices (padding between columns or matrices) hold `fill`."""
    n_el = span(batch, rows, cols, ld, stride)
    out = np.full(max(n_el, 1), fill, dtype=dtype)
    if n_el == 0:
        return out[:0]
    vals = DISTS[dist](g, (batch, cols, rows), dtype)
    p = np.arange(batch, dtype=np.int64)[:, None, None]
    c = np.arange(cols, dtype=np.int64)[None, :, None]
    r = np.arange(rows, dtype=np.int64)[None, None, :]
    out[p * stride + c * ld + r] = vals
    return out


def varsize_dims(g, batch, p8=0.40, p16=0.30):
    """m, n, k drawn independently from {1..16}: mass p8 at 8, p16 at 16, the
    rest uniform over the other 14 values."""
    vals = np.arange(1, 17)
    probs = np.full(16, (1.0 - p8 - p16) / 14.0)
    probs[7] = p8
    probs[15] = p16
    dims = g.choice(vals, size=(3, batch), p=probs).astype(np.int32)
    return dims[0], dims[1], dims[2]


def fem_element_batch(g, batch):
    """B_e (6 x 12, U[-1,1]), D_e = L L^T + 6 I (6 x 6, L U[-0.5,0.5]) and the
    upstream gradient dK_e (12 x 12, U[-1,1]), fp32, shaped (batch, rows, cols)."""
    B = g.uniform(-1, 1, size=(batch, 6, 12)).astype(np.float32)
    L = g.uniform(-0.5, 0.5, size=(batch, 6, 6))
    D = (L @ np.swapaxes(L, 1, 2) + 6.0 * np.eye(6)).astype(np.float32)
    dK = g.uniform(-1, 1, size=(batch, 12, 12)).astype(np.float32)
    return B, D, dK
