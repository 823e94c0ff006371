"""GPU parity of the team kernel (sizes <= 8) over every shape it serves:
all (m, n, k) in {1..8}^3 for binary32 with a random op pair per shape (team
sizes max(n, k) and, for a transposed A, m; vector and element-wise column
modes; vectors with and without the overlapping last one), a random subset of
shapes for the other three types, both batch forms, and ragged batches that
end inside a wave.  Acceptance: 4 max(k, 1) u against the oracle."""
import numpy as np
import pytest

from paper_1304_7053_amd import inputs, sbg
from gpu_util import Case, check, say

pytestmark = pytest.mark.gpu


def _scalars(dtype):
    if np.dtype(dtype).kind == "c":
        return complex(0.75, -0.5), complex(-0.25, 1.0)
    return 1.5, -0.5


def _name(dtype, ta, tb, m, n, k, batch):
    t = {np.float32: "s", np.float64: "d", np.complex64: "c", np.complex128: "z"}[np.dtype(dtype).type]
    ra, ca = (m, k) if ta in "NR" else (k, m)
    rb, cb = (k, n) if tb in "NR" else (n, k)
    return sbg.describe_strided(t, ta, tb, m, n, k, max(ra, 1), ra * ca, max(rb, 1), rb * cb, m, m * n, batch)


def test_team_every_shape_f32(gpu_lib):
    g = inputs.rng(211)
    al, be = _scalars(np.float32)
    with sbg.tuned(path=2):
        for m in range(1, 9):
            for n in range(1, 9):
                for k in range(1, 9):
                    ta, tb = "NTC"[g.integers(3)], "NTC"[g.integers(3)]
                    batch = int(g.integers(1, 200))
                    assert "gemm_team_kernel" in _name(np.float32, ta, tb, m, n, k, batch)
                    c = Case(np.float32, ta, tb, m, n, k, batch, al, be, g)
                    check(c, c.run_gpu(), label="team")
        say("f32: 512 shapes")


@pytest.mark.parametrize("dtype", [np.float64, np.complex64, np.complex128], ids=lambda d: np.dtype(d).name)
def test_team_shapes_other_types(gpu_lib, dtype):
    g = inputs.rng(212)
    al, be = _scalars(dtype)
    ops = "NTCR" if np.dtype(dtype).kind == "c" else "NTC"
    with sbg.tuned(path=2):
        for _ in range(160):
            m, n, k = (int(v) for v in g.integers(1, 9, size=3))
            ta, tb = ops[g.integers(len(ops))], ops[g.integers(len(ops))]
            batch = int(g.integers(1, 300))
            say(f"team {np.dtype(dtype).name} {ta}{tb} {m}x{n}x{k} batch={batch}")
            c = Case(dtype, ta, tb, m, n, k, batch, al, be, g)
            check(c, c.run_gpu(), label="team")


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.complex64, np.complex128], ids=lambda d: np.dtype(d).name)
def test_team_padded_and_special_scalars(gpu_lib, dtype):
    """Leading dimensions above the minimum (NaN in the gaps, never read or
    written), alpha = 0 (A, B never read), beta = 0 (C never read), k = 0."""
    g = inputs.rng(213)
    al, be = _scalars(dtype)
    with sbg.tuned(path=2):
        for (ta, tb, m, n, k) in [("N", "N", 5, 3, 7), ("T", "T", 8, 2, 6), ("C", "N", 3, 8, 5), ("N", "C", 7, 7, 1)]:
            c = Case(dtype, ta, tb, m, n, k, 97, al, be, g, lda=(m if ta == "N" else k) + 3,
                     ldb=(k if tb == "N" else n) + 1, ldc=m + 2, pad_stride=5)
            out = c.run_gpu()
            check(c, out, label="team padded")
            inside = np.zeros(c.C.shape, dtype=bool)
            p = np.arange(c.batch)[:, None, None]
            inside[p * c.sC + np.arange(m)[None, :, None] + np.arange(n)[None, None, :] * c.ldc] = True
            assert np.array_equal(out[~inside].view(np.uint8), c.C[~inside].view(np.uint8))
            c0 = Case(dtype, ta, tb, m, n, k, 61, 0.0, be, g)
            got = c0.unpack(c0.run_gpu(A=np.full_like(c0.A, np.nan), B=np.full_like(c0.B, np.nan)))
            assert np.all(np.isfinite(got))
            c1 = Case(dtype, ta, tb, m, n, k, 61, al, 0.0, g)
            out1 = c1.run_gpu(C=np.full_like(c1.C, np.nan))
            check(c1, out1, label="team beta0")
            ck = Case(dtype, ta, tb, m, n, 0, 61, al, be, g)
            check(ck, ck.run_gpu(), label="team k0")
