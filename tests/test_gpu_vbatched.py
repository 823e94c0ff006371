"""GPU parity of the variable-size form (device-side size binning plus one
persistent launch) against the CPU oracle, its rejection of invalid matrices,
and HIP-graph capture and replay."""
import numpy as np
import pytest
import torch

from paper_1304_7053_amd import inputs, sbg
from gpu_util import Case, VarCase, check_var, from_dev, say, to_dev

pytestmark = pytest.mark.gpu

ALL = [np.float32, np.float64, np.complex64, np.complex128]


def scalars(dtype):
    if np.dtype(dtype).kind == "c":
        return complex(1.0, 0.5), complex(0.25, -1.0)
    return 1.5, -0.5


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
def test_vbatched_mixed_sizes_all_ops(gpu_lib, dtype):
    """Sizes drawn as in the variable-size workload (40% at 8, 30% at 16, the rest
    uniform), padded leading dimensions, every op pair; each matrix against the
    oracle; C entries outside the matrices keep their bits."""
    g = inputs.rng(4, salt=1)
    al, be = scalars(dtype)
    ops = "NTCR" if np.dtype(dtype).kind == "c" else "NTC"
    for ta in ops:
        for tb in ops:
            dims = inputs.varsize_dims(g, 301)
            c = VarCase(dtype, ta, tb, dims, al, be, g)
            say(f"vbatched {np.dtype(dtype).name} {ta}{tb} N={c.batch}")
            out, d = c.run_gpu()
            check_var(c, out, label="vbatched")
            ws = from_dev(d["ws"])
            assert ws[3] == 0
            if np.dtype(dtype).kind == "c":
                # the MFMA path bins the batch: the class counts cover it
                assert ws[0] + ws[1] + ws[2] == c.batch
            inside = np.zeros(c.C.shape, dtype=bool)
            for p in range(c.batch):
                inside[c.offC[p] + np.arange(c.m[p])[:, None] + np.arange(c.n[p])[None, :] * c.ldc[p]] = True
            assert np.array_equal(out[~inside].view(np.uint8), c.C[~inside].view(np.uint8))


@pytest.mark.parametrize("bound", [4, 8], ids=lambda b: f"max{b}")
@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=lambda d: np.dtype(d).name)
def test_vbatched_team_size_from_bounds(gpu_lib, dtype, bound):
    """Real types run with teams of the size class of the declared bounds:
    sizes 0..bound drawn independently (NaN between the matrices), every op
    pair against the oracle; a matrix above the bounds is skipped and counted."""
    g = inputs.rng(4, salt=10 + bound)
    al, be = scalars(dtype)
    N = 517
    for ta in "NT":
        for tb in "NT":
            m, n, k = (g.integers(0, bound + 1, size=N).astype(np.int32) for _ in range(3))
            m[7], n[7], k[7] = bound, bound, bound
            m[8] = bound + 1                   # above max_m: rejected
            c = VarCase(dtype, ta, tb, (m, n, k), al, be, g)
            say(f"vbatched team bound={bound} {np.dtype(dtype).name} {ta}{tb}")
            out, d = c.run_gpu(maxes=(bound, bound, bound))
            ws = from_dev(d["ws"])
            assert ws[3] == 1
            assert np.array_equal(c.got(out, 8).view(np.uint8), c.got(c.C, 8).view(np.uint8))
            check_var(c, out, idx=np.array([p for p in range(N) if p != 8]), label=f"bound {bound}")


@pytest.mark.parametrize("dtype", [np.float32, np.complex128], ids=lambda d: np.dtype(d).name)
def test_vbatched_edge_sizes(gpu_lib, dtype):
    """Zero sizes (m or n = 0: nothing to do; k = 0: C <- beta C), size-1 and
    size-16 extremes, a single matrix, alpha = 0 and beta = 0."""
    g = inputs.rng(4, salt=2)
    al, be = scalars(dtype)
    m = np.array([0, 3, 1, 16, 16, 5, 1, 16, 0, 7], dtype=np.int32)
    n = np.array([4, 0, 1, 16, 1, 5, 16, 16, 0, 2], dtype=np.int32)
    k = np.array([4, 2, 1, 16, 16, 0, 1, 1, 0, 16], dtype=np.int32)
    for (a_, b_) in [(al, be), (0.0, be), (al, 0.0)]:
        c = VarCase(dtype, "N", "T", (m, n, k), a_, b_, g)
        say(f"vbatched edges {np.dtype(dtype).name} alpha={a_} beta={b_}")
        out, _ = c.run_gpu()
        check_var(c, out, label="edges")
    one = VarCase(dtype, "T", "N", (np.array([9]), np.array([13]), np.array([11])), al, be, g)
    out, _ = one.run_gpu()
    check_var(one, out, label="single")


def test_vbatched_rejects_invalid_matrices(gpu_lib):
    """Matrices whose sizes exceed the declared maxima or whose leading
    dimensions are too small are skipped (C untouched) and counted."""
    g = inputs.rng(4, salt=3)
    dims = inputs.varsize_dims(g, 200)
    c = VarCase(np.float64, "N", "N", dims, 1.5, -0.5, g)
    d = c.device()
    bad = np.zeros(c.batch, dtype=bool)
    lda = c.lda.copy()
    lda[5] = int(c.m[5]) - 1              # one short of the minimum max(1, m)
    bad[5] = True
    d["lda"] = torch.from_numpy(lda).to("cuda")
    maxes = (16, 12, 16)                  # n above 12 is out of bounds
    bad |= c.n > 12
    say(f"vbatched invalid: {int(bad.sum())} bad matrices")
    out, d = c.run_gpu(maxes=maxes, d=d)
    ws = from_dev(d["ws"])
    assert ws[3] == int(bad.sum())
    for p in np.nonzero(bad)[0]:
        assert np.array_equal(c.got(out, p).view(np.uint8), c.got(c.C, p).view(np.uint8))
    good = np.nonzero(~bad)[0]
    check_var(c, out, idx=good, label="valid part")


def _vbatched_uniform(cs, dtype, al, be):
    """The strided case `cs` (one size) run through the variable-size entry
    point; returns the resulting C."""
    s, N = cs.m, cs.batch
    esz = np.dtype(dtype).itemsize
    dA, dB, dC = to_dev(cs.A), to_dev(cs.B), to_dev(cs.C)
    p = np.arange(N)
    full = lambda v: torch.full((N,), v, dtype=torch.int32, device="cuda")  # noqa: E731
    ws = torch.zeros(sbg.vbatched_workspace_size(N) // 4 + 1, dtype=torch.int32, device="cuda")
    sbg.gemm_vbatched(cs.ta, cs.tb, full(s), full(s), full(s), s, s, s, al,
                      torch.tensor(dA.data_ptr() + p * cs.sA * esz, device="cuda"), full(cs.lda),
                      torch.tensor(dB.data_ptr() + p * cs.sB * esz, device="cuda"), full(cs.ldb), be,
                      torch.tensor(dC.data_ptr() + p * cs.sC * esz, device="cuda"), full(cs.ldc), N, ws,
                      dC.dtype)
    torch.cuda.synchronize()
    return from_dev(dC)


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.complex64], ids=lambda d: np.dtype(d).name)
def test_vbatched_matches_strided_bitwise(gpu_lib, dtype):
    """With every matrix of one size the variable-size kernels run the same
    per-matrix arithmetic as the strided ones: the MFMA variable-size kernel
    (path 1) equals the strided MFMA tile kernel, and the team variable-size
    kernel (the default for real types) equals the strided team kernel, bit
    for bit, for every op pair."""
    g = inputs.rng(4, salt=4)
    al, be = scalars(dtype)
    real = np.dtype(dtype).kind == "f"
    for ta, tb in (("T", "N"), ("N", "N"), ("N", "T"), ("T", "T")):
        for s in (3, 8, 13, 16):
            cs = Case(dtype, ta, tb, s, s, s, 257, al, be, g)
            say(f"vbatched == strided {np.dtype(dtype).name} {ta}{tb} n={s} (MFMA)")
            with sbg.tuned(path=1):
                ref = cs.run_gpu()
                got = _vbatched_uniform(cs, dtype, al, be)
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
            if real:
                say(f"vbatched == strided {np.dtype(dtype).name} {ta}{tb} n={s} (team)")
                with sbg.tuned(path=3):
                    assert "gemm_team_kernel" in cs.describe()
                    ref = cs.run_gpu()
                got = _vbatched_uniform(cs, dtype, al, be)
                assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=lambda d: np.dtype(d).name)
def test_vbatched_graph_replay_matches_eager(gpu_lib, dtype):
    """The three launches of one call (counter reset, binning, persistent GEMM)
    are captured once and replayed; eager work and synchronisations between the
    replays; every replay must equal the eager result bit for bit.  With device
    scalars a replay picks up new alpha/beta values."""
    g = inputs.rng(4, salt=5)
    dims = inputs.varsize_dims(g, 4000)
    c = VarCase(dtype, "N", "N", dims, 1.5, -0.5, g, pad=False)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    d = c.device()
    C0 = d["C"].clone()
    eager, _ = c.run_gpu(d=d)
    alpha = torch.tensor([1.5], dtype=tdt, device="cuda")
    beta = torch.tensor([-0.5], dtype=tdt, device="cuda")
    d["C"].copy_(C0)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        # warm-up on the capture stream (resolves occupancy queries outside capture)
        sbg.gemm_vbatched("N", "N", d["m"], d["n"], d["k"], 16, 16, 16, alpha, d["pA"], d["lda"], d["pB"],
                          d["ldb"], beta, d["pC"], d["ldc"], c.batch, d["ws"], tdt)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        sbg.gemm_vbatched("N", "N", d["m"], d["n"], d["k"], 16, 16, 16, alpha, d["pA"], d["lda"], d["pB"],
                          d["ldb"], beta, d["pC"], d["ldc"], c.batch, d["ws"], tdt)
    torch.cuda.synchronize()
    for rep in range(3):
        d["C"].copy_(C0)
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        say(f"graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(d["C"]).view(np.uint8), eager.view(np.uint8)), rep
        del junk
    # new scalars, same graph
    alpha.fill_(-2.0)
    beta.fill_(0.0)
    d["C"].copy_(C0)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    c.alpha, c.beta = -2.0, 0.0
    check_var(c, from_dev(d["C"]), label="replay with new scalars")
