"""The variable-size form at its full workload size: N = 200,000 matrices
with m, n, k drawn independently (40% at 8, 30% at 16, the rest uniform over
the other values), pointer arrays, alpha = 1.5, beta = -0.5, both input
sets (U[-1, 1] and log-uniform magnitudes) and all five precision modes.

Each mode is checked on a sample of 1,000+ matrices against the oracle:
random matrices, the first and last matrix of each size class, the first and
last of the batch, and, for the binned MFMA path (BF16x3), the first and
last record of each class list read back from the workspace.  The launcher's
own plan (sbg.describe_vbatched) shows that the persistent waves iterate
more than once and, on the binned path, cross from one class list into the
next.  A second test runs 20,000 matrices with one work-group per CU and
XCD runs of one, so every wave iterates many times, and checks every matrix."""
import numpy as np
import pytest
import torch

import oracle
from paper_1304_7053_amd import inputs, sbg
from gpu_util import VarCase, check_var, from_dev, normalised_error, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
MODES = ["f32", "bf16", "f16", "e4m3", "bf16x3"]
REC_BYTES = 48          # one class-list record: A, B, C pointers, lda, ldb, ldc, sizes, scale, pad
HEADER_BYTES = 64


def packed_case(dims, dist, g):
    """A VarCase with the matrices packed back to back (leading dimension =
    rows), built without a per-matrix loop."""
    c = VarCase.__new__(VarCase)
    c.dtype, c.ta, c.tb = np.float32, "N", "N"
    c.m, c.n, c.k = (np.asarray(d, dtype=np.int32) for d in dims)
    c.batch = len(c.m)
    c.alpha, c.beta = 1.5, -0.5
    c.store = np.float32
    c.lda = np.maximum(c.m, 1).astype(np.int32)
    c.ldb = np.maximum(c.k, 1).astype(np.int32)
    c.ldc = np.maximum(c.m, 1).astype(np.int32)

    def fill(ld, cols):
        sizes = np.maximum(np.where(cols > 0, ld.astype(np.int64) * cols, 0), 1)
        off = np.zeros(c.batch, dtype=np.int64)
        off[1:] = np.cumsum(sizes)[:-1]
        return inputs.DISTS[dist](g, (int(sizes.sum()),), np.float32), off

    c.A, c.offA = fill(c.lda, c.k)
    c.B, c.offB = fill(c.ldb, c.n)
    c.C, c.offC = fill(c.ldc, c.n)
    return c


def size_class(m, n, k):
    mx = np.maximum(np.maximum(m, n), k)
    return np.where(mx <= 4, 4, np.where(mx <= 8, 8, 16))


def base_sample(c, count, g):
    idx = set(g.choice(c.batch, size=count, replace=False).tolist())
    cls = size_class(c.m, c.n, c.k)
    for d in (4, 8, 16):
        mem = np.nonzero(cls == d)[0]
        if len(mem):
            idx.update((int(mem[0]), int(mem[-1])))
    idx.update((0, c.batch - 1))
    return idx


def list_ends(ws, batch, pC_host, offC):
    """Matrix indices of the first and last record of each class list, found
    by their C pointers."""
    raw = ws.view(np.uint8)
    counts = ws[:3].astype(np.int64)
    ptr_to_idx = {int(v): i for i, v in enumerate(pC_host)}
    out = set()
    for c in range(3):
        if counts[c] == 0:
            continue
        for r in (0, counts[c] - 1):
            o = HEADER_BYTES + (c * batch + int(r)) * REC_BYTES
            cptr = int(raw[o + 16:o + 24].view(np.uint64)[0])
            out.add(ptr_to_idx[cptr])
    return out, counts


def run_mode(c, d, mode, ws):
    """One variable-size call in `mode`; returns (C on the host, oracle kwargs)."""
    N = c.batch
    kw = {}
    if mode in ("bf16", "f16"):
        tdt = torch.bfloat16 if mode == "bf16" else torch.float16
        code = sbg.R_16BF if mode == "bf16" else sbg.R_16F
        nA, nB = d["A"].to(tdt), d["B"].to(tdt)
        pA = torch.tensor(nA.data_ptr() + c.offA * 2, device="cuda")
        pB = torch.tensor(nB.data_ptr() + c.offB * 2, device="cuda")
        sA = sB = None
        cmode = sbg.MODE_PLAIN
        kw = dict(types=(mode, mode, "f32"), A=nA.view(torch.int16).cpu().numpy().view(np.uint16),
                  B=nB.view(torch.int16).cpu().numpy().view(np.uint16))
        keep = (nA, nB)
    elif mode == "e4m3":
        code, cmode = sbg.R_8F_E4M3, sbg.MODE_PLAIN
        qA = torch.zeros(c.A.size, dtype=torch.uint8, device="cuda")
        qB = torch.zeros(c.B.size, dtype=torch.uint8, device="cuda")
        sA = torch.empty(N, dtype=torch.float32, device="cuda")
        sB = torch.empty(N, dtype=torch.float32, device="cuda")
        pA = torch.tensor(qA.data_ptr() + c.offA, device="cuda")
        pB = torch.tensor(qB.data_ptr() + c.offB, device="cuda")
        sbg.quantize_e4m3_vbatched(d["m"], d["k"], 16, 16, d["pA"], d["lda"], pA, d["lda"], sA, N)
        sbg.quantize_e4m3_vbatched(d["k"], d["n"], 16, 16, d["pB"], d["ldb"], pB, d["ldb"], sB, N)
        torch.cuda.synchronize()
        kw = dict(types=("e4m3", "e4m3", "f32"), A=from_dev(qA), B=from_dev(qB),
                  scaleA=from_dev(sA).astype(np.float64), scaleB=from_dev(sB).astype(np.float64))
        keep = (qA, qB, sA, sB)
    else:
        code = sbg.R_32F
        cmode = sbg.MODE_BF16X3 if mode == "bf16x3" else sbg.MODE_PLAIN
        pA, pB, sA, sB = d["pA"], d["pB"], None, None
        keep = ()
    d["C"].copy_(torch.from_numpy(c.C).to("cuda"))
    sbg.gemm_vbatched_ex("N", "N", d["m"], d["n"], d["k"], 16, 16, 16, 1.5, pA, d["lda"], sA, pB, d["ldb"], sB,
                         -0.5, d["pC"], d["ldc"], N, code, cmode, ws)
    torch.cuda.synchronize()
    del keep
    return from_dev(d["C"]), kw, code, cmode


def check_split3(c, out, idx):
    idx = np.asarray(sorted(idx))
    hi, lo, bnd, offO, mm, nn = oracle.gemm_split3_general(
        "N", "N", c.m[idx], c.n[idx], c.k[idx], 1.5, c.A, c.offA[idx], c.lda[idx], c.B, c.offB[idx], c.ldb[idx],
        -0.5, c.C, c.offC[idx], c.ldc[idx], len(idx))
    for q, p in enumerate(idx):
        m, n = int(mm[q]), int(nn[q])
        if m == 0 or n == 0:
            continue
        o = int(offO[q])
        e = normalised_error(c.got(out, p), hi[o:o + m * n].reshape(n, m).T, lo[o:o + m * n].reshape(n, m).T,
                             bnd[o:o + m * n].reshape(n, m).T)
        assert np.max(e) <= 12 * max(int(c.k[p]), 1) * U32, (p, m, n, int(c.k[p]), np.max(e) / U32)


def check_mode(c, out, idx, mode, kw):
    if mode == "bf16x3":
        check_split3(c, out, idx)
    else:
        check_var(c, out, idx=np.asarray(sorted(idx)), label=f"N={c.batch} {mode}", **kw)


def assert_waves_iterate(N, code, cmode, ws_host):
    plan = sbg.describe_vbatched("s", "N", "N", 16, 16, 16, N, code, cmode)
    assert plan is not None
    waves = 4 * plan["grid"]
    if "u16" not in plan:
        # team path: one wave step per 64 / 16 matrices, in batch order
        assert "gemm_vbteam_kernel" in plan["kernel"]
        assert plan["units"] == (N + 3) // 4
        assert plan["units"] > waves, plan
        return
    # binned MFMA path: units per class list as the kernel counts them
    c4, c8, c16 = (int(x) for x in ws_host[:3])
    g16 = -(-c16 // plan["u16"])
    g8 = -(-((c8 + 1) // 2) // plan["u8"])
    g4 = -(-((c4 + 3) // 4) // plan["u4"])
    total = g16 + g8 + g4
    assert total > waves, (plan, c4, c8, c16)
    # wave w runs units w, w + waves, ...: some wave has a unit in the 16 list
    # and its next one in a later list iff max(g16, waves) < total
    assert g16 > 0 and max(g16, waves) < total, (plan, g16, g8, g4)


@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_vbatched_full_size_all_modes(gpu_lib, dist):
    N = 200_000
    g = inputs.rng(4)                     # the workload's own size draw
    dims = inputs.varsize_dims(g, N)
    c = packed_case(dims, dist, inputs.rng(4, salt=40 if dist == "uniform" else 41))
    d = c.device()
    ws = d["ws"]
    sample = base_sample(c, 1000, inputs.rng(4, salt=42))
    pC_host = from_dev(d["pC"])
    results = {}
    for mode in ["bf16x3"] + [m for m in MODES if m != "bf16x3"]:
        say(f"vbatched full N={N} {dist} {mode}")
        out, kw, code, cmode = run_mode(c, d, mode, ws)
        ws_host = from_dev(ws)
        assert ws_host[3] == 0
        if mode == "bf16x3":
            ends, counts = list_ends(ws_host, N, pC_host, c.offC)
            assert counts.sum() == N
            sample |= ends
        assert_waves_iterate(N, code, cmode, ws_host)
        results[mode] = (out, kw)
    assert len(sample) >= 1000
    for mode, (out, kw) in results.items():
        check_mode(c, out, sample, mode, kw)


@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_vbatched_many_iterations_every_matrix(gpu_lib, dist):
    """20,000 matrices, one work-group per CU, XCD runs of one: waves iterate
    many times (and cross class lists on the binned path); every matrix
    against the oracle, binary32, bf16 and BF16x3."""
    N = 20_000
    g = inputs.rng(4, salt=50)
    dims = inputs.varsize_dims(g, N)
    c = packed_case(dims, dist, inputs.rng(4, salt=51 if dist == "uniform" else 52))
    d = c.device()
    ws = d["ws"]
    everything = set(range(N))
    with sbg.tuned(wg_per_cu=1, xcd_chunk=1):
        for mode in ("f32", "bf16", "bf16x3"):
            say(f"vbatched N={N} one work-group per CU {dist} {mode}")
            out, kw, code, cmode = run_mode(c, d, mode, ws)
            ws_host = from_dev(ws)
            assert ws_host[3] == 0
            assert_waves_iterate(N, code, cmode, ws_host)
            check_mode(c, out, everything, mode, kw)
