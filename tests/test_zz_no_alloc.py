"""The allocation-free variable-size entry point (sbg_gemm_vbatched_ex_noalloc)
against the entry point it varies (sbg_gemm_vbatched_ex with a caller
workspace): same kernels, so the results must agree bit for bit; two calls in
a row, the second on a smaller batch (the shared scratch keeps the first
call's contents), in binary32 and with bf16 inputs; the first call also
against the oracle within 4 max(k, 1) u; a batch above the scratch's limit is
rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1304_7053_amd import inputs, sbg
from gpu_util import VarCase, check_var, from_dev, say

pytestmark = pytest.mark.gpu


def _run(c, d, mode, noalloc):
    """One call on fresh copies of C; returns the flat C buffer."""
    C0 = torch.from_numpy(c.C).to("cuda")
    d["C"].copy_(C0)
    torch.cuda.synchronize()
    pA, pB = d["pA"], d["pB"]
    code = sbg.R_32F
    if mode == "bf16":
        code = sbg.R_16BF
        pA, pB = d["pA16"], d["pB16"]
    args = ("N", "T", d["m"], d["n"], d["k"], 16, 16, 16, 1.5, pA, d["lda"], None, pB, d["ldb"], None, -0.5,
            d["pC"], d["ldc"], c.batch, code, sbg.MODE_PLAIN)
    if noalloc:
        sbg.gemm_vbatched_ex_noalloc(*args)
    else:
        sbg.gemm_vbatched_ex(*args, d["ws"])
    torch.cuda.synchronize()
    return from_dev(d["C"])


def _case(g, batch):
    c = VarCase(np.float32, "N", "T", inputs.varsize_dims(g, batch), 1.5, -0.5, g)
    d = c.device()
    nA = d["A"].to(torch.bfloat16)
    nB = d["B"].to(torch.bfloat16)
    d["A16"], d["B16"] = nA, nB
    d["pA16"] = torch.tensor(nA.data_ptr() + c.offA * 2, device="cuda")
    d["pB16"] = torch.tensor(nB.data_ptr() + c.offB * 2, device="cuda")
    return c, d


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_noalloc_matches_workspace_entry(gpu_lib, mode):
    g = inputs.rng(4, salt=40)
    for i, batch in enumerate((3001, 1203)):
        c, d = _case(g, batch)
        say(f"no-alloc {mode} call {i} batch={batch}")
        ref = _run(c, d, mode, noalloc=False)
        got = _run(c, d, mode, noalloc=True)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (mode, batch)
        if i == 0 and mode == "f32":
            check_var(c, got, label="no-alloc")


def test_noalloc_rejects_batch_above_limit(gpu_lib):
    L = sbg.load()
    small = torch.zeros(16, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(small.data_ptr())
    one = (ctypes.c_float * 1)(1.0)
    a = ctypes.cast(one, ctypes.c_void_p)
    st = L.sbg_gemm_vbatched_ex_noalloc(b"N", b"N", p, p, p, 16, 16, 16, a, p, p, None, p, p, None, a, p, p,
                                        sbg.NOALLOC_MAX_BATCH + 1, sbg.R_32F, sbg.MODE_PLAIN, None)
    assert st == sbg.SBG_WORKSPACE_TOO_SMALL
    torch.cuda.synchronize()
