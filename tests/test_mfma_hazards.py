"""CPU check of the library's gfx950 assembly (see tests/asm_hazards.py):
every MFMA -> accumulator-read path keeps at least 8 wait states."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from asm_hazards import min_wait_states

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1304_7053_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
UNITS = ["gemm_f32.hip", "gemm_f64.hip", "gemm_ex_bf16.hip"]


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_mfma_accumulator_reads_keep_wait_states():
    with tempfile.TemporaryDirectory() as tmp:
        def build(unit):
            out = os.path.join(tmp, unit + ".s")
            cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                   "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip", "-S",
                   "--offload-device-only", os.path.join(CSRC, unit), "-o", out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            with open(out) as f:
                return unit, min_wait_states(f.read())
        with ThreadPoolExecutor(len(UNITS)) as ex:
            results = list(ex.map(build, UNITS))
    for unit, mins in results:
        assert mins, f"no MFMA kernels found in {unit}"
        bad = {k: v for k, v in mins.items() if v < 8}
        assert not bad, f"{unit}: MFMA -> accumulator read with fewer than 8 wait states: {sorted(bad.items())[:5]}"
