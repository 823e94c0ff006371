"""CPU check of the library's gfx950 assembly (see tests/asm_hazards.py):
every MFMA -> accumulator-read path keeps at least 8 wait states, and every
fused DPP FMA (the variable-size team kernel's inline asm) has at least two
wait states after the last write of its DPP source.  The translation units
checked are every csrc/*.hip whose include closure uses MFMA or the fused
DPP FMA."""
import glob
import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from asm_hazards import dpp_fma_hazards, min_wait_states

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1304_7053_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _closure(path, seen=None):
    """Local files a source includes, transitively (quoted includes in csrc)."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path) as f:
        for inc in re.findall(r'^#include "([^"]+)"', f.read(), re.M):
            _closure(os.path.join(CSRC, inc), seen)
    return seen


def _uses(unit, pattern):
    for p in _closure(os.path.join(CSRC, unit)):
        with open(p) as f:
            if re.search(pattern, f.read()):
                return True
    return False


ALL_UNITS = sorted(os.path.basename(p) for p in glob.glob(os.path.join(CSRC, "*.hip")))
UNITS = [u for u in ALL_UNITS if _uses(u, r"__builtin_amdgcn_mfma|_dpp ")]


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_mfma_and_dpp_wait_states():
    with tempfile.TemporaryDirectory() as tmp:
        def build(unit):
            out = os.path.join(tmp, unit + ".s")
            cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                   "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip", "-S",
                   "--offload-device-only", os.path.join(CSRC, unit), "-o", out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            with open(out) as f:
                text = f.read()
            return unit, min_wait_states(text), dpp_fma_hazards(text)
        with ThreadPoolExecutor(min(8, len(UNITS))) as ex:
            results = list(ex.map(build, UNITS))
    assert {"gemm_f32.hip", "gemm_f64.hip", "gemm_c64.hip", "gemm_c128.hip"} <= set(UNITS)
    fused = 0
    for unit, mins, (ndpp, dbad) in results:
        bad = {k: v for k, v in mins.items() if v < 8}
        assert not bad, f"{unit}: MFMA -> accumulator read with fewer than 8 wait states: {sorted(bad.items())[:5]}"
        assert not dbad, f"{unit}: DPP source written fewer than 2 wait states before a fused DPP FMA: {dbad[:3]}"
        fused += ndpp
    assert any(mins for _, mins, _ in results), "no MFMA kernels found"
    assert fused > 0, "no fused DPP FMA found"
