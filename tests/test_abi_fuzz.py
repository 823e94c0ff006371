"""The C-ABI host layer (argument validation, quick returns, scalar classes,
kernel planning in paper_1304_7053_amd/csrc/api.cpp, and the tuned-table
reader) under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/abi_fuzz.cpp links it against stubs in place of the kernel launchers
and the HIP runtime and calls every entry point 60,000 times with seeded
boundary arguments (negative and huge sizes, strides and batch counts up to
INT64_MAX, null and misaligned pointers, invalid op characters, NaN scalars),
half of the GEMM calls with consistent shapes so that accepted calls reach the
launch path.  No GPU is involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CSRC = os.path.join(ROOT, "paper_1304_7053_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_c_abi_host_layer_under_sanitizers(tmp_path):
    exe = tmp_path / "abi_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fsanitize=float-cast-overflow", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(HERE, "abi_fuzz.cpp"), os.path.join(CSRC, "api.cpp"),
           os.path.join(CSRC, "tuned_table.cpp"), "-o", str(exe), "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", SBG_TUNE_FILE="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-3000:])
    assert "abi fuzz ok" in r.stdout
    calls, accepted = (int(x) for x in r.stdout.split()[3:5])
    assert calls == 60000 and accepted > 1000
