"""The tuned-table reader (host code that parses a user-supplied file) under
AddressSanitizer and UndefinedBehaviorSanitizer: tests/tuned_table_fuzz.cpp
compiles the reader's translation unit for the host with the sanitizers and
feeds it every prefix of a valid table, 20,000 seeded mutations and hostile
inputs (deep nesting, numbers outside int's range, NaN, unterminated strings).
No GPU is involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_tuned_table_reader_under_sanitizers(tmp_path):
    exe = tmp_path / "tuned_table_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fsanitize=float-cast-overflow", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1304_7053_amd", "csrc"),
           os.path.join(HERE, "tuned_table_fuzz.cpp"), "-o", str(exe), "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-3000:])
    assert "fuzz ok" in r.stdout
