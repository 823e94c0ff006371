"""The tuned table (JSON written by the autotuner, read by libsbg.so at load
time): entries select the kernel and launch shape of matching calls, knobs set
to non-automatic values override them, and a table of another version, a
malformed file or an empty SBG_TUNE_FILE leave the built-in rules in charge.
Checked through sbg_describe_strided, which plans a call exactly as a launch
does and needs no GPU (each case in a fresh process, since the table is read
once per process)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
from paper_1304_7053_amd import sbg
sbg.load()
out = {"info": sbg.tuned_table_info()}
def d(p, ops, s, batch=100000):
    ra = s
    return sbg.describe_strided(p, ops[0], ops[1], s, s, s, s, s * s, s, s * s, s, s * s, batch)
for key, (p, ops, s) in {"s_NN_5": ("s", "NN", 5), "s_NN_12": ("s", "NN", 12), "d_TN_10": ("d", "TN", 10),
                         "s_NT_16": ("s", "NT", 16), "c_NN_4": ("c", "NN", 4), "s_TT_5": ("s", "TT", 5)}.items():
    out[key] = d(p, ops, s)
old = sbg.set_tuning("path", 2)
out["s_NN_5_forced_team"] = d("s", "NN", 5)
sbg.set_tuning("path", old)
old = sbg.set_tuning("table", 0)
out["s_NN_5_table_off"] = d("s", "NN", 5)
sbg.set_tuning("table", old)
print(json.dumps(out))
"""


def _probe(tmp_path, table_text):
    env = dict(os.environ)
    if table_text is None:
        env["SBG_TUNE_FILE"] = ""
    else:
        f = tmp_path / "table.json"
        f.write_text(table_text)
        env["SBG_TUNE_FILE"] = str(f)
    for k in ("SBG_PATH", "SBG_STAGED", "SBG_UNROLL", "SBG_TABLE"):
        env.pop(k, None)
    r = subprocess.run([sys.executable, "-c", PROBE, ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def _entry(**kw):
    e = {"type": "s", "form": "strided", "ops": "NN", "size": 5, "path": "team", "unroll": 0, "wg_per_cu": 0,
         "xcd_chunk": 0, "us": 1.0, "default_us": 1.0, "paths_us": {"mfma": 2.0, "team": 1.0}}
    e.update(kw)
    return e


TABLE = {"version": 1, "library": "libsbg", "entries": [
    _entry(size=5, path="mfma", unroll=1),
    _entry(size=12, path="team"),
    _entry(type="d", ops="TN", size=10, path="staged"),
    _entry(ops="NT", size=16, path="mfma", unroll=1),
    _entry(type="c", size=4, path="mfma"),
    _entry(type="q", size=5, path="team"),          # unknown type: ignored
    _entry(size=40, path="team"),                   # size out of range: ignored
], "grid_sweep": [{"type": "s", "points": [{"work_groups": 8, "us": 1.0}]}]}


def test_table_entries_select_kernels(tmp_path):
    out = _probe(tmp_path, json.dumps(TABLE, indent=1))
    n, info = out["info"]
    assert n == 5 and "version=1" in info
    assert "gemm_mfma_kernel<float, float, 0, 8, 1," in out["s_NN_5"]      # MFMA, unroll 1
    assert "gemm_team_kernel<float, 16," in out["s_NN_12"]                # team in the 16 class
    assert "gemm_staged_kernel<double" in out["d_TN_10"]
    assert "gemm_mfma_kernel<float, float, 0, 16, 1," in out["s_NT_16"]
    assert "gemm_mfma_kernel<HIP_vector_type<float, 2u>" in out["c_NN_4"]
    assert "gemm_team_kernel<float, 8," in out["s_TT_5"]                  # no entry: built-in rule
    assert "gemm_team_kernel<float, 8," in out["s_NN_5_forced_team"]      # knob beats table
    assert "gemm_team_kernel<float, 8," in out["s_NN_5_table_off"]        # table switched off


def test_other_version_malformed_or_no_table(tmp_path):
    for text in (json.dumps(dict(TABLE, version=2)), json.dumps(TABLE)[:-40], "not json", None):
        out = _probe(tmp_path, text)
        assert out["info"][0] == 0
        assert "gemm_team_kernel<float, 8," in out["s_NN_5"]
        assert "gemm_mfma_kernel" in out["s_NN_12"] or "gemm_staged_kernel" in out["s_NN_12"]
