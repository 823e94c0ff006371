"""Autotuner of the batched GEMM library: kernel choice and launch shape per
(type, batch form, op pair, size), written as a versioned JSON table that
libsbg.so reads at load time (tuned.json beside the library, or the file
named by SBG_TUNE_FILE).

The paper tunes one launch parameter by hand -- the number of thread blocks,
whose plateau it reports near 2,000 on its GPU (Sec. 7 and the block-count
study of Sec. 8) -- and picks kernels per size with templates (Sec. 6-7).
Here every choice the library makes per call is measured on the device:

  * the kernel: MFMA tile kernel, LDS-staged kernel (packed strided batches)
    or team kernel (sizes <= 8, and <= 16 for real types);
  * for the persistent kernels: the tile unroll U, the work-groups per CU and
    the XCD run length (coordinate search in that order);
  * a key whose best choice is not at least 3% faster than the built-in rules
    keeps the rules (entry path "rule");

and the launch-shape (grid-size) sweep itself is recorded beside the table.

Timing (timing.py): HIP events on the launch stream around each call, the
series queued behind a spin kernel so that no host launch time enters an
interval, medians over repetitions, operands rotated over buffer sets whose
total exceeds the 256 MB Infinity Cache, so every call reads its operands
from HBM.

Usage (on the GPU):  python -m paper_1304_7053_amd.tune --out tuned.json
"""
import argparse
import json
import math
import os
import sys
import time

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_1304_7053_amd import sbg, timing  # noqa: E402

TABLE_VERSION = 1
DEFAULT_OUT = os.path.join(HERE, "tuned.json")
MIN_SET_BYTES = 768 << 20          # rotate buffers until this much is touched
MAX_TOTAL_BYTES = 6 << 30
TYPES = {"s": torch.float32, "d": torch.float64, "c": torch.complex64, "z": torch.complex128}
PATH_NAME = {1: "mfma", 2: "team", 3: "staged"}
MARGIN = 0.97          # a tuned choice must beat the built-in rules by 3%


def stored(op, rows, cols):
    return (rows, cols) if op in "NR" else (cols, rows)


class Workload:
    """Rotating operand sets of one (type, size, batch) square workload, in
    the strided packed layout; pointer arrays address the same matrices."""

    def __init__(self, prefix, s, batch):
        self.prefix, self.s, self.batch = prefix, s, batch
        dt = TYPES[prefix]
        esz = torch.empty(0, dtype=dt).element_size()
        per = 3 * s * s * batch * esz
        self.nsets = max(2, min(math.ceil(MIN_SET_BYTES / per), max(1, MAX_TOTAL_BYTES // per)))
        g = torch.Generator(device="cuda").manual_seed(13047053 + s)
        self.sets = []
        for _ in range(self.nsets):
            bufs = []
            for _ in range(3):
                x = torch.empty(s * s * batch, dtype=dt, device="cuda")
                if x.is_complex():
                    torch.view_as_real(x).uniform_(-1, 1, generator=g)
                else:
                    x.uniform_(-1, 1, generator=g)
                bufs.append(x)
            ptrs = [torch.arange(batch, device="cuda", dtype=torch.int64) * (s * s * esz) + b.data_ptr()
                    for b in bufs]
            self.sets.append((bufs, ptrs))
        self.i = 0

    def call(self, ops, form, alpha=1.5, beta=-0.5):
        s = self.s
        (A, B, C), (pA, pB, pC) = self.sets[self.i % self.nsets]
        self.i += 1
        ra, ca = stored(ops[0], s, s)
        rb, cb = stored(ops[1], s, s)
        if form == "strided":
            sbg.gemm_strided(ops[0], ops[1], s, s, s, alpha, A, ra, ra * ca, B, rb, rb * cb, beta, C, s, s * s,
                             self.batch)
        else:
            sbg.gemm_batched(ops[0], ops[1], s, s, s, alpha, pA, ra, pB, rb, beta, pC, s, self.batch, C.dtype)

    def time(self, ops, form, reps=15, warmup=3):
        """Median microseconds of one call (the series queued behind a spin
        kernel, so the events bracket the kernels alone)."""
        for _ in range(warmup):
            self.call(ops, form)
        ts = timing.time_series(lambda i: self.call(ops, form), reps)
        return timing.median(ts) * 1e6


def measure(w, ops, form, knobs, reps):
    with sbg.tuned(**knobs):
        return w.time(ops, form, reps)


def tune_key(w, ops, form, reps):
    """Best kernel and launch shape for one key; returns the table entry."""
    prefix, s = w.prefix, w.s
    real = prefix in "sd"
    default = measure(w, ops, form, {"table": 0}, reps)
    best = None
    cands = [("mfma", {"table": 0, "path": 1, "staged": 0})]
    if form == "strided":
        cands.append(("staged", {"table": 0, "path": 1, "staged": 1}))
    if s <= 8 or real:
        cands.append(("team", {"table": 0, "path": 2 if s <= 8 else 3}))
    results = {}
    for name, kn in cands:
        results[name] = measure(w, ops, form, kn, reps)
        if best is None or results[name] < best[1]:
            best = (name, results[name], dict(kn))
    name, us, kn = best
    entry = {"path": name, "unroll": 0, "wg_per_cu": 0, "xcd_chunk": 0}
    if name in ("mfma", "staged"):
        # coordinate search over the persistent launch shape
        if name == "mfma":
            for u in (1, 2, 4, 8):
                t = measure(w, ops, form, dict(kn, unroll=u), reps)
                if t < us:
                    us, entry["unroll"] = t, u
            if entry["unroll"]:
                kn["unroll"] = entry["unroll"]
        for wg in (1, 2, 3, 6, 8, 16, 32):
            t = measure(w, ops, form, dict(kn, wg_per_cu=wg), reps)
            if t < us:
                us, entry["wg_per_cu"] = t, wg
        if entry["wg_per_cu"]:
            kn["wg_per_cu"] = entry["wg_per_cu"]
        for xc in (1, 4, 64):
            t = measure(w, ops, form, dict(kn, xcd_chunk=xc), reps)
            if t < us:
                us, entry["xcd_chunk"] = t, xc
    if us > MARGIN * default:
        # not clearly ahead of the built-in rules: keep them (a choice inside
        # the timing noise would only add run-to-run variation)
        entry = {"path": "rule", "unroll": 0, "wg_per_cu": 0, "xcd_chunk": 0}
        us = default
    esz = torch.empty(0, dtype=TYPES[prefix]).element_size()
    algo = 4 * s * s * esz * w.batch + (24 * w.batch if form == "pointer" else 0)
    entry.update({"type": prefix, "form": form, "ops": ops, "size": s, "us": round(us, 3),
                  "default_us": round(default, 3), "paths_us": {k: round(v, 3) for k, v in results.items()},
                  "hbm_frac": round(algo / (us * 1e-6) / 8e12, 4),
                  "default_hbm_frac": round(algo / (default * 1e-6) / 8e12, 4)})
    return entry


def grid_sweep(batch, reps):
    """Launch-shape sweep: the persistent MFMA kernel at fixed work, the
    work-group count varied (the paper's block-count study)."""
    out = []
    for prefix, s in (("s", 16), ("s", 8), ("d", 16)):
        w = Workload(prefix, s, batch)
        esz = torch.empty(0, dtype=TYPES[prefix]).element_size()
        algo = 4 * s * s * esz * batch
        pts = []
        for g in (8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192):
            t = measure(w, "NN", "strided", {"table": 0, "path": 1, "staged": 0, "grid": g}, reps)
            pts.append({"work_groups": g, "us": round(t, 3), "hbm_frac": round(algo / (t * 1e-6) / 8e12, 4)})
        out.append({"type": prefix, "size": s, "ops": "NN", "batch": batch, "kernel": "mfma", "points": pts})
        del w
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--types", default="sdcz")
    ap.add_argument("--forms", default="strided,pointer")
    ap.add_argument("--ops", default="NN,NT,TN,TT")
    ap.add_argument("--sizes", default="1-16")
    ap.add_argument("--batch", type=int, default=100_000)
    ap.add_argument("--reps", type=int, default=15)
    ap.add_argument("--no-grid-sweep", action="store_true")
    a = ap.parse_args(argv)
    lo, _, hi = a.sizes.partition("-")
    sizes = list(range(int(lo), int(hi or lo) + 1))
    sbg.load()
    props = torch.cuda.get_device_properties(0)
    t0 = time.time()
    entries = []
    for prefix in a.types:
        for s in sizes:
            w = Workload(prefix, s, a.batch)
            for form in a.forms.split(","):
                for ops in a.ops.split(","):
                    e = tune_key(w, ops, form, a.reps)
                    entries.append(e)
                    print(f"{prefix} {form:7s} {ops} n={s:2d}: {e['path']:6s} U={e['unroll']} wg={e['wg_per_cu']} "
                          f"xcd={e['xcd_chunk']}  {e['us']:9.2f} us ({e['hbm_frac']:.3f})  default "
                          f"{e['default_us']:9.2f} us ({e['default_hbm_frac']:.3f})", flush=True)
            del w
            torch.cuda.empty_cache()
    sweep = [] if a.no_grid_sweep else grid_sweep(a.batch, a.reps)
    doc = {
        "version": TABLE_VERSION,
        "library": "libsbg",
        "device": props.name,
        "gcn_arch": getattr(props, "gcnArchName", ""),
        "compute_units": props.multi_processor_count,
        "batch": a.batch,
        "alpha_beta": [1.5, -0.5],
        "timing": "median of HIP-event timed calls queued behind a spin kernel, operands rotated over sets "
                  "larger than the Infinity Cache",
        "seconds": round(time.time() - t0, 1),
        "entries": entries,
        "grid_sweep": sweep,
    }
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {len(entries)} entries to {a.out} in {doc['seconds']} s", flush=True)


if __name__ == "__main__":
    main()
