"""Summaries of rocprofv3 output for this library's kernels.

rocprofv3 writes one CSV row per (dispatch, counter) in counter-collection
mode and one row per kernel in the `--stats` table; this module turns them
into per-kernel figures:

  traffic    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what
             the same counter reads for a copy of known size, averaged over
             the dispatches of each kernel: HBM bytes per launch;
  occupancy  SQ counters per kernel: waves, mean resident waves per CU, VALU
             and MFMA busy fractions, instructions per wave;
  stats      the kernel-trace statistics table, filtered by name.

Usage (from the repository root):

  python3 -m paper_1304_7053_amd.profsum traffic FETCH_CSV WRITE_CSV BENCH_JSON OUT_JSON
  python3 -m paper_1304_7053_amd.profsum occupancy SQ_CSV [REGEX]
  python3 -m paper_1304_7053_amd.profsum stats KERNEL_STATS_CSV [REGEX]

The markdown tables go to stdout.

Counter conventions (CDNA3/CDNA4 SQ block): SQ_WAVE_CYCLES,
SQ_BUSY_CYCLES, SQ_ACTIVE_INST_VALU count in quad-cycles summed over all
SQs; SQ_VALU_MFMA_BUSY_CYCLES counts MFMA-busy cycles summed over the CUs'
SIMDs; GRBM_GUI_ACTIVE counts GPU-busy cycles once per XCD.  The kernel's own
cycle count is taken as GRBM_GUI_ACTIVE / XCDS; every derived figure names
its formula in the table header."""
import csv
import json
import re
import sys
from collections import defaultdict

CUS = 256
SIMDS = 4 * CUS
XCDS = 8
CLOCK_GHZ = 2.4
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def norm(name):
    """Kernel name without a leading 'void ' and without spaces, to match the
    library's own demangled names against the profiler's."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    return re.sub(r"\s+", "", name)


def dispatches(path, regex=None):
    """{dispatch id: {"kernel": name, counter: value, ...}} from a
    counter-collection CSV."""
    out = {}
    rx = re.compile(regex) if regex else None
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            k = r["Kernel_Name"]
            if rx and not rx.search(k):
                continue
            d = out.setdefault(int(r["Dispatch_Id"]), {"kernel": k, "grid": int(r["Grid_Size"]),
                                                      "wg": int(r["Workgroup_Size"]), "vgpr": int(r["VGPR_Count"]),
                                                      "agpr": int(r.get("Accum_VGPR_Count") or 0),
                                                      "lds": int(r["LDS_Block_Size"]),
                                                      "scratch": int(r["Scratch_Size"]),
                                                      "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def copy_scale(disp, counter, nbytes):
    """Bytes per counter KiB: the largest dispatch of the copy kernel moves
    nbytes in that direction."""
    vals = [d[counter] for d in disp.values() if COPY_KERNEL in d["kernel"] and counter in d]
    if not vals:
        raise SystemExit(f"no {COPY_KERNEL} dispatch with {counter}: run with the calibration copy")
    return nbytes / (max(vals) * 1024.0), max(vals)


def per_kernel_mean(disp, counter):
    acc = defaultdict(lambda: [0.0, 0])
    for d in disp.values():
        if counter in d:
            a = acc[d["kernel"]]
            a[0] += d[counter]
            a[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def traffic(fetch_csv, write_csv, bench_json, out_json, source_hash):
    fe = dispatches(fetch_csv)
    wr = dispatches(write_csv)
    fs, fcopy = copy_scale(fe, "FETCH_SIZE", COPY_BYTES)
    ws, wcopy = copy_scale(wr, "WRITE_SIZE", COPY_BYTES)
    fm = per_kernel_mean(fe, "FETCH_SIZE")
    wm = per_kernel_mean(wr, "WRITE_SIZE")
    with open(bench_json) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])
    alg = {norm(k): v.get("algorithmic_bytes_per_launch") for k, v in bench.get("per_kernel", {}).items()}
    # secondary sections that name their kernel: the mean over the calls that use it
    sec = defaultdict(list)
    for part in (bench.get("secondary") or {}).values():
        for item in _leaves(part):
            if item.get("kernel") and item.get("algorithmic_bytes"):
                sec[norm(item["kernel"])].append(item["algorithmic_bytes"])
    for k, v in sec.items():
        alg.setdefault(k, sum(v) / len(v))
    # the step's dominant kernel is taken from the instance with the largest
    # algorithmic bytes over the step (timings under counter collection are
    # not representative)
    per = bench.get("per_kernel", {})
    dom = max(per, key=lambda k: per[k]["algorithmic_bytes_per_launch"] * per[k]["launches"]) if per else None
    rows = {}
    for k in sorted(set(fm) & set(wm)):
        if COPY_KERNEL in k:
            continue
        t = fm[k][0] * 1024 * fs + wm[k][0] * 1024 * ws
        rows[k] = {"fetch_kib": fm[k][0], "write_kib": wm[k][0], "launches": fm[k][1], "traffic": t,
                   "algorithmic": alg.get(norm(k))}
    by_lib = {}
    for k, r in rows.items():
        for lk in bench.get("per_kernel", {}):
            if norm(lk) == norm(k):
                by_lib[lk] = r["traffic"]
    dom_row = next((r for k, r in rows.items() if dom and norm(k) == norm(dom)), None)
    out = {"kernel": dom, "source_hash": source_hash,
           "traffic_bytes_per_launch": dom_row["traffic"] if dom_row else None,
           "algorithmic_bytes_per_launch": dom_row["algorithmic"] if dom_row else None,
           "fetch_scale": fs, "write_scale": ws,
           "copy_fetch_kib": fcopy, "copy_write_kib": wcopy,
           "all_kernels_traffic_bytes_per_launch": by_lib,
           "other_kernels_traffic_bytes_per_launch": {k: r["traffic"] for k, r in rows.items()
                                                      if not any(norm(k) == norm(x) for x in by_lib)}}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(f"FETCH_SIZE of the 1 GiB copy: {fcopy:.1f} KiB -> scale {fs:.4f}\n"
          f"WRITE_SIZE of the 1 GiB copy: {wcopy:.1f} KiB -> scale {ws:.4f}\n")
    print("| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | traffic MB | algorithmic MB | ratio |")
    print("|---|---|---|---|---|---|---|")
    for k, r in sorted(rows.items(), key=lambda kv: -kv[1]["traffic"] * kv[1]["launches"]):
        a = r["algorithmic"]
        print(f"| `{short(k)}` | {r['launches']} | {r['fetch_kib']:.0f} | {r['write_kib']:.0f} | "
              f"{r['traffic'] / 1e6:.2f} | {a / 1e6 if a else float('nan'):.2f} | "
              f"{r['traffic'] / a if a else float('nan'):.4f} |")


def _leaves(x):
    """Every dict in a nested bench section that has no dict values."""
    if isinstance(x, dict):
        subs = [v for v in x.values() if isinstance(v, dict)]
        if not subs:
            yield x
        for v in subs:
            yield from _leaves(v)


def short(k):
    """Kernel name without 'void ' and without its argument list."""
    k = re.sub(r"^void ", "", k.strip())
    if k.endswith(")"):
        depth = 0
        for i in range(len(k) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(k[i], 0)
            if depth == 0:
                return k[:i]
    return k


def occupancy(sq_csv, regex=None):
    disp = dispatches(sq_csv, regex)
    acc = defaultdict(lambda: defaultdict(float))
    for d in disp.values():
        a = acc[d["kernel"]]
        a["launches"] += 1
        for key in ("grid", "wg", "vgpr", "agpr", "lds", "scratch"):
            a[key] = d[key]
        a["ns"] += d["ns"]
        for c, v in d.items():
            if c.startswith(("SQ_", "GRBM_")):
                a[c] += v
    have_mfma = any("SQ_VALU_MFMA_BUSY_CYCLES" in a for a in acc.values())
    print("Per kernel, summed over its launches: cycles = GRBM_GUI_ACTIVE / 8 (XCDs), or the dispatch's "
          "timestamps x 2.4 GHz without that counter; "
          "resident waves per CU = 4 SQ_WAVE_CYCLES / (cycles x 256); "
          "VALU busy = 4 SQ_ACTIVE_INST_VALU / (cycles x 1024 SIMDs); "
          + ("MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x 1024 SIMDs); " if have_mfma else "")
          + "VALU and VMEM-read instructions per wave = SQ_INSTS_VALU / SQ_WAVES, SQ_INSTS_VMEM_RD / SQ_WAVES.\n")
    head = ["kernel", "launches", "VGPR+AGPR", "LDS B", "waves/launch", "cycles/launch", "us/launch (timestamps)",
            "resident waves/CU",
            "VALU busy", "MFMA busy" if have_mfma else None, "VALU inst/wave", "VMEM rd/wave", "LDS inst/wave"]
    head = [h for h in head if h]
    print("| " + " | ".join(head) + " |")
    print("|" + "---|" * len(head))
    for k, a in sorted(acc.items(), key=lambda kv: -kv[1].get("GRBM_GUI_ACTIVE", 0)):
        n = a["launches"]
        cyc = a.get("GRBM_GUI_ACTIVE", 0) / XCDS or a["ns"] * CLOCK_GHZ
        waves = a.get("SQ_WAVES", 0)
        row = [f"`{short(k)}`", f"{int(n)}", f"{int(a['vgpr'])}+{int(a['agpr'])}", f"{int(a['lds'])}",
               f"{waves / n:.0f}", f"{cyc / n:.0f}", f"{a['ns'] / n / 1e3:.1f}",
               f"{4 * a.get('SQ_WAVE_CYCLES', 0) / (cyc * CUS):.2f}" if cyc else "-",
               f"{4 * a.get('SQ_ACTIVE_INST_VALU', 0) / (cyc * SIMDS):.3f}" if cyc else "-"]
        if have_mfma:
            row.append(f"{a.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) / (cyc * SIMDS):.3f}" if cyc else "-")
        row += [f"{a.get('SQ_INSTS_VALU', 0) / waves:.1f}" if waves else "-",
                f"{a.get('SQ_INSTS_VMEM_RD', 0) / waves:.2f}" if waves else "-",
                f"{a.get('SQ_INSTS_LDS', 0) / waves:.2f}" if waves and "SQ_INSTS_LDS" in a else "-"]
        print("| " + " | ".join(row) + " |")


def stats(path, regex=None):
    rx = re.compile(regex) if regex else None
    with open(path, newline="") as f:
        rows = [r for r in csv.DictReader(f) if not rx or rx.search(r["Name"])]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | total ms | avg us | min us | max us |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")


def main(argv):
    if len(argv) >= 5 and argv[0] == "traffic":
        sys.path.insert(0, ".")
        from bench import kernel_source_hash
        traffic(argv[1], argv[2], argv[3], argv[4], kernel_source_hash())
    elif len(argv) >= 2 and argv[0] == "occupancy":
        occupancy(argv[1], argv[2] if len(argv) > 2 else None)
    elif len(argv) >= 2 and argv[0] == "stats":
        stats(argv[1], argv[2] if len(argv) > 2 else None)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
