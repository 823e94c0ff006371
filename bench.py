"""Benchmark: batched small-matrix GEMM throughput on one MI355X.

Workload ("size sweep", the paper's basic set of Sec. 8 widened to two real
types and four op pairs): N = 100,000 independent square pairs for every
n = 2..16, op in {NN, NT, TN, TT}, fp32 and fp64, alpha = 1.5, beta = -0.5,
minimal leading dimensions, entries U[-1,1].  One step = 120 batched GEMM
calls (one per dtype x n x op pair), each on its own buffers, so no call finds
its operands in a cache another call warmed (one step moves 28.7 GB).

Reported: GFLOP/s over the whole step (flops counted 2 n^3 per matrix for all
alpha, beta and ops, as in Sec. 8), the roofline of the kernel instance that
takes most of the step's time (algorithmic bytes per launch / mean launch
duration, timed with HIP events on the stream the kernels run on), the fp32
n = 16 case alone, and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12
N_BATCH = 100_000
SIZES = list(range(2, 17))
OPS = ["NN", "NT", "TN", "TT"]
ALPHA, BETA = 1.5, -0.5
METRIC = "batched GEMM GFLOP/s + % HBM roofline, n≤16, N=1e5; mixed/var-size vs plain FP32"


def kernel_source_hash():
    """Hash of the HIP sources, to tell whether stored counter readings still
    describe the kernels being timed."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1304_7053_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy), or None when the
    summary is for another kernel or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "gemm_sizesweep_hbm_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel") != kernel or d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000,
                    help="matrices per (dtype, n, op) call timed on the CPU oracle")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed region, copy 1 GiB once (reference kernel for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the batch shards across GPUs with no exchange, so run it once per GPU.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1304_7053_amd import sbg

    sbg.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device=dev)
    gen.manual_seed(13047053 + 2)

    # one set of buffers per call
    calls = []
    for dt_name, tdt, esz in (("float", torch.float32, 4), ("double", torch.float64, 8)):
        for n in SIZES:
            for ops in OPS:
                el = N_BATCH * n * n
                A = torch.rand(el, generator=gen, device=dev, dtype=tdt) * 2 - 1
                B = torch.rand(el, generator=gen, device=dev, dtype=tdt) * 2 - 1
                C = torch.rand(el, generator=gen, device=dev, dtype=tdt) * 2 - 1
                kname = sbg.describe_strided("s" if esz == 4 else "d", ops[0], ops[1], n, n, n, n, n * n,
                                             n, n * n, n, n * n, N_BATCH)
                calls.append(dict(dt=dt_name, tdt=tdt, esz=esz, n=n, ops=ops, A=A, B=B, C=C,
                                  flops=2.0 * n ** 3 * N_BATCH, bytes=4.0 * n * n * esz * N_BATCH,
                                  kernel=kname))
    torch.cuda.synchronize()

    def launch(c):
        n = c["n"]
        sbg.gemm_strided(c["ops"][0], c["ops"][1], n, n, n, ALPHA, c["A"], n, n * n, c["B"], n, n * n,
                         BETA, c["C"], n, n * n, N_BATCH, stream=stream)

    for _ in range(args.warmup):
        for c in calls:
            launch(c)
    torch.cuda.synchronize()

    # timed region: every launch bracketed by events on the launch stream
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in calls]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for i, c in enumerate(calls):
            ev[s][i][0].record(stream)
            launch(c)
            ev[s][i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    calib = None
    if args.calib_copy:
        src = torch.rand(1 << 28, generator=gen, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"kernel": "torch copy_ of 1 GiB float32", "bytes_read": 1 << 30, "bytes_written": 1 << 30}
        del src, dst

    flops_step = sum(c["flops"] for c in calls)
    bytes_step = sum(c["bytes"] for c in calls)
    per_kernel = {}
    per_call_ms = [0.0] * len(calls)
    for s in range(args.steps):
        for i, c in enumerate(calls):
            ms = ev[s][i][0].elapsed_time(ev[s][i][1])
            per_call_ms[i] += ms / args.steps
            d = per_kernel.setdefault(c["kernel"], {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0})
            d["ms"] += ms
            d["bytes"] += c["bytes"]
            d["flops"] += c["flops"]
            d["launches"] += 1
    dom_name, dom = max(per_kernel.items(), key=lambda kv: kv[1]["ms"])
    dom_avg_s = dom["ms"] / dom["launches"] / 1e3
    dom_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_bytes / dom_avg_s / 1e9

    # fp32 n = 16 (the headline case of the paper's abstract), per op pair
    head = {}
    for i, c in enumerate(calls):
        if c["dt"] == "float" and c["n"] == 16:
            t = per_call_ms[i] / 1e3
            head[c["ops"]] = {"us": round(t * 1e6, 2), "gflops": round(c["flops"] / t / 1e9, 1),
                              "hbm_frac": round(c["bytes"] / t / HBM_PEAK, 4)}

    per_size = {}
    for i, c in enumerate(calls):
        key = f"{'s' if c['dt'] == 'float' else 'd'}{c['n']}"
        d = per_size.setdefault(key, [0.0, 0.0, 0.0])
        d[0] += c["flops"]
        d[1] += c["bytes"]
        d[2] += per_call_ms[i] / 1e3
    sizes_out = {k: {"gflops": round(v[0] / v[2] / 1e9, 1), "hbm_frac": round(v[1] / v[2] / HBM_PEAK, 4)}
                 for k, v in per_size.items()}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(calls, args.cpu_sample)

    out = {
        "metric": METRIC,
        "value": round(flops_step * args.steps / elapsed / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded U[-1,1], generated on device)",
        "config": {"workload": "size sweep: N=100000 square n=2..16, ops NN/NT/TN/TT, fp32+fp64, "
                               "alpha=1.5 beta=-0.5, strided minimal-LD layout, 120 calls per step",
                   "global_batch": N_BATCH, "parallelism": "single GPU"},
        "hbm_frac_step": round(bytes_step * args.steps / elapsed / HBM_PEAK, 4),
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved * 1e9 / HBM_PEAK, 4),
                     "traffic": stored_traffic(dom_name), "mean_launch_us": round(dom_avg_s * 1e6, 3),
                     "launches": dom["launches"], "algorithmic_bytes_per_launch": dom_bytes},
        "fp32_n16": head,
        "per_size": sizes_out,
        "cpu_baseline": cpu,
    }
    if calib:
        out["calib_copy"] = calib
    print(json.dumps(out), flush=True)


def cpu_baseline(calls, sample):
    """The CPU oracle (FP64 accumulation, OpenMP over the batch) on `sample`
    matrices of every call of one step, scaled to GFLOP/s."""
    import numpy as np

    import oracle

    threads = oracle.max_threads()
    flops = 0.0
    t_total = 0.0
    for c in calls:
        n = c["n"]
        el = sample * n * n
        A = c["A"][:el].cpu().numpy()
        B = c["B"][:el].cpu().numpy()
        C = c["C"][:el].cpu().numpy()
        t0 = time.perf_counter()
        oracle.gemm_strided(c["ops"][0], c["ops"][1], n, n, n, ALPHA, A, n, n * n, B, n, n * n, BETA, C, n,
                            n * n, sample)
        t_total += time.perf_counter() - t0
        flops += 2.0 * n ** 3 * sample
    del np
    return {"value": round(flops / t_total / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} matrices of each of the 120 calls of one step "
                      f"({flops / 1e9:.2f} GFLOP, {t_total:.1f} s)"}


if __name__ == "__main__":
    main()
