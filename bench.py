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
    summary has no reading for that kernel or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "gemm_sizesweep_hbm_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    if d.get("kernel") == kernel:
        return d.get("traffic_bytes_per_launch")
    # the dominant instance of a run can be another of the near-equal op variants
    return d.get("all_kernels_traffic_bytes_per_launch", {}).get(kernel)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000,
                    help="matrices per (dtype, n, op) call timed on the CPU oracle")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (small batch, complex, variable-size modes, FEM)")
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

    # free the sweep's 29 GB before the secondary workloads
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(calls, args.cpu_sample)
    del calls
    torch.cuda.empty_cache()
    secondary = None
    if not args.no_extras:
        secondary = {}
        for name, fn in (("small_batch", sec_small_batch), ("complex", sec_complex_sweep),
                         ("varsize_precision", sec_varsize_modes), ("fem", sec_fem_chain),
                         ("fixed_operand", sec_fixed_operand), ("batch_sweep", sec_batch_sweep),
                         ("large_sizes", sec_large_sizes), ("blas_routines", sec_blas_routines)):
            try:
                secondary[name] = fn(stream)
            except Exception as e:  # a secondary failure must not hide the primary line
                secondary[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()

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
        "secondary": secondary,
    }
    if calib:
        out["calib_copy"] = calib
    print(json.dumps(out), flush=True)


# ---- secondary workloads (reported beside the primary line) ---------------

def _graph(fn, stream):
    """Capture fn() (library calls on the current stream) in a HIP graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        fn()                       # warm-up outside capture
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        fn()
    torch.cuda.synchronize()
    return g


def _time_replays(g, reps, flush=None):
    """Median and min seconds of graph replays, the Infinity Cache flushed
    (a 512 MB write) before each one outside the timed interval."""
    import torch
    ts = []
    for _ in range(reps):
        if flush is not None:
            flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cur = torch.cuda.current_stream()
        e0.record(cur)
        g.replay()
        e1.record(cur)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    return ts[len(ts) // 2], ts[0]


def sec_small_batch(stream):
    """N = 1000 pairs of 8x8x8, NN, alpha = 1, beta = 0 (C not read): launch
    latency regime.  Median time of an eager call and of a graph replay."""
    import torch

    from paper_1304_7053_amd import sbg
    N, s = 1000, 8
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 1)
    A = torch.rand(N * s * s, generator=gen, device="cuda") * 2 - 1
    B = torch.rand(N * s * s, generator=gen, device="cuda") * 2 - 1
    C = torch.empty(N * s * s, device="cuda")
    call = lambda: sbg.gemm_strided("N", "N", s, s, s, 1.0, A, s, s * s, B, s, s * s, 0.0, C, s, s * s, N)  # noqa
    ts = []
    for _ in range(200):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    ts.sort()
    g = _graph(call, stream)
    med_g, _ = _time_replays(g, 200)
    return {"workload": "N=1000, 8x8x8, NN, alpha=1, beta=0, fp32", "us_per_call_median": round(ts[100], 2),
            "us_per_graph_replay_median": round(med_g * 1e6, 2),
            "gflops_per_call": round(2 * s ** 3 * N / (ts[100] * 1e-6) / 1e9, 1)}


def sec_complex_sweep(stream):
    """N = 100,000 complex pairs, n in {4, 8, 12, 16}, all nine op pairs over
    {N, T, C}, alpha = (1, 0.5), beta = (0.25, -1); GFLOP/s (8 n^3 per
    matrix) and HBM fraction per (type, n), each call on its own buffers."""
    import torch

    from paper_1304_7053_amd import sbg
    N = 100_000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 3)
    out = {}
    for tdt, esz, name in ((torch.complex64, 8, "c"), (torch.complex128, 16, "z")):
        rdt = torch.float32 if tdt == torch.complex64 else torch.float64
        for n in (4, 8, 12, 16):
            el = N * n * n
            bufs = []
            for _ in range(9):
                bufs.append([(torch.rand(2 * el, generator=gen, device="cuda", dtype=rdt) * 2 - 1).view(tdt)
                             for _ in range(3)])
            ops = [a + b for a in "NTC" for b in "NTC"]
            for i, op in enumerate(ops):     # warm-up
                A, B, C = bufs[i]
                sbg.gemm_strided(op[0], op[1], n, n, n, complex(1, 0.5), A, n, n * n, B, n, n * n,
                                 complex(0.25, -1), C, n, n * n, N)
            torch.cuda.synchronize()
            evs = []
            for rep in range(3):
                for i, op in enumerate(ops):
                    A, B, C = bufs[i]
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    sbg.gemm_strided(op[0], op[1], n, n, n, complex(1, 0.5), A, n, n * n, B, n, n * n,
                                     complex(0.25, -1), C, n, n * n, N)
                    e1.record(stream)
                    evs.append((op, e0, e1))
            torch.cuda.synchronize()
            t_op = {}
            for op, e0, e1 in evs:
                t_op.setdefault(op, []).append(e0.elapsed_time(e1) / 1e3)
            tmed = {op: sorted(v)[len(v) // 2] for op, v in t_op.items()}
            tot = sum(tmed.values())
            flops = 8.0 * n ** 3 * N * 9
            byts = 4.0 * n * n * esz * N * 9
            out[f"{name}{n}"] = {"gflops": round(flops / tot / 1e9, 1), "hbm_frac": round(byts / tot / HBM_PEAK, 4),
                                 "op_vs_NN": {op: round(tmed["NN"] / t, 3) for op, t in tmed.items()}}
            del bufs
            torch.cuda.empty_cache()
    return out


def sec_varsize_modes(stream):
    """N = 200,000 matrices with m, n, k drawn independently (40% at 8, 30% at
    16, the rest uniform), pointer arrays, one variable-size call (binning +
    persistent GEMM) captured in a HIP graph; for each precision mode and
    both input sets: GFLOP/s, HBM fraction (algorithmic bytes incl. per-matrix
    pointers, sizes, leading dimensions and scales) and the deviation from the
    binary32 result of the same call."""
    import numpy as np
    import torch

    from paper_1304_7053_amd import inputs, sbg
    N = 200_000
    g = inputs.rng(4)
    m, n, k = inputs.varsize_dims(g, N)
    m64, n64, k64 = (x.astype(np.int64) for x in (m, n, k))
    offs = {}
    for name, cnt in (("A", m64 * k64), ("B", k64 * n64), ("C", m64 * n64)):
        o = np.zeros(N, dtype=np.int64)
        o[1:] = np.cumsum(cnt)[:-1]
        offs[name] = (o, int(cnt.sum()))
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    dm, dn, dk = dev(m), dev(n), dev(k)
    dlda, dldb, dldc = dev(np.maximum(m, 1)), dev(np.maximum(k, 1)), dev(np.maximum(m, 1))
    ws = torch.zeros(sbg.vbatched_workspace_size(N) // 4 + 1, dtype=torch.int32, device="cuda")
    flush = torch.empty(128 * 1024 * 1024, device="cuda")
    flops = float(np.sum(2 * m64 * n64 * k64))
    meta = 24 + 24                          # three pointers, six int32 sizes / leading dimensions
    res = {"workload": "N=200000 variable m,n,k (40% 8, 30% 16, rest uniform), NN, alpha=1.5, beta=-0.5",
           "gflop_per_call": round(flops / 1e9, 4)}
    for dist in ("uniform", "logu"):
        A32 = dev(inputs.DISTS[dist](g, (offs["A"][1],), np.float32))
        B32 = dev(inputs.DISTS[dist](g, (offs["B"][1],), np.float32))
        C0 = dev(inputs.DISTS[dist](g, (offs["C"][1],), np.float32))
        C = torch.empty_like(C0)
        pC = torch.tensor(C.data_ptr() + offs["C"][0] * 4, device="cuda")
        results = {}
        ref = None
        for mode in ("f32", "bf16", "f16", "e4m3", "bf16x3"):
            sA = sB = None
            qtime = None
            if mode in ("bf16", "f16"):
                tdt = torch.bfloat16 if mode == "bf16" else torch.float16
                Ain, Bin, esz = A32.to(tdt), B32.to(tdt), 2
                code, cmode = (sbg.R_16BF if mode == "bf16" else sbg.R_16F), sbg.MODE_PLAIN
            elif mode == "e4m3":
                Ain = torch.empty(offs["A"][1], dtype=torch.uint8, device="cuda")
                Bin = torch.empty(offs["B"][1], dtype=torch.uint8, device="cuda")
                esz, code, cmode = 1, sbg.R_8F_E4M3, sbg.MODE_PLAIN
                sA = torch.empty(N, device="cuda")
                sB = torch.empty(N, device="cuda")
                pA32 = torch.tensor(A32.data_ptr() + offs["A"][0] * 4, device="cuda")
                pB32 = torch.tensor(B32.data_ptr() + offs["B"][0] * 4, device="cuda")
                pAq = torch.tensor(Ain.data_ptr() + offs["A"][0], device="cuda")
                pBq = torch.tensor(Bin.data_ptr() + offs["B"][0], device="cuda")

                def quant():
                    sbg.quantize_e4m3_vbatched(dm, dk, 16, 16, pA32, dlda, pAq, dlda, sA, N)
                    sbg.quantize_e4m3_vbatched(dk, dn, 16, 16, pB32, dldb, pBq, dldb, sB, N)
                qg = _graph(quant, stream)
                qtime, _ = _time_replays(qg, 5, flush)
            else:
                Ain, Bin, esz = A32, B32, 4
                code = sbg.R_32F
                cmode = sbg.MODE_BF16X3 if mode == "bf16x3" else sbg.MODE_PLAIN
            pA = torch.tensor(Ain.data_ptr() + offs["A"][0] * esz, device="cuda")
            pB = torch.tensor(Bin.data_ptr() + offs["B"][0] * esz, device="cuda")

            def call():
                sbg.gemm_vbatched_ex("N", "N", dm, dn, dk, 16, 16, 16, 1.5, pA, dlda, sA, pB, dldb, sB, -0.5, pC,
                                     dldc, N, code, cmode, ws)
            C.copy_(C0)
            gr = _graph(call, stream)
            C.copy_(C0)
            torch.cuda.synchronize()
            gr.replay()                      # one clean replay for the deviation
            torch.cuda.synchronize()
            if ref is None:
                ref = C.clone()
                dev_info = {"max_abs_dev_over_max_abs": 0.0}
            else:
                d = (C - ref).abs()
                dev_info = {"max_abs_dev_over_max_abs": float(d.max() / ref.abs().max())}
            med, mn = _time_replays(gr, 7, flush)
            byts = float(np.sum((m64 * k64 + k64 * n64) * esz + 2 * m64 * n64 * 4)) + N * meta + \
                (8 * N if mode == "e4m3" else 0)
            results[mode] = {"us": round(med * 1e6, 1), "gflops": round(flops / med / 1e9, 1),
                             "hbm_frac": round(byts / med / HBM_PEAK, 4), **dev_info}
            if qtime is not None:
                results[mode]["quantize_us"] = round(qtime * 1e6, 1)
            del gr
        res[dist] = results
        del A32, B32, C0, C
        torch.cuda.empty_cache()
    return res


def sec_fem_chain(stream):
    """N = 1,000,000 FEM elements: K = B^T (D B) (two batched GEMMs) and its
    backward from dK (four), each sequence captured as one HIP graph."""
    import numpy as np
    import torch

    from paper_1304_7053_amd import inputs
    from paper_1304_7053_amd.autograd import gemm_rm
    N = 1_000_000
    g = inputs.rng(5)
    B, D, dK = (torch.from_numpy(x).cuda() for x in inputs.fem_element_batch(g, N))
    T = torch.empty((N, 6, 12), device="cuda")
    K = torch.empty((N, 12, 12), device="cuda")
    dT = torch.empty_like(T)
    dB = torch.empty_like(B)
    dD = torch.empty_like(D)
    flush = torch.empty(128 * 1024 * 1024, device="cuda")

    def fwd():
        gemm_rm("N", "N", 1.0, D, B, 0.0, T)
        gemm_rm("T", "N", 1.0, B, T, 0.0, K)

    def bwd():
        gemm_rm("N", "N", 1.0, B, dK, 0.0, dT)
        gemm_rm("N", "T", 1.0, T, dK, 0.0, dB)
        gemm_rm("T", "N", 1.0, D, dT, 1.0, dB)
        gemm_rm("N", "T", 1.0, dT, B, 0.0, dD)
    gf, gb = _graph(fwd, stream), _graph(bwd, stream)
    tf, _ = _time_replays(gf, 7, flush)
    tb, _ = _time_replays(gb, 7, flush)
    ffl, bfl = 2592.0 * N, 5184.0 * N
    fby, bby = 1872.0 * N, 4032.0 * N
    del np
    return {"workload": "N=1e6 elements, B 6x12, D 6x6, fp32",
            "forward": {"us": round(tf * 1e6, 1), "gflops": round(ffl / tf / 1e9, 1),
                        "hbm_frac": round(fby / tf / HBM_PEAK, 4)},
            "backward": {"us": round(tb * 1e6, 1), "gflops": round(bfl / tb / 1e9, 1),
                         "hbm_frac": round(bby / tb / HBM_PEAK, 4)}}


def _time_calls(call, reps, flush):
    """Median seconds of `call` (eager launches on the current stream), the
    Infinity Cache flushed before each one outside the timed interval."""
    import torch
    ts = []
    cur = torch.cuda.current_stream()
    call()
    for _ in range(reps):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        call()
        e1.record(cur)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def sec_fixed_operand(stream):
    """The fixed-operand case the paper names as a next step (Sec. 9): one A
    (strideA = 0) or one B (strideB = 0) shared by the whole batch, against
    the ordinary batch; N = 100,000, NN, alpha = 1.5, beta = -0.5.  The HBM
    fraction counts the shared matrix once."""
    import torch

    from paper_1304_7053_amd import sbg
    N = 100_000
    flush = torch.empty(128 * 1024 * 1024, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 6)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        for n in (8, 16):
            el = N * n * n
            A = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            B = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            C = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            res = {}
            for case, sa, sb in (("batched", n * n, n * n), ("shared_A", 0, n * n), ("shared_B", n * n, 0)):
                call = lambda: sbg.gemm_strided("N", "N", n, n, n, 1.5, A, n, sa, B, n, sb, -0.5, C, n,  # noqa: E731
                                                n * n, N)
                t = _time_calls(call, 7, flush)
                byts = esz * n * n * (N * (2 + (sa > 0) + (sb > 0)) + (sa == 0) + (sb == 0))
                res[case] = {"us": round(t * 1e6, 1), "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                             "hbm_frac": round(byts / t / HBM_PEAK, 4)}
            out[f"{tname}_n{n}"] = res
            del A, B, C
    return out


def sec_batch_sweep(stream):
    """Batch-size sweep (the paper's plateau question, Sec. 8): fp32 NN,
    alpha = 1.5, beta = -0.5, n in {8, 16}, N from 2,000 to 1,000,000."""
    import torch

    from paper_1304_7053_amd import sbg
    flush = torch.empty(128 * 1024 * 1024, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 7)
    out = {}
    for n in (8, 16):
        row = {}
        for N in (2000, 5000, 20000, 100_000, 1_000_000):
            el = N * n * n
            A = torch.rand(el, generator=gen, device="cuda") * 2 - 1
            B = torch.rand(el, generator=gen, device="cuda") * 2 - 1
            C = torch.rand(el, generator=gen, device="cuda") * 2 - 1
            call = lambda: sbg.gemm_strided("N", "N", n, n, n, 1.5, A, n, n * n, B, n, n * n, -0.5, C, n,  # noqa: E731
                                            n * n, N)
            t = _time_calls(call, 7, flush)
            row[str(N)] = {"us": round(t * 1e6, 2), "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                           "hbm_frac": round(16.0 * n * n * N / t / HBM_PEAK, 4)}
            del A, B, C
        out[f"f32_n{n}"] = row
    return out


def sec_large_sizes(stream):
    """Sizes above 16 (the sub-blocked kernel, the paper's extension remark):
    square n in {24, 32, 48, 64}, NN and TN, alpha = 1.5, beta = -0.5, with
    about 400 MB per fp32 operand (800 MB fp64).  HBM fraction counts A, B
    and C read once and C written once (the kernel re-reads A and B blocks
    from L2 for each block of C)."""
    import torch

    from paper_1304_7053_amd import sbg
    flush = torch.empty(128 * 1024 * 1024, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 8)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        for n in (24, 32, 48, 64):
            N = 100_000_000 // (n * n)
            el = N * n * n
            A = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            B = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            C = torch.rand(el, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            for ops in ("NN", "TN"):
                call = lambda: sbg.gemm_strided(ops[0], ops[1], n, n, n, 1.5, A, n, n * n, B, n, n * n,  # noqa: E731
                                                -0.5, C, n, n * n, N)
                t = _time_calls(call, 5, flush)
                out[f"{tname}_n{n}_{ops}"] = {"N": N, "us": round(t * 1e6, 1),
                                               "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                                               "hbm_frac": round(4.0 * esz * el / t / HBM_PEAK, 4)}
            del A, B, C
    return out


def sec_blas_routines(stream):
    """Batched GEMV and TRSM in the strided interface (formulated on batched
    GEMM, the paper's outlook): GEMV y = 1.5 op(A) x - 0.5 y with A 16 x 16,
    N = 10^6, ops N and T; TRSM op(A) X = 1.5 B with A 16 x 16 lower, 16
    right-hand sides, N = 200,000, and a blocked order-64 case (N = 20,000).
    HBM bytes: GEMV A + x + y read + y written; TRSM the triangle of A + B
    read + B written."""
    import torch

    from paper_1304_7053_amd import sbg
    flush = torch.empty(128 * 1024 * 1024, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 9)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        N, m, n = 1_000_000, 16, 16
        A = torch.rand(N * m * n, generator=gen, device="cuda", dtype=tdt) * 2 - 1
        x = torch.rand(N * n, generator=gen, device="cuda", dtype=tdt) * 2 - 1
        y = torch.rand(N * m, generator=gen, device="cuda", dtype=tdt) * 2 - 1
        for trans in "NT":
            call = lambda: sbg.gemv_strided(trans, m, n, 1.5, A, m, m * n, x, 1, n, -0.5, y, 1, m, N)  # noqa: E731
            t = _time_calls(call, 7, flush)
            byts = esz * N * (m * n + n + 2 * m)
            out[f"gemv_{tname}_16x16_{trans}"] = {"N": N, "us": round(t * 1e6, 1),
                                                 "gflops": round(2.0 * m * n * N / t / 1e9, 1),
                                                 "hbm_frac": round(byts / t / HBM_PEAK, 4)}
        del A, x, y
        for s, N in ((16, 200_000), (64, 20_000)):
            A = torch.rand(N * s * s, generator=gen, device="cuda", dtype=tdt) / s
            A.view(N, s, s).diagonal(dim1=1, dim2=2).add_(2.0)
            B = torch.rand(N * s * 16, generator=gen, device="cuda", dtype=tdt) * 2 - 1
            call = lambda: sbg.trsm_strided("L", "L", "N", "N", s, 16, 1.5, A, s, s * s, B, s, s * 16, N)  # noqa: E731
            t = _time_calls(call, 7, flush)
            byts = esz * N * (s * (s + 1) // 2 + 2 * s * 16)
            out[f"trsm_{tname}_LLNN_{s}x16"] = {"N": N, "us": round(t * 1e6, 1),
                                               "gflops": round(1.0 * s * s * 16 * N / t / 1e9, 1),
                                               "hbm_frac": round(byts / t / HBM_PEAK, 4)}
            del A, B
    return out


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
