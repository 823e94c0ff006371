"""Benchmark: batched small-matrix GEMM throughput on one MI355X.

Workload ("size sweep", the paper's basic set of Sec. 8 widened to two real
types and four op pairs): N = 100,000 independent square pairs for every
n = 2..16, op in {NN, NT, TN, TT}, fp32 and fp64, alpha = 1.5, beta = -0.5,
minimal leading dimensions, entries U[-1,1].  One step = 120 batched GEMM
calls (one per dtype x n x op pair), each on its own buffers, so no call finds
its operands in a cache another call warmed (one step moves 28.7 GB).

Timed region: K steps, each one replay of a HIP graph holding the step's 120
launches, bracketed by device synchronisations (wall clock).  `value` is the
step's GFLOP/s (flops counted 2 n^3 per matrix for all alpha, beta and ops,
as in Sec. 8).

Per-launch durations (the roofline of the kernel instance that takes most of
the step's time, the per-size fractions, fp32 n = 16 per op pair) come from
HIP events on the launch stream around each of the same 120 calls launched
eagerly, queued behind a spin kernel so the events bracket kernels only.

Secondary sections (timing.py: spin-prefilled events, Infinity Cache flushed
by a read between calls): the shape of the paper's Table tab:gflop (S/D/C/Z,
n = 1..16, alpha = 1, beta = 0) with the general-epilogue comparison, the
pointer-array form against the strided one, complex op pairs, the
variable-size precision modes (error against the FP64 oracle in the CPU
leg), the FEM chain, the fixed operand, batch-size and grid-size sweeps,
tuned against default kernel choices, sizes above 16, GEMV/TRSM/LU, and a
copy kernel at equal bytes.  The CPU oracle is timed on a bounded sample.
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
# the paper's single-precision figures quoted as context (Tesla K20c, Table tab:gflop)
PAPER_K20C_SGEMM = {"n10_gflops": 104, "n16_gflops": 216}


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
    return d.get("all_kernels_traffic_bytes_per_launch", {}).get(kernel)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000,
                    help="matrices per (dtype, n, op) call timed on the CPU oracle")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", default="", help="comma-separated secondary sections to run (default: all)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed region, copy 1 GiB once (reference kernel for HBM byte counters)")
    return ap.parse_args()


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


def _med(call, reps, flush):
    """Median seconds of `call` over reps calls, each after a cache flush."""
    from paper_1304_7053_amd import timing
    call(0)
    return timing.median(timing.time_series(call, reps, flush=flush))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the batch shards across GPUs with no exchange, so run it once per GPU.", file=sys.stderr)
        sys.exit(2)

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
                         BETA, c["C"], n, n * n, N_BATCH)

    def step():
        for c in calls:
            launch(c)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    g_step = _graph(step, stream)
    print(f"bench: {len(calls)} calls per step captured", file=sys.stderr, flush=True)

    # timed region: K steps, one graph replay each
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g_step.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per-launch durations: the same calls launched eagerly behind a spin kernel
    passes = 3
    ts = timing_per_call(calls, launch, passes)

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
    for i, c in enumerate(calls):
        d = per_kernel.setdefault(c["kernel"], {"s": 0.0, "bytes": 0.0, "launches": 0})
        d["s"] += ts[i] * passes
        d["bytes"] += c["bytes"] * passes
        d["launches"] += passes
    dom_name, dom = max(per_kernel.items(), key=lambda kv: kv[1]["s"])
    dom_avg_s = dom["s"] / dom["launches"]
    dom_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_bytes / dom_avg_s / 1e9

    head = {}
    for i, c in enumerate(calls):
        if c["dt"] == "float" and c["n"] == 16:
            head[c["ops"]] = {"us": round(ts[i] * 1e6, 2), "gflops": round(c["flops"] / ts[i] / 1e9, 1),
                              "hbm_frac": round(c["bytes"] / ts[i] / HBM_PEAK, 4)}
    per_size = {}
    for i, c in enumerate(calls):
        key = f"{'s' if c['dt'] == 'float' else 'd'}{c['n']}"
        d = per_size.setdefault(key, [0.0, 0.0, 0.0])
        d[0] += c["flops"]
        d[1] += c["bytes"]
        d[2] += ts[i]
    sizes_out = {k: {"gflops": round(v[0] / v[2] / 1e9, 1), "hbm_frac": round(v[1] / v[2] / HBM_PEAK, 4)}
                 for k, v in per_size.items()}
    kernels_out = {k: {"launches": v["launches"], "mean_us": round(v["s"] / v["launches"] * 1e6, 3),
                       "hbm_frac": round(v["bytes"] / v["s"] / HBM_PEAK, 4),
                       "algorithmic_bytes_per_launch": v["bytes"] / v["launches"]} for k, v in per_kernel.items()}

    cpu_calls = calls if not args.no_cpu_baseline else None
    cpu_sample = [dict(n=c["n"], ops=c["ops"], A=c["A"][:args.cpu_sample * c["n"] ** 2].cpu(),
                       B=c["B"][:args.cpu_sample * c["n"] ** 2].cpu(), C=c["C"][:args.cpu_sample * c["n"] ** 2].cpu())
                  for c in cpu_calls] if cpu_calls else None
    del calls, g_step
    torch.cuda.empty_cache()

    secondary = None
    vs_samples = []
    if not args.no_extras:
        secondary = {}
        only = set(x for x in args.only.split(",") if x)
        sections = (("small_batch", sec_small_batch), ("tab_gflop", sec_tab_gflop),
                    ("pointer_vs_strided", sec_pointer_vs_strided), ("complex", sec_complex_sweep),
                    ("varsize_precision", lambda st: sec_varsize_modes(st, vs_samples)),
                    ("fem", sec_fem_chain), ("fixed_operand", sec_fixed_operand), ("batch_sweep", sec_batch_sweep),
                    ("grid_sweep", sec_grid_sweep), ("tuned_vs_default", sec_tuned_vs_default),
                    ("large_sizes", sec_large_sizes), ("blas_routines", sec_blas_routines),
                    ("copy_ceiling", sec_copy_ceiling))
        for name, fn in sections:
            if only and name not in only:
                continue
            t_sec = time.perf_counter()
            try:
                secondary[name] = fn(stream)
            except Exception as e:  # a secondary failure must not hide the primary line
                secondary[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
            print(f"bench: section {name} done in {time.perf_counter() - t_sec:.1f} s", file=sys.stderr, flush=True)

    cpu = None
    if cpu_sample:
        cpu = cpu_baseline(cpu_sample, args.cpu_sample, vs_samples,
                           secondary.get("varsize_precision") if secondary else None)

    ntab, tab_info = sbg.tuned_table_info()
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
                               "alpha=1.5 beta=-0.5, strided minimal-LD layout, 120 calls per step "
                               "(one HIP graph replay per step)",
                   "global_batch": N_BATCH, "parallelism": "single GPU"},
        "hbm_frac_step": round(bytes_step * args.steps / elapsed / HBM_PEAK, 4),
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved * 1e9 / HBM_PEAK, 4),
                     "traffic": stored_traffic(dom_name), "mean_launch_us": round(dom_avg_s * 1e6, 3),
                     "launches": dom["launches"], "algorithmic_bytes_per_launch": dom_bytes},
        "fp32_n16": head,
        "per_size": sizes_out,
        "per_kernel": kernels_out,
        "tuned_table": {"entries": ntab, "info": tab_info},
        "paper_context_k20c": PAPER_K20C_SGEMM,
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    if calib:
        out["calib_copy"] = calib
    print(json.dumps(out), flush=True)


def timing_per_call(calls, launch, passes):
    """Mean seconds per call over `passes` eager passes of all calls, every
    pass queued behind a spin kernel and every call bracketed by events."""
    import torch

    from paper_1304_7053_amd import timing
    stream = torch.cuda.current_stream()
    acc = [0.0] * len(calls)
    for _ in range(passes):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in calls]
        torch.cuda.synchronize()
        timing.spin(len(calls) * 300.0 + 1000.0)   # longer than enqueueing the pass, also under a tracer
        for c, (e0, e1) in zip(calls, evs):
            e0.record(stream)
            launch(c)
            e1.record(stream)
        torch.cuda.synchronize()
        for i, (e0, e1) in enumerate(evs):
            acc[i] += e0.elapsed_time(e1) / 1e3
    return [a / passes for a in acc]


# ---- secondary workloads (reported beside the primary line) ---------------

def sec_small_batch(stream):
    """N = 1000 pairs of 8x8x8, NN, alpha = 1, beta = 0 (C not read): the
    launch-latency regime.  Median of an eager call as a Python caller sees it
    (host launch included), of the kernel alone, and of a graph replay."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    N, s = 1000, 8
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 1)
    A = torch.rand(N * s * s, generator=gen, device="cuda") * 2 - 1
    B = torch.rand(N * s * s, generator=gen, device="cuda") * 2 - 1
    C = torch.empty(N * s * s, device="cuda")
    call = lambda *_: sbg.gemm_strided("N", "N", s, s, s, 1.0, A, s, s * s, B, s, s * s, 0.0, C, s, s * s, N)  # noqa
    ts = []
    for _ in range(200):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    ts.sort()
    kern = timing.median(timing.time_series(call, 50)) * 1e6
    g = _graph(call, stream)
    tg = timing.median(timing.time_series(lambda i: g.replay(), 50)) * 1e6
    return {"workload": "N=1000, 8x8x8, NN, alpha=1, beta=0, fp32", "us_per_eager_call_median": round(ts[100], 2),
            "us_kernel_median": round(kern, 2), "us_per_graph_replay_median": round(tg, 2),
            "gflops_kernel": round(2 * s ** 3 * N / (kern * 1e-6) / 1e9, 1),
            "kernel": sbg.describe_strided("s", "N", "N", s, s, s, s, s * s, s, s * s, s, s * s, N)}


def _rand(gen, n, tdt):
    import torch
    if tdt.is_complex:
        rdt = torch.float32 if tdt == torch.complex64 else torch.float64
        return (torch.rand(2 * n, generator=gen, device="cuda", dtype=rdt) * 2 - 1).view(tdt)
    return torch.rand(n, generator=gen, device="cuda", dtype=tdt) * 2 - 1



def _types():
    import torch
    return (("s", torch.float32, 4, 1.5, -0.5), ("d", torch.float64, 8, 1.5, -0.5),
            ("c", torch.complex64, 8, complex(1, 0.5), complex(0.25, -1)),
            ("z", torch.complex128, 16, complex(1, 0.5), complex(0.25, -1)))


def sec_tab_gflop(stream):
    """The shape of the paper's Table tab:gflop: every square size 1..16 for
    S, D, C and Z, N = 100,000, NN, alpha = 1, beta = 0 (a1b0: C written, not
    read), GFLOP/s (2 n^3 real, 8 n^3 complex) and HBM fraction (3 n^2 elements
    per matrix); beside it the general epilogue (alpha, beta != 0: C read too,
    4 n^2 elements) -- the paper's a1b0-vs-general comparison."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    N = N_BATCH
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 10)
    out = {}
    for p, tdt, esz, al, be in _types():
        row = {}
        for n in range(1, 17):
            el = N * n * n
            A, B, C = _rand(gen, el, tdt), _rand(gen, el, tdt), _rand(gen, el, tdt)
            fl = (8.0 if tdt.is_complex else 2.0) * n ** 3 * N
            res = {}
            for case, a_, b_, nbytes in (("a1b0", 1.0, 0.0, 3.0), ("general", al, be, 4.0)):
                t = _med(lambda i: sbg.gemm_strided("N", "N", n, n, n, a_, A, n, n * n, B, n, n * n, b_, C, n,
                                                    n * n, N), 5, flush)
                res[case] = (t, fl / t / 1e9, nbytes * n * n * esz * N / t / HBM_PEAK)
            row[str(n)] = {"a1b0_gflops": round(res["a1b0"][1], 1), "a1b0_hbm_frac": round(res["a1b0"][2], 4),
                           "general_gflops": round(res["general"][1], 1),
                           "general_hbm_frac": round(res["general"][2], 4),
                           "general_over_a1b0_time": round(res["general"][0] / res["a1b0"][0], 3)}
            del A, B, C
        out[p] = row
    return out


def sec_pointer_vs_strided(stream):
    """The pointer-array form against the strided form (the paper's nounif
    vs unif interfaces), fp32 and fp64, N = 100,000, square n = 2..16, NN,
    alpha = 1.5, beta = -0.5.  HBM fraction of the pointer form counts its
    three 8-byte pointers per matrix."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    N = N_BATCH
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 11)
    out = {}
    for p, tdt, esz, al, be in _types()[:2]:
        row = {}
        for n in range(2, 17):
            el = N * n * n
            A, B, C = _rand(gen, el, tdt), _rand(gen, el, tdt), _rand(gen, el, tdt)
            ptr = [torch.arange(N, device="cuda", dtype=torch.int64) * (n * n * esz) + x.data_ptr() for x in (A, B, C)]
            ts = _med(lambda i: sbg.gemm_strided("N", "N", n, n, n, al, A, n, n * n, B, n, n * n, be, C, n, n * n, N),
                      5, flush)
            tp = _med(lambda i: sbg.gemm_batched("N", "N", n, n, n, al, ptr[0], n, ptr[1], n, be, ptr[2], n, N, tdt),
                      5, flush)
            byts = 4.0 * n * n * esz * N
            row[str(n)] = {"strided_hbm_frac": round(byts / ts / HBM_PEAK, 4),
                           "pointer_hbm_frac": round((byts + 24.0 * N) / tp / HBM_PEAK, 4),
                           "pointer_over_strided_time": round(tp / ts, 3)}
            del A, B, C, ptr
        out[p] = row
    return out


def sec_complex_sweep(stream):
    """N = 100,000 complex pairs, n in {4, 8, 12, 16}, all nine op pairs over
    {N, T, C}, alpha = (1, 0.5), beta = (0.25, -1); GFLOP/s (8 n^3 per
    matrix) and HBM fraction per (type, n), each call on its own buffers."""
    import torch

    from paper_1304_7053_amd import sbg
    N = N_BATCH
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 3)
    out = {}
    ops = [a + b for a in "NTC" for b in "NTC"]
    for p, tdt, esz, al, be in _types()[2:]:
        for n in (4, 8, 12, 16):
            el = N * n * n
            bufs = [[_rand(gen, el, tdt) for _ in range(3)] for _ in range(9)]
            calls = [(op, bufs[i]) for i, op in enumerate(ops)]

            def launch(c):
                op, (A, B, C) = c
                sbg.gemm_strided(op[0], op[1], n, n, n, al, A, n, n * n, B, n, n * n, be, C, n, n * n, N)
            for c in calls:
                launch(c)
            ts = timing_per_call(calls, launch, 3)
            tmed = {op: ts[i] for i, op in enumerate(ops)}
            tot = sum(tmed.values())
            out[f"{p}{n}"] = {"gflops": round(8.0 * n ** 3 * N * 9 / tot / 1e9, 1),
                              "hbm_frac": round(4.0 * n * n * esz * N * 9 / tot / HBM_PEAK, 4),
                              "op_vs_NN": {op: round(tmed["NN"] / t, 3) for op, t in tmed.items()}}
            del bufs, calls
            torch.cuda.empty_cache()
    return out


def _varsize_sample(m, n, k, count, g):
    """About `count` matrix indices spread over the three size classes, with
    the first and last matrix of the batch."""
    import numpy as np
    mx = np.maximum(np.maximum(m, n), k)
    cls = np.where(mx <= 4, 0, np.where(mx <= 8, 1, 2))
    idx = [0, len(m) - 1]
    for c in range(3):
        sel = np.nonzero(cls == c)[0]
        if len(sel):
            idx.extend(g.choice(sel, size=min(len(sel), count // 3), replace=False).tolist())
    return np.unique(np.array(idx, dtype=np.int64))


def _gather(flat_host, offs, counts, idx):
    """Compact host copy of matrices idx of a flat packed buffer."""
    import numpy as np
    parts = [flat_host[offs[p]:offs[p] + counts[p]] for p in idx]
    new_off = np.zeros(len(idx), dtype=np.int64)
    if len(idx) > 1:
        new_off[1:] = np.cumsum([len(x) for x in parts])[:-1]
    return (np.concatenate(parts) if parts else flat_host[:0]), new_off


def sec_varsize_modes(stream, samples):
    """N = 200,000 matrices with m, n, k drawn independently (40% at 8, 30% at
    16, the rest uniform), pointer arrays, one variable-size call (binning +
    persistent GEMM) captured in a HIP graph; for each precision mode and
    both input sets: GFLOP/s and HBM fraction (algorithmic bytes incl.
    per-matrix pointers, sizes, leading dimensions and scales), each replay
    after a cache flush.  A stratified sample of about 2,000 matrices (with the
    first and last) is copied to the host for the error report against the
    FP64 oracle, computed in the CPU leg."""
    import numpy as np
    import torch

    from paper_1304_7053_amd import inputs, sbg, timing
    N = 200_000
    g = inputs.rng(4)
    m, n, k = inputs.varsize_dims(g, N)
    m64, n64, k64 = (x.astype(np.int64) for x in (m, n, k))
    offs = {}
    for name, cnt in (("A", m64 * k64), ("B", k64 * n64), ("C", m64 * n64)):
        o = np.zeros(N, dtype=np.int64)
        o[1:] = np.cumsum(cnt)[:-1]
        offs[name] = (o, int(cnt.sum()), cnt)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    dm, dn, dk = dev(m), dev(n), dev(k)
    dlda, dldb, dldc = dev(np.maximum(m, 1)), dev(np.maximum(k, 1)), dev(np.maximum(m, 1))
    ws = torch.zeros(sbg.vbatched_workspace_size(N) // 4 + 1, dtype=torch.int32, device="cuda")
    flush = timing.Flusher()
    flops = float(np.sum(2 * m64 * n64 * k64))
    meta = 24 + 24                          # three pointers, six int32 sizes / leading dimensions
    idx = _varsize_sample(m, n, k, 2000, inputs.rng(4, salt=77))
    res = {"workload": "N=200000 variable m,n,k (40% 8, 30% 16, rest uniform), NN, alpha=1.5, beta=-0.5",
           "gflop_per_call": round(flops / 1e9, 4), "error_sample_matrices": int(len(idx))}
    for dist in ("uniform", "logu"):
        A32h = inputs.DISTS[dist](g, (offs["A"][1],), np.float32)
        B32h = inputs.DISTS[dist](g, (offs["B"][1],), np.float32)
        C0h = inputs.DISTS[dist](g, (offs["C"][1],), np.float32)
        A32, B32, C0 = dev(A32h), dev(B32h), dev(C0h)
        C = torch.empty_like(C0)
        pC = torch.tensor(C.data_ptr() + offs["C"][0] * 4, device="cuda")
        sA_, oA = _gather(A32h, offs["A"][0], offs["A"][2], idx)
        sB_, oB = _gather(B32h, offs["B"][0], offs["B"][2], idx)
        sC_, oC = _gather(C0h, offs["C"][0], offs["C"][2], idx)
        results = {}
        for mode in ("f32", "bf16", "f16", "e4m3", "bf16x3"):
            sA = sB = None
            qtime = None
            stored = None
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
                qtime = _med(lambda i: qg.replay(), 5, flush)
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
            gr.replay()                      # one clean replay for the error sample
            torch.cuda.synchronize()
            out_s, _ = _gather(C.cpu().numpy(), offs["C"][0], offs["C"][2], idx)
            if mode in ("bf16", "f16"):
                stA, _ = _gather(Ain.view(torch.int16).cpu().numpy().view(np.uint16), offs["A"][0], offs["A"][2], idx)
                stB, _ = _gather(Bin.view(torch.int16).cpu().numpy().view(np.uint16), offs["B"][0], offs["B"][2], idx)
                stored = (stA, stB, None, None)
            elif mode == "e4m3":
                stA, _ = _gather(Ain.cpu().numpy(), offs["A"][0], offs["A"][2], idx)
                stB, _ = _gather(Bin.cpu().numpy(), offs["B"][0], offs["B"][2], idx)
                stored = (stA, stB, sA.cpu().numpy()[idx].astype(np.float64), sB.cpu().numpy()[idx].astype(np.float64))
            samples.append(dict(dist=dist, mode=mode, m=m[idx], n=n[idx], k=k[idx], A=sA_, oA=oA, B=sB_, oB=oB,
                                C=sC_, oC=oC, out=out_s, stored=stored))
            med = _med(lambda i: gr.replay(), 7, flush)
            byts = float(np.sum((m64 * k64 + k64 * n64) * esz + 2 * m64 * n64 * 4)) + N * meta + \
                (8 * N if mode == "e4m3" else 0)
            plan = sbg.describe_vbatched("s", "N", "N", 16, 16, 16, N, code, cmode)
            results[mode] = {"us": round(med * 1e6, 1), "gflops": round(flops / med / 1e9, 1),
                             "hbm_frac": round(byts / med / HBM_PEAK, 4), "algorithmic_bytes": byts,
                             "kernel": plan["kernel"] if plan else None}
            if qtime is not None:
                results[mode]["quantize_us"] = round(qtime * 1e6, 1)
            del gr
        for mode in results:
            results[mode]["time_vs_f32"] = round(results[mode]["us"] / results["f32"]["us"], 3)
        res[dist] = results
        del A32, B32, C0, C
        torch.cuda.empty_cache()
    return res


def sec_fem_chain(stream):
    """N = 1,000,000 FEM elements: K = B^T (D B) (two batched GEMMs) and its
    backward from dK (four), each sequence captured as one HIP graph."""
    import torch

    from paper_1304_7053_amd import inputs, timing
    from paper_1304_7053_amd.autograd import gemm_rm
    N = 1_000_000
    g = inputs.rng(5)
    B, D, dK = (torch.from_numpy(x).cuda() for x in inputs.fem_element_batch(g, N))
    T = torch.empty((N, 6, 12), device="cuda")
    K = torch.empty((N, 12, 12), device="cuda")
    dT = torch.empty_like(T)
    dB = torch.empty_like(B)
    dD = torch.empty_like(D)
    flush = timing.Flusher()

    def fwd():
        gemm_rm("N", "N", 1.0, D, B, 0.0, T)
        gemm_rm("T", "N", 1.0, B, T, 0.0, K)

    def bwd():
        gemm_rm("N", "N", 1.0, B, dK, 0.0, dT)
        gemm_rm("N", "T", 1.0, T, dK, 0.0, dB)
        gemm_rm("T", "N", 1.0, D, dT, 1.0, dB)
        gemm_rm("N", "T", 1.0, dT, B, 0.0, dD)
    gf, gb = _graph(fwd, stream), _graph(bwd, stream)
    tf = _med(lambda i: gf.replay(), 7, flush)
    tb = _med(lambda i: gb.replay(), 7, flush)
    ffl, bfl = 2592.0 * N, 5184.0 * N
    fby, bby = 1872.0 * N, 4032.0 * N
    return {"workload": "N=1e6 elements, B 6x12, D 6x6, fp32",
            "forward": {"us": round(tf * 1e6, 1), "gflops": round(ffl / tf / 1e9, 1),
                        "hbm_frac": round(fby / tf / HBM_PEAK, 4)},
            "backward": {"us": round(tb * 1e6, 1), "gflops": round(bfl / tb / 1e9, 1),
                         "hbm_frac": round(bby / tb / HBM_PEAK, 4)}}


def sec_fixed_operand(stream):
    """The fixed-operand case the paper names as a next step (Sec. 9): one A
    (strideA = 0) or one B (strideB = 0) shared by the whole batch, against
    the ordinary batch; N = 100,000, NN, alpha = 1.5, beta = -0.5.  The HBM
    fraction counts the shared matrix once."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    N = N_BATCH
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 6)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        for n in (8, 16):
            el = N * n * n
            A, B, C = _rand(gen, el, tdt), _rand(gen, el, tdt), _rand(gen, el, tdt)
            res = {}
            for case, sa, sb in (("batched", n * n, n * n), ("shared_A", 0, n * n), ("shared_B", n * n, 0)):
                t = _med(lambda i: sbg.gemm_strided("N", "N", n, n, n, 1.5, A, n, sa, B, n, sb, -0.5, C, n, n * n, N),
                         7, flush)
                byts = esz * n * n * (N * (2 + (sa > 0) + (sb > 0)) + (sa == 0) + (sb == 0))
                res[case] = {"us": round(t * 1e6, 1), "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                             "hbm_frac": round(byts / t / HBM_PEAK, 4)}
            res["kernel_shared_A"] = sbg.describe_strided("s" if esz == 4 else "d", "N", "N", n, n, n, n, 0, n,
                                                          n * n, n, n * n, N)
            out[f"{tname}_n{n}"] = res
            del A, B, C
    return out


def sec_batch_sweep(stream):
    """Batch-size sweep (the paper's plateau question, Sec. 8): fp32 NN,
    alpha = 1.5, beta = -0.5, n in {8, 16}, N from 2,000 to 1,000,000."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 7)
    out = {}
    for n in (8, 16):
        row = {}
        for N in (2000, 5000, 20000, 100_000, 1_000_000):
            el = N * n * n
            A, B, C = (_rand(gen, el, torch.float32) for _ in range(3))
            t = _med(lambda i: sbg.gemm_strided("N", "N", n, n, n, 1.5, A, n, n * n, B, n, n * n, -0.5, C, n, n * n,
                                                N), 7, flush)
            row[str(N)] = {"us": round(t * 1e6, 2), "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                           "hbm_frac": round(16.0 * n * n * N / t / HBM_PEAK, 4)}
            del A, B, C
        out[f"f32_n{n}"] = row
    return out


def sec_grid_sweep(stream):
    """Launch-shape sweep (the paper's block-count study, Sec. 7-8): the
    persistent MFMA tile kernel at fixed work -- fp32 n = 8 and 16, fp64
    n = 16, N = 100,000, NN -- with the number of work-groups varied."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 12)
    out = {}
    N = N_BATCH
    for p, tdt, esz, n in (("s", torch.float32, 4, 8), ("s", torch.float32, 4, 16), ("d", torch.float64, 8, 16)):
        el = N * n * n
        A, B, C = (_rand(gen, el, tdt) for _ in range(3))
        row = {}
        for grid in (32, 64, 128, 256, 512, 1024, 2048, 4096, 8192):
            with sbg.tuned(path=1, staged=0, grid=grid, table=0):
                t = _med(lambda i: sbg.gemm_strided("N", "N", n, n, n, 1.5, A, n, n * n, B, n, n * n, -0.5, C, n,
                                                    n * n, N), 5, flush)
            row[str(grid)] = {"us": round(t * 1e6, 2), "hbm_frac": round(4.0 * esz * el / t / HBM_PEAK, 4)}
        out[f"{p}{n}"] = row
        del A, B, C
    return out


def sec_tuned_vs_default(stream):
    """Each size of the fp32 / fp64 NN sweep with the tuned table and with the
    built-in rules (table off), same buffers, cache flushed between calls."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 13)
    N = N_BATCH
    out = {}
    for p, tdt, esz, al, be in _types()[:2]:
        row = {}
        for n in range(2, 17):
            el = N * n * n
            A, B, C = (_rand(gen, el, tdt) for _ in range(3))
            f = lambda i: sbg.gemm_strided("N", "N", n, n, n, al, A, n, n * n, B, n, n * n, be, C, n, n * n, N)  # noqa
            tt = _med(f, 5, flush)
            with sbg.tuned(table=0):
                td = _med(f, 5, flush)
            byts = 4.0 * esz * el
            row[str(n)] = {"tuned_hbm_frac": round(byts / tt / HBM_PEAK, 4),
                           "default_hbm_frac": round(byts / td / HBM_PEAK, 4), "speedup": round(td / tt, 3)}
            del A, B, C
        out[p] = row
    return out


def sec_large_sizes(stream):
    """Sizes above 16 (the sub-blocked kernel, the paper's extension remark):
    square n in {24, 32, 48, 64}, NN and TN, alpha = 1.5, beta = -0.5, with
    about 400 MB per fp32 operand (800 MB fp64).  HBM fraction counts A, B
    and C read once and C written once."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 8)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        for n in (24, 32, 48, 64):
            N = 100_000_000 // (n * n)
            el = N * n * n
            A, B, C = (_rand(gen, el, tdt) for _ in range(3))
            for ops in ("NN", "TN"):
                t = _med(lambda i: sbg.gemm_strided(ops[0], ops[1], n, n, n, 1.5, A, n, n * n, B, n, n * n, -0.5, C,
                                                    n, n * n, N), 5, flush)
                out[f"{tname}_n{n}_{ops}"] = {"N": N, "us": round(t * 1e6, 1),
                                               "gflops": round(2.0 * n ** 3 * N / t / 1e9, 1),
                                               "hbm_frac": round(4.0 * esz * el / t / HBM_PEAK, 4),
                                               "algorithmic_bytes": 4.0 * esz * el,
                                               "kernel": sbg.describe_strided("s" if esz == 4 else "d", ops[0],
                                                                              ops[1], n, n, n, n, n * n, n, n * n,
                                                                              n, n * n, N)}
            del A, B, C
    return out


def sec_blas_routines(stream):
    """Batched GEMV, TRSM and LU in the strided interface (formulated on
    batched GEMM, the paper's outlook): GEMV y = 1.5 op(A) x - 0.5 y with A
    16 x 16, N = 10^6, ops N and T; TRSM op(A) X = 1.5 B with A 16 x 16 lower,
    16 right-hand sides, N = 200,000, and a blocked order-64 case (N =
    20,000); LU with partial pivoting of order 4, 8, 16 (N = 100,000) and 32
    (N = 50,000).  HBM bytes: GEMV A + x + y read + y written; TRSM the
    triangle of A + B read + B written; LU A read and written plus the
    interchanges and info."""
    import torch

    from paper_1304_7053_amd import sbg, timing
    flush = timing.Flusher()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13047053 + 9)
    out = {}
    for tname, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        N, m, n = 1_000_000, 16, 16
        A = _rand(gen, N * m * n, tdt)
        x = _rand(gen, N * n, tdt)
        y = _rand(gen, N * m, tdt)
        for trans in "NT":
            t = _med(lambda i: sbg.gemv_strided(trans, m, n, 1.5, A, m, m * n, x, 1, n, -0.5, y, 1, m, N), 7, flush)
            byts = esz * N * (m * n + n + 2 * m)
            out[f"gemv_{tname}_16x16_{trans}"] = {"N": N, "us": round(t * 1e6, 1),
                                                 "gflops": round(2.0 * m * n * N / t / 1e9, 1),
                                                 "hbm_frac": round(byts / t / HBM_PEAK, 4)}
        del A, x, y
        for s, N in ((16, 200_000), (64, 20_000)):
            A = torch.rand(N * s * s, generator=gen, device="cuda", dtype=tdt) / s
            A.view(N, s, s).diagonal(dim1=1, dim2=2).add_(2.0)
            B = _rand(gen, N * s * 16, tdt)
            t = _med(lambda i: sbg.trsm_strided("L", "L", "N", "N", s, 16, 1.5, A, s, s * s, B, s, s * 16, N), 7,
                     flush)
            byts = esz * N * (s * (s + 1) // 2 + 2 * s * 16)
            out[f"trsm_{tname}_LLNN_{s}x16"] = {"N": N, "us": round(t * 1e6, 1),
                                               "gflops": round(1.0 * s * s * 16 * N / t / 1e9, 1),
                                               "hbm_frac": round(byts / t / HBM_PEAK, 4)}
            del A, B
        # LU with partial pivoting, in place (repeated factorisations of the
        # factors time the same work); flops 2 n^3 / 3 per matrix
        for s, N in ((4, 100_000), (8, 100_000), (16, 100_000), (32, 50_000)):
            A = _rand(gen, N * s * s, tdt)
            ipiv = torch.empty(N * s, dtype=torch.int32, device="cuda")
            info = torch.empty(N, dtype=torch.int32, device="cuda")
            t = _med(lambda i: sbg.getrf_strided(s, A, s, s * s, ipiv, s, info, N), 7, flush)
            byts = N * (2 * s * s * esz + 4 * s + 4)
            out[f"getrf_{tname}_{s}"] = {"N": N, "us": round(t * 1e6, 1),
                                         "gflops": round(2.0 * s ** 3 / 3 * N / t / 1e9, 1),
                                         "hbm_frac": round(byts / t / HBM_PEAK, 4)}
            del A, ipiv, info
    return out


def sec_copy_ceiling(stream):
    """A plain device copy (torch) moving the algorithmic bytes of three
    size-sweep calls -- fp32 n = 5 and 16, fp64 n = 16 (N = 100,000, general
    alpha, beta: 4 n^2 elements per matrix, half read and half written here) --
    as the achievable-bandwidth reference beside the GEMM kernels."""
    import torch

    from paper_1304_7053_amd import timing
    flush = timing.Flusher()
    out = {}
    for name, esz, n in (("s5", 4, 5), ("s16", 4, 16), ("d16", 8, 16)):
        nbytes = 4 * n * n * esz * N_BATCH
        src = torch.ones(nbytes // 8, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        t = _med(lambda i: dst.copy_(src), 7, flush)
        out[name] = {"bytes": nbytes, "us": round(t * 1e6, 2), "hbm_frac": round(nbytes / t / HBM_PEAK, 4)}
        del src, dst
    return out


def cpu_baseline(sample_calls, sample, vs_samples, vs_section):
    """The CPU leg: the oracle (FP64 accumulation, OpenMP over the batch) on
    `sample` matrices of every call of one step, on all host threads and on
    one; and the FP64-oracle errors of the variable-size precision modes on
    their sampled matrices, written into that section."""
    import numpy as np

    import oracle

    threads = oracle.max_threads()
    flops = 0.0
    t_total = 0.0
    for c in sample_calls:
        n = c["n"]
        A, B, C = c["A"].numpy(), c["B"].numpy(), c["C"].numpy()
        t0 = time.perf_counter()
        oracle.gemm_strided(c["ops"][0], c["ops"][1], n, n, n, ALPHA, A, n, n * n, B, n, n * n, BETA, C, n,
                            n * n, sample)
        t_total += time.perf_counter() - t0
        flops += 2.0 * n ** 3 * sample
    # one thread, on a tenth of the sample
    s1 = max(1, sample // 10)
    oracle.set_threads(1)
    f1 = 0.0
    t1 = 0.0
    for c in sample_calls:
        n = c["n"]
        t0 = time.perf_counter()
        oracle.gemm_strided(c["ops"][0], c["ops"][1], n, n, n, ALPHA, c["A"].numpy(), n, n * n, c["B"].numpy(), n,
                            n * n, BETA, c["C"].numpy(), n, n * n, s1)
        t1 += time.perf_counter() - t0
        f1 += 2.0 * n ** 3 * s1
    oracle.set_threads(threads)
    if vs_section is not None and vs_samples:
        for s in vs_samples:
            cnt = len(s["m"])
            lda, ldb, ldc = np.maximum(s["m"], 1), np.maximum(s["k"], 1), np.maximum(s["m"], 1)
            # end to end: the oracle on the binary32 inputs (quantisation included)
            args = ("N", "N", s["m"], s["n"], s["k"], 1.5, s["A"], s["oA"], lda, s["B"], s["oB"], ldb, -0.5, s["C"],
                    s["oC"], ldc, cnt)
            hi, lo, offO, mm, nn = oracle.gemm_general(*args, ext=True)
            bnd, _ = oracle.bound_general(*args)
            e2e = _max_norm_err(s, hi, lo, bnd, offO, mm, nn)
            # kernel only: the oracle on the operands as stored (decoded, scaled)
            kmax = np.maximum(s["k"], 1).astype(np.float64)
            if s["mode"] == "bf16x3":
                hk, lk, bk, offK, mk, nk = oracle.gemm_split3_general(*args)
                kern = _max_norm_err(s, hk, lk, bk, offK, mk, nk, per_matrix_scale=1.0 / (3 * 4 * kmax * 2.0 ** -24))
            elif s["stored"] is None:
                kern = _max_norm_err(s, hi, lo, bnd, offO, mm, nn, per_matrix_scale=1.0 / (4 * kmax * 2.0 ** -24))
            else:
                stA, stB, scA, scB = s["stored"]
                types = {"bf16": ("bf16", "bf16", "f32"), "f16": ("f16", "f16", "f32"),
                         "e4m3": ("e4m3", "e4m3", "f32")}[s["mode"]]
                kargs = ("N", "N", s["m"], s["n"], s["k"], 1.5, stA, s["oA"], lda, stB, s["oB"], ldb, -0.5, s["C"],
                         s["oC"], ldc, cnt)
                hk, lk, offK, mk, nk = oracle.gemm_general(*kargs, ext=True, types=types, scaleA=scA, scaleB=scB)
                bk, _ = oracle.bound_general(*kargs, types=types, scaleA=scA, scaleB=scB)
                kern = _max_norm_err(s, hk, lk, bk, offK, mk, nk, per_matrix_scale=1.0 / (4 * kmax * 2.0 ** -24))
            d = vs_section.get(s["dist"], {}).get(s["mode"])
            if d is not None:
                d["max_err_vs_fp64_oracle"] = e2e
                d["kernel_err_over_bound"] = kern
    return {"value": round(flops / t_total / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} matrices of each of the 120 calls of one step "
                      f"({flops / 1e9:.2f} GFLOP, {t_total:.1f} s)",
            "single_thread": {"value": round(f1 / t1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"{s1} matrices of each call ({f1 / 1e9:.3f} GFLOP, {t1:.1f} s)"}}


def _max_norm_err(s, hi, lo, bnd, offO, mm, nn, per_matrix_scale=None):
    """Largest |C - Cref| / (|alpha| |A||B| + |beta| |C_in|) over the sampled
    matrices (entries with a zero denominator must be exact); scaled per
    matrix when per_matrix_scale is given (e.g. by 1 / (4 k u))."""
    import numpy as np
    worst = 0.0
    bstart = np.concatenate([[0], np.cumsum(mm.astype(np.int64) * nn)])
    for q in range(len(mm)):
        m, n = int(mm[q]), int(nn[q])
        if m == 0 or n == 0:
            continue
        o = int(offO[q])
        got = s["out"][s["oC"][q]:s["oC"][q] + m * n].astype(np.float64)
        diff = np.abs((got - hi[o:o + m * n]) - lo[o:o + m * n])
        b = bnd[bstart[q]:bstart[q] + m * n]
        with np.errstate(divide="ignore", invalid="ignore"):
            e = np.where(b > 0, diff / np.where(b > 0, b, 1.0), np.where(diff == 0, 0.0, np.inf))
        w = float(np.max(e))
        if per_matrix_scale is not None:
            w *= float(per_matrix_scale[q])
        worst = max(worst, w)
    return worst


if __name__ == "__main__":
    main()
