"""Throughput benchmark of the compact fourth-order Yee stepper on one MI355X.

Default workload (--workload batch): 512 independent 2D TM PEC cavities,
N ~ U{64..768} (seed 2306), modes (k, l) ~ U{1..8}^2, amplitude U(0.5, 2),
CFL 0.5, FP64, PAPER closure with the carried Laplacian, advanced together
by the batched form; one bench step is one time step (Step 1 + Step 2) of
every member, and the default K = 200 steps is the workload's run length.
About 3.5 GB of state: HBM-resident (the 256 MB Infinity Cache holds a
small part).  The fields are resident in HBM before the timed region.

Prints ONE JSON line with the metric, the roofline block of the dominant
kernel (every launch of the timed region bracketed by HIP events on the
batch's stream) and the CPU baseline (the oracle on the host cores over a
bounded sample of the same workload).  Other workloads: the single N = 2048
cavity (2d), the refinement sweep (sweep), the 3D cube (3d), serving.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline; p50/p99 latency"
CLOSURES_O = {"paper": 0, "reflect": 1}
LAPS_O = {"tracked": 0, "discrete": 1}
# kernels of each class in the batched strip form (one launch per stage)
BATCH_KERNELS = {
    ("rhs_e", True): "k_batch_stage<K, T, 0> (Step 1 x-line tiles: raw x-derivatives, T0 on the end-band columns; band-table rows)",
    ("solve_e", True): "k_batch_stage<K, T, 1> (Step 1 wave strips: y-lines, T0, Chebyshev solve, Ez and G_E update)",
    ("rhs_h", True): "k_batch_xstage<T, 2> (Step 2 x-line tiles of G_E; band-table rows; one workgroup per item)",
    ("solve_h", True): "k_batch_stage<K, T, 3> (Step 2 Hx and Hy wave strips: solves and updates)",
    ("step", False): "k_batch_step<K, T> (the whole step: all four stages, per-problem stage counters)",
}


# sources each workload's kernels are built from (a change elsewhere does
# not void its counter results)
KERNEL_SOURCES = {
    "2d": ["c4m_internal.h", "c4m_tiles_2d.h", "c4m_stream_2d.h", "c4m_kernels_2d.hip", "c4m_host.hip"],
    "batch": ["c4m_internal.h", "c4m_tiles_2d.h", "c4m_stream_2d.h", "c4m_batch.hip"],
    "3d": ["c4m_internal.h", "c4m_kernels_3d.hip", "c4m_host.hip"],
}


def kernel_source_hash(workload: str = "2d") -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_17263_amd", "csrc")
    for name in sorted(KERNEL_SOURCES.get(workload.split("_")[0], os.listdir(csrc))):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash(workload):
        return None
    return ent.get("bytes_per_launch")


COPY_PROBE_BYTES = 256 << 20
# kernel-class -> kernel-name pattern of the 2D path (rocprofv3 names)
CLASS_PATTERNS = {
    "rhs_e": r"k_xlines<[01][,>]",
    "solve_e": r"k_(?:strip|col)<\d+, [01],",
    "rhs_h": r"k_xlines<[23][,>]",
    "solve_h": r"k_(?:strip_h|strip|col)<\d+, [234],",
}
# kernels of each class in the default single-problem form
CLASS_KERNELS = {
    "rhs_e": "k_xlines<0|1, true> (Step 1 raw x-line derivatives, T0 on the end-band columns, and the band table of the Hx y-lines)",
    "solve_e": "k_strip<K, 0|1> (Step 1 y-lines, T0 from the raw x-line derivatives, Chebyshev solve, Ez and G_E update)",
    "rhs_h": "k_xlines<2|3, false> (Step 2 x-lines and the band table of the G_E y-lines)",
    "solve_h": "k_strip_h<K, 2|3> (Step 2 Hx and Hy solves and updates, one launch)",
}


# 3D kernel classes: the Pade line terms of each half-step and the
# Chebyshev passes of both (the same kernels), per component launch group
# (every line term reads a raw source in both half-steps, so the counters
# attribute the right-hand sides of Step 1 and Step 2 together)
CLASS_PATTERNS_3D = {
    "rhs": r"k_term3<|k_march3<|k_condition3<",
    "solve": r"k_cheb3t<",
}
KERNELS_3D = {
    "rhs": "k_condition3 (conditioned sources, once per half-step), k_term3<0, raw> (x-line terms) and "
           "k_march3<1|2, raw> (y/z-line terms): 4 terms per E component, 2 per H",
    "solve": "k_cheb3t<...> (one application of M in the three-term Chebyshev recurrence; K per component, "
             "the last writes the field and G_E updates)",
}
# component launch groups per step of each 3D class (the rhs figure is the
# mean over the three Step 1 and three Step 2 groups)
CALLS_3D = {"rhs": 6, "solve": 6}

# kernel-class -> kernel-name pattern of the batched form (strip stage
# launches, the single launch per step, the column-tile form)
BATCH_CLASS_PATTERNS = {
    "rhs_e": r"k_batch_stage<\d+, (?:true|false), 0>|k_batch_xstage<(?:true|false), 0>|k_batch_x<[01]>",
    "solve_e": r"k_batch_stage<\d+, (?:true|false), 1>|k_batch_col<\d+, [01],",
    "rhs_h": r"k_batch_stage<\d+, (?:true|false), 2>|k_batch_xstage<(?:true|false), 2>|k_batch_x<[23]>",
    "solve_h": r"k_batch_stage<\d+, (?:true|false), 3>|k_batch_col<\d+, [234],",
    "step": r"k_batch_step<",
}


def traffic_key(n, args):
    if getattr(args, "workload", "2d") == "3d":
        n3 = args.n if args.n != 2048 else 256
        return f"3d_n{n3}_{args.closure}_{args.lap}_{args.precision}_{args.solver}"
    if getattr(args, "workload", "2d") == "batch":
        return f"batch_{args.count}_{args.closure}_{args.lap}_{args.precision}"
    return f"2d_n{n}_{args.closure}_{args.lap}_{args.precision}_{args.solver}"


def pmc_probe(args):
    """A plain elementwise copy of COPY_PROBE_BYTES (reads and writes that
    many bytes), then a few steps of the 2D workload, each on a dedicated
    stream; run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE)."""
    import torch
    from paper_2306_17263_amd import Problem
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
    st.synchronize()
    if args.workload == "3d":
        from workloads import mode_fields
        n = args.n if args.n != 2048 else 256
        init = mode_fields(3, n, (2, 3, 4), 0.0, 0.2 / n)
        prob = Problem(3, n, 0.4, closure=args.closure, lap_mode=args.lap, precision=args.precision,
                       solver=args.solver, stream=st)
        for name in prob.fields():
            prob.set(name, init[name])
        st.synchronize()
        prob.step(args.steps or 2)
        st.synchronize()
        prob.close()
        print(json.dumps({"pmc_probe": f"3d_n{n}", "copy_bytes": COPY_PROBE_BYTES}), flush=True)
        return
    if args.workload == "batch":
        from paper_2306_17263_amd import Batch
        from workloads import batch_mix, mode_fields
        specs = batch_mix(count=args.count)
        b = Batch(specs, stream=st, closure=args.closure, lap_mode=args.lap, precision=args.precision)
        for p, sp in zip(b.problems, specs):
            init = mode_fields(2, sp["n"], sp["k"], 0.0, sp["r"] / sp["n"] / 2, amp=sp["amp"])
            for name in p.fields():
                p.set(name, init[name])
        b.step(args.steps or 4)
        st.synchronize()
        b.close()
        print(json.dumps({"pmc_probe": traffic_key(0, args), "copy_bytes": COPY_PROBE_BYTES}), flush=True)
        return
    n = args.n
    k = tuple(int(v) for v in args.mode.split(","))
    ht = args.cfl / n
    init = exact_fields(n, k, 0.0, ht / 2)
    prob = Problem(2, n, args.cfl, closure=args.closure, lap_mode=args.lap, precision=args.precision, stream=st)
    for name in prob.fields():
        prob.set(name, init[name])
    prob.step(args.steps or 4)
    st.synchronize()
    prob.close()
    print(json.dumps({"pmc_probe": traffic_key(n, args), "copy_bytes": COPY_PROBE_BYTES}), flush=True)


def _counter_means(folder):
    """Mean counter value per kernel name from a rocprofv3 --pmc CSV."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    acc = {}
    with open(files[0]) as f:
        for row in csv.DictReader(f):
            key = row.get("Kernel_Name", "")
            acc.setdefault(key, []).append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _counter_sums(folder):
    """Sum and count of the counter values per kernel name."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    acc = {}
    with open(files[0]) as f:
        for row in csv.DictReader(f):
            key = row.get("Kernel_Name", "")
            s, c = acc.get(key, (0.0, 0))
            acc[key] = (s + float(row["Counter_Value"]), c + 1)
    return acc


def traffic_from(args):
    """HBM bytes per launch of each kernel class: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) divided by what the same counters read for the copy
    kernel of known size (bytes counted / bytes moved)."""
    import re
    fetch = _counter_means(args.traffic_from[0])
    write = _counter_means(args.traffic_from[1])

    def copy_value(table):
        vals = [v for name, v in table.items() if "MulFunctor" in name]
        if not vals:
            raise SystemExit("copy kernel not found in the counter run")
        return max(vals) * 1024.0

    scale_f = copy_value(fetch) / COPY_PROBE_BYTES
    scale_w = copy_value(write) / COPY_PROBE_BYTES
    out = {}
    if args.workload == "3d":
        # every dispatch of a class, per component launch group
        import re as _re
        fs, ws = _counter_sums(args.traffic_from[0]), _counter_sums(args.traffic_from[1])
        steps = args.steps or 2
        for cls, pat in CLASS_PATTERNS_3D.items():
            rx = _re.compile(pat)
            groups = CALLS_3D[cls] * steps
            fb = sum(v[0] for name, v in fs.items() if rx.search(name)) * 1024.0 / scale_f / groups
            wb = sum(v[0] for name, v in ws.items() if rx.search(name)) * 1024.0 / scale_w / groups
            out[cls] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                        "copy_scale": {"fetch": scale_f, "write": scale_w},
                        "source_hash": kernel_source_hash("3d")}
        key = traffic_key(args.n, args)
        path = os.path.join(ROOT, "profiles", "traffic.json")
        data = json.load(open(path)) if os.path.exists(path) else {}
        data[key] = out
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        print(json.dumps({key: out}, indent=1))
        return
    pats = BATCH_CLASS_PATTERNS if args.workload == "batch" else CLASS_PATTERNS
    for cls, pat in pats.items():
        rx = re.compile(pat)
        fb = sum(v for name, v in fetch.items() if rx.search(name)) * 1024.0 / scale_f
        wb = sum(v for name, v in write.items() if rx.search(name)) * 1024.0 / scale_w
        if fb or wb:
            out[cls] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                        "copy_scale": {"fetch": scale_f, "write": scale_w},
                        "source_hash": kernel_source_hash(traffic_key(args.n, args))}
    key = traffic_key(args.n, args)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = out
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({key: out}, indent=1))


def exact_fields(n, k, tau_e, tau_h):
    from workloads import mode_fields
    return mode_fields(2, n, k, tau_e, tau_h)


def rel_l2(a: dict, b: dict, names):
    num = sum(float(np.sum((a[x] - b[x]) ** 2)) for x in names)
    den = sum(float(np.sum(b[x] ** 2)) for x in names)
    return float(np.sqrt(num / den))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--mode", type=str, default="4,3")
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--closure", default="paper")
    ap.add_argument("--lap", default="tracked")
    ap.add_argument("--profile-steps", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="batch", choices=["2d", "batch", "3d", "serve", "sweep", "nc", "source"],
                    help="batch: 512 seeded 2D cavities of uneven N (default); 2d: the N=2048 "
                         "refinement-sweep cavity; 3d: the cube cavity")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--serve-count", type=int, default=2000, help="serving: requests of the mix")
    ap.add_argument("--serve-limit", type=float, default=60.0, help="serving: seconds of the 200/s run")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="serving: rate of the full-mix run (default 70%% of the measured capacity)")
    ap.add_argument("--serve-chunk", type=int, default=96)
    ap.add_argument("--serve-chunk3", type=int, default=32, help="serving: steps per chunk of the 3D cohort")
    ap.add_argument("--serve-active", type=int, default=128, help="serving: requests active at once")
    ap.add_argument("--serve-streams", type=int, default=8, help="serving: side streams of the 3D requests")
    ap.add_argument("--serve-queues", type=int, default=16, help="serving: HIP hardware queues of the process")
    ap.add_argument("--serve-skip-full", action="store_true", help="serving: only the 200/s run")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refined"])
    ap.add_argument("--solver", default="chebyshev", choices=["chebyshev", "pcg", "transform"],
                    help="2d/3d workloads: fused fixed-sweep Chebyshev (default) or PCG with device reductions")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for a rocprofv3 --pmc run: one plain copy kernel of known size, then a few "
                         "steps of the 2D workload")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="read the FETCH_SIZE and WRITE_SIZE counter runs of --pmc-probe and write "
                         "profiles/traffic.json")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.traffic_from:
        return traffic_from(args)
    if args.pmc_probe:
        return pmc_probe(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "3d":
        return bench_3d(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "nc":
        return bench_nc(args)
    if args.workload == "source":
        return bench_source(args)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd import _lib as L

    n = args.n
    k = tuple(int(v) for v in args.mode.split(","))
    cfl = args.cfl
    h = 1.0 / n
    ht = cfl * h
    steps = args.steps if args.steps is not None else int(round(1.0 / ht))
    names = ["ez", "hx", "hy"]
    init = exact_fields(n, k, 0.0, ht / 2)
    stream = torch.cuda.Stream()              # a dedicated stream (default priority)
    kw = dict(closure=args.closure, lap_mode=args.lap, precision=args.precision, solver=args.solver, stream=stream)
    prec_name = "FP64" if args.precision == "fp64" else "FP32 Chebyshev rounds + FP64 residual"

    prob = Problem(2, n, cfl, **kw)

    def load_initial(p):
        for name in p.fields():
            p.set(name, init[name])

    load_initial(prob)
    prob.step(args.warmup)
    torch.cuda.synchronize()
    load_initial(prob)                         # timed run starts from the initial data
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    prob.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    cells = n * n
    value = cells * steps / elapsed / 1e6
    got = {x: prob.get(x) for x in names}
    ex = exact_fields(n, k, steps * ht, (steps + 0.5) * ht)
    l2_exact = rel_l2(got, ex, names)
    pinf = prob.info()
    sweeps = pinf["sweeps"]
    pcg_stats = None
    if args.solver == "pcg":
        pcg_stats = {"last_iters": pinf["last_iters"], "max_iters": pinf["max_iters"],
                     "last_rel_residual": pinf["last_rel_residual"], "noconv": pinf["noconv"]}
    prob.close()

    # ---- profiled pass: per-kernel durations from HIP events on the stream
    pp = Problem(2, n, cfl, flags=L.FLAG_PROFILE, **kw)
    load_initial(pp)
    pp.step(args.profile_steps)
    inf = pp.info()
    pp.close()
    per = {}
    for ci, cname in enumerate(L.KERNEL_CLASSES):
        cnt = inf["kernel_launches"][ci]
        if cnt:
            per[cname] = {"avg_us": 1e3 * inf["kernel_ms"][ci] / cnt, "launches": cnt,
                          "alg_bytes": inf["kernel_alg_bytes"][ci]}
    dom = max(per, key=lambda c: per[c]["avg_us"] * per[c]["launches"])
    dom_ach = per[dom]["alg_bytes"] / (per[dom]["avg_us"] * 1e-6) / 1e9
    workload_key = traffic_key(n, args)
    traffic = measured_traffic(dom, workload_key)
    roofline = {"bound": "hbm", "achieved": round(dom_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernels": CLASS_KERNELS.get(dom) if args.solver == "chebyshev" else None,
                "avg_us": round(per[dom]["avg_us"], 3),
                "step_alg_bytes_per_cell": sum(per[c]["alg_bytes"] for c in per) / cells,
                "per_kernel_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()}}
    step_alg = sum(per[c]["alg_bytes"] for c in per)
    roofline["step_frac"] = round(step_alg * value * 1e6 / cells / 1e9 / HBM_PEAK_GBS, 4)
    if args.solver == "transform":
        roofline = transform_roofline(2, n, per)

    # ---- CPU baseline: the oracle on the host cores, bounded sample of the
    # same workload; the device result after the same steps is compared.
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.OracleProblem(2, n, cfl, 1.0, closure=oracle.CLOSURE_PAPER if args.closure == "paper"
                                 else oracle.CLOSURE_REFLECT,
                                 lap_mode=oracle.LAP_TRACKED if args.lap == "tracked" else oracle.LAP_DISCRETE)
        for name in o.fields():
            o.set(name, init[name])
        t1 = time.perf_counter()
        done = 0
        while True:
            o.step(1)
            done += 1
            spent = time.perf_counter() - t1
            if spent >= args.cpu_seconds or done >= steps:
                break
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": round(cells * done / spent / 1e6, 3), "unit": "Mcell-steps/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{done} steps of the N={n} workload from the initial data ({spent:.1f} s, "
                         f"OpenMP over lines, {cores} threads)"}
        g = Problem(2, n, cfl, **kw)
        load_initial(g)
        g.step(done)
        gf = {x: g.get(x) for x in names}
        g.close()
        of = {x: o.get(x) for x in names}
        parity = {"steps": done, "rel_l2_vs_oracle": rel_l2(gf, of, names),
                  "max_abs_vs_oracle": max(float(np.max(np.abs(gf[x] - of[x]))) for x in names)}

    line = {
        "metric": "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline",
        "value": round(value, 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (exact PEC cavity mode sampled on the Yee grids)",
        "config": {"workload": f"2D TM PEC cavity N={n}, mode {k}, CFL {cfl}, T={steps * ht:g} "
                               f"({steps} steps), {args.closure} closure, {args.lap} Laplacian, {prec_name}",
                   "precision": args.precision,
                   "n": n, "mode": list(k), "cfl": cfl, "closure": args.closure,
                   "lap_mode": args.lap,
                   "solver": f"chebyshev x{sweeps}" if args.solver == "chebyshev" else args.solver},
        "l2_vs_exact": l2_exact,
        "parity_sample": parity,
        **({"pcg": pcg_stats} if pcg_stats else {}),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _cpu_cores():
    return len(os.sched_getaffinity(0))


def _omp_threads(n):
    """Thread count of the oracle's OpenMP loops (its runtime is loaded with it)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def _batch_run(specs, steps, warmup, stream, **kw):
    """Create a batch, load the exact modes, warm up, reload, and time
    `steps` steps between HIP events on its stream.  Returns (batch, inits,
    elapsed seconds)."""
    import torch
    from paper_2306_17263_amd import Batch
    from workloads import mode_fields
    b = Batch(specs, stream=stream, **kw)
    inits = []
    for p, s in zip(b.problems, specs):
        init = mode_fields(2, s["n"], s["k"], 0.0, s["r"] / s["n"] / 2, amp=s["amp"])
        inits.append(init)
        for name in p.fields():
            p.set(name, init[name])
    b.step(warmup)
    for p, init in zip(b.problems, inits):
        for name in p.fields():
            p.set(name, init[name])
    b.warm_info = b.info()                     # profiling counters after the warm-up (subtracted later)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
    return b, inits, elapsed


def _member_errors(problems, specs, steps):
    from workloads import mode_fields
    names = ["ez", "hx", "hy"]
    errs = []
    for p, s in zip(problems, specs):
        ht = s["r"] / s["n"]
        ex = mode_fields(2, s["n"], s["k"], steps * ht, (steps + 0.5) * ht, amp=s["amp"], with_laplacian=False)
        errs.append(rel_l2({a: p.get(a) for a in names}, ex, names))
    return errs


def bench_batch(args):
    """Batched form on the seeded 512-cavity mix (the default workload)."""
    import torch
    from paper_2306_17263_amd import Problem, autotune
    from paper_2306_17263_amd import _lib as L
    from workloads import batch_mix
    specs = batch_mix(count=args.count)
    steps = args.steps if args.steps is not None else 200
    st = torch.cuda.Stream()
    settings = dict(closure=args.closure, lap_mode=args.lap, precision=args.precision)
    tuned = autotune.tune_batch([{"n": s["n"]} for s in specs], steps=2, **settings)
    form = dict(tile_x=tuned["tile_x"], tile_y=tuned["tile_y"])
    cells = sum(s["n"] ** 2 for s in specs)
    names = ["ez", "hx", "hy"]

    # ---- timed region: every launch bracketed by HIP events on the stream
    b, inits, elapsed = _batch_run(specs, steps, args.warmup, st, flags=L.FLAG_PROFILE, **form, **settings)
    value = cells * steps / elapsed / 1e6
    inf, w0 = b.info(), b.warm_info
    per = {}
    for ci, cname in enumerate(L.KERNEL_CLASSES):
        cnt = inf["kernel_launches"][ci] - w0["kernel_launches"][ci]
        if cnt:
            per[cname] = {"avg_us": 1e3 * (inf["kernel_ms"][ci] - w0["kernel_ms"][ci]) / cnt, "launches": cnt,
                          "alg_bytes": inf["kernel_alg_bytes"][ci]}
    dom = max(per, key=lambda c: per[c]["avg_us"] * per[c]["launches"])
    dom_ach = per[dom]["alg_bytes"] / (per[dom]["avg_us"] * 1e-6) / 1e9
    step_alg = sum(per[c]["alg_bytes"] * per[c]["launches"] for c in per) / steps
    traffic = measured_traffic(dom, traffic_key(0, args))
    strips = form["tile_x"] == 0 and args.precision == "fp64"
    kernels = BATCH_KERNELS.get((dom, strips and form["tile_y"] != 1)) if strips else None
    roofline = {"bound": "hbm", "achieved": round(dom_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom, "kernels": kernels,
                "avg_us": round(per[dom]["avg_us"], 3), "alg_bytes_per_launch": per[dom]["alg_bytes"],
                "step_alg_bytes_per_cell": round(step_alg / cells, 3),
                "per_kernel_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()},
                "step_frac": round(step_alg * steps / elapsed / 1e9 / HBM_PEAK_GBS, 4)}
    errs = _member_errors(b.problems, specs, steps)

    # ---- full-size parity sample: members the oracle steps in seconds,
    # the same steps from the same initial data, element by element
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        order = sorted(range(len(specs)), key=lambda i: specs[i]["n"])
        mid = min(range(len(specs)), key=lambda i: abs(specs[i]["n"] - 160))
        parity = []
        for i in order[:4] + [mid]:
            s = specs[i]
            o = oracle.OracleProblem(2, s["n"], s["r"], 1.0, closure=CLOSURES_O[args.closure],
                                     lap_mode=LAPS_O[args.lap])
            for name in o.fields():
                o.set(name, inits[i][name])
            o.step(steps)
            gf = {a: b.problems[i].get(a) for a in names}
            of = {a: o.get(a) for a in names}
            scale = max(float(np.max(np.abs(of[a]))) for a in names)
            parity.append({"n": s["n"], "steps": steps, "rel_l2_vs_oracle": rel_l2(gf, of, names),
                           "max_abs_over_scale": max(float(np.max(np.abs(gf[a] - of[a]))) for a in names) / scale})
    b.close()

    # ---- the same steps in the default graph-replayed launches, and the
    # single persistent launch per step (strip form)
    extra = {}
    b2, _, el2 = _batch_run(specs, steps, args.warmup, st, **form, **settings)
    b2.close()
    extra["graph_ms_per_step"] = round(el2 * 1e3 / steps, 4)
    if strips:
        b3, _, el3 = _batch_run(specs, steps, args.warmup, st, tile_x=0, tile_y=1, **settings)
        b3.check()
        b3.close()
        extra["single_launch_ms_per_step"] = round(el3 * 1e3 / steps, 4)

    # ---- the plain FP64 stepper: the same problems one after another
    plain = dict(settings, precision="fp64")
    singles = []
    for s, init in zip(specs, inits):
        q = Problem(2, s["n"], s["r"], stream=st, **plain)
        for name in q.fields():
            q.set(name, init[name])
        singles.append(q)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for q in singles:
        q.step(steps)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    errs_plain = _member_errors(singles, specs, steps)
    for q in singles:
        q.close()

    # ---- precision form: FP32 Chebyshev rounds around FP64 residuals, same batch
    prec = None
    if args.precision == "fp64":
        b4, _, el4 = _batch_run(specs, steps, args.warmup, st, **dict(settings, precision="fp32_refined"))
        errs4 = _member_errors(b4.problems, specs, steps)
        b4.close()
        prec = {"ms_per_step": round(el4 * 1e3 / steps, 4), "speedup_vs_fp64_batch": round(elapsed / el4, 3),
                "max_l2_ratio_vs_fp64": max(e / f for e, f in zip(errs4, errs)),
                "form": "column tiles 128 x 4, FP32 Chebyshev rounds + FP64 residual"}

    # ---- CPU baseline: the oracle on 32 seeded members of the mix, on
    # every host core and on one
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(2306)
        sample = sorted(rng.choice(len(specs), 32, replace=False).tolist())

        def run_oracle(nsteps):
            t = time.perf_counter()
            done = 0
            for i in sample:
                s = specs[i]
                o = oracle.OracleProblem(2, s["n"], s["r"], 1.0, closure=CLOSURES_O[args.closure],
                                         lap_mode=LAPS_O[args.lap])
                for name in o.fields():
                    o.set(name, inits[i][name])
                o.step(nsteps)
                done += s["n"] ** 2 * nsteps
            return done, time.perf_counter() - t

        cores = _cpu_cores()
        _omp_threads(cores)
        done, spent = run_oracle(16)
        one = None
        if _omp_threads(1):
            done1, spent1 = run_oracle(2)
            one = round(done1 / spent1 / 1e6, 3)
            _omp_threads(cores)
        cpu = {"value": round(done / spent / 1e6, 3), "unit": "Mcell-steps/s", "cores": cores, "kind": "oracle",
               "sample": f"16 steps of each of 32 seeded members of the mix ({done / 1e6:.1f} M cell-steps, "
                         f"{spent:.1f} s, OpenMP over lines, {cores} threads); 2 steps each on 1 thread "
                         f"({spent1:.1f} s)" if one else f"16 steps of each of 32 seeded members ({spent:.1f} s)",
               "value_1thread": one}

    line = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "Mcell-steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded exact PEC cavity modes sampled on the Yee grids)",
        "config": {"workload": f"batched: {len(specs)} 2D TM PEC cavities, N uniform 64..768 (seed 2306), "
                               f"modes 1..8, amplitude 0.5..2, CFL 0.5, {steps} steps each, {args.closure} "
                               f"closure, {args.lap} Laplacian, {args.precision}",
                   "problems": len(specs), "cells_per_step": cells, "tile_x": form["tile_x"],
                   "tile_y": form["tile_y"],
                   "form": ("wave strips, one persistent launch per stage" if strips and form["tile_y"] != 1 else
                            "wave strips, one persistent launch per step" if strips else "column tiles"),
                   "autotune_s_per_step": tuned["timings"]},
        "l2_vs_exact": {"max": max(errs), "median": float(np.median(errs))},
        "parity_sample": parity,
        **extra,
        "plain_fp64_sequential_s": round(seq, 4), "speedup_vs_plain_fp64_sequential": round(seq / elapsed, 3),
        "max_l2_ratio_vs_plain_fp64": max(e / f for e, f in zip(errs, errs_plain)),
        "precision_form": prec,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_3d(args):
    """3D PEC cube cavity, mode (2,3,4), e = (-1,2,-1)/sqrt 6, CFL 0.4,
    T = 0.5 (1.25 N steps); every kernel-class launch group of the timed
    region bracketed by HIP events on the problem's stream."""
    import torch
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd import _lib as L
    from workloads import mode_fields
    n = args.n if args.n != 2048 else 256
    r = 0.4
    h = 1.0 / n
    ht = r * h
    steps = args.steps if args.steps is not None else int(round(0.5 / ht))
    st = torch.cuda.Stream()
    settings = dict(closure=args.closure, lap_mode=args.lap, precision=args.precision, solver=args.solver)
    init = mode_fields(3, n, (2, 3, 4), 0.0, ht / 2)
    p = Problem(3, n, r, stream=st, flags=L.FLAG_PROFILE, **settings)
    for name in p.fields():
        p.set(name, init[name])
    p.step(min(args.warmup, 4))
    for name in p.fields():
        p.set(name, init[name])
    w0 = p.info()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    p.step(steps)
    ev1.record(st)
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
    cells = n ** 3
    value = cells * steps / elapsed / 1e6
    names = ["ex", "ey", "ez", "hx", "hy", "hz"]
    ex = mode_fields(3, n, (2, 3, 4), steps * ht, (steps + 0.5) * ht, with_laplacian=False)
    l2 = rel_l2({a: p.get(a) for a in names}, ex, names)
    inf = p.info()
    p.close()
    per = {}
    for ci, cname in enumerate(L.KERNEL_CLASSES):
        cnt = inf["kernel_launches"][ci] - w0["kernel_launches"][ci]
        if cnt:
            per[cname] = {"avg_us": 1e3 * (inf["kernel_ms"][ci] - w0["kernel_ms"][ci]) / cnt, "launches": cnt,
                          "alg_bytes": inf["kernel_alg_bytes"][ci]}
    dom = max(per, key=lambda c: per[c]["avg_us"] * per[c]["launches"])
    dom_ach = per[dom]["alg_bytes"] / (per[dom]["avg_us"] * 1e-6) / 1e9
    step_alg = sum(per[c]["alg_bytes"] * per[c]["launches"] for c in per) / steps
    key = f"3d_n{n}_{args.closure}_{args.lap}_{args.precision}_{args.solver}"
    traffic = measured_traffic("solve" if dom.startswith("solve") else "rhs", key)
    roofline = {"bound": "hbm", "achieved": round(dom_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "kernels": KERNELS_3D.get(dom.split("_")[0]), "avg_us": round(per[dom]["avg_us"], 3),
                "alg_bytes_per_launch": per[dom]["alg_bytes"],
                "launch": "one component's launch group of the class (3 per step and half-step class)",
                "step_alg_bytes_per_cell": round(step_alg / cells, 3),
                "per_kernel_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()},
                "step_frac": round(step_alg * steps / elapsed / 1e9 / HBM_PEAK_GBS, 4)}
    if args.solver == "transform":
        roofline = transform_roofline(3, n, per)
    line = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "Mcell-steps/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 4),
        "ms_per_step": round(elapsed * 1e3 / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (exact PEC cube-cavity mode)",
        "config": {"workload": f"3D PEC cube cavity N={n}, mode (2,3,4), CFL 0.4, T={steps * ht:g} ({steps} steps), "
                               f"{args.closure} closure, {args.lap} Laplacian, {args.precision}", "n": n},
        "l2_vs_exact": l2,
        "roofline": roofline,
    }
    print(json.dumps(line), flush=True)


def bench_nc(args):
    """The comparison scheme NC (Section 5.2) on the 2D cavity of the
    refinement sweep (N = 2048, mode (4, 3), CFL 0.5, T = 1), next to the
    compact scheme on the same grid and steps: throughput and the L2 error
    against the exact mode of each (accuracy per cost)."""
    import torch
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd import _lib as L
    n = args.n
    k = tuple(int(v) for v in args.mode.split(","))
    cfl = args.cfl
    ht = cfl / n
    steps = args.steps if args.steps is not None else int(round(1.0 / ht))
    names = ["ez", "hx", "hy"]
    init = exact_fields(n, k, 0.0, ht / 2)
    st = torch.cuda.Stream()
    runs = {}
    per = {}
    for scheme in ("nc", "c4"):
        p = Problem(2, n, cfl, stream=st, scheme=scheme)
        for name in p.fields():
            p.set(name, init[name])
        p.step(args.warmup)
        for name in p.fields():
            p.set(name, init[name])
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        p.step(steps)
        ev1.record(st)
        torch.cuda.synchronize()
        el = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
        ex = exact_fields(n, k, steps * ht, (steps + 0.5) * ht)
        runs[scheme] = {"ms_per_step": round(el * 1e3 / steps, 5), "l2_vs_exact": rel_l2({a: p.get(a) for a in names}, ex, names),
                        "mcell_steps_per_s": round(n * n * steps / el / 1e6, 2)}
        if scheme == "nc":
            value = n * n * steps / el / 1e6
        p.close()
    # per-kernel averages from a separate profiled run (events around every launch)
    p = Problem(2, n, cfl, stream=st, scheme="nc", flags=L.FLAG_PROFILE)
    for name in p.fields():
        p.set(name, init[name])
    p.step(args.warmup)
    w0 = p.info()
    p.step(min(steps, args.profile_steps))
    inf = p.info()
    for ci, cname in enumerate(L.KERNEL_CLASSES):
        cnt = inf["kernel_launches"][ci] - w0["kernel_launches"][ci]
        if cnt:
            per[cname] = {"avg_us": 1e3 * (inf["kernel_ms"][ci] - w0["kernel_ms"][ci]) / cnt,
                          "alg_bytes": inf["kernel_alg_bytes"][ci]}
    p.close()
    dom = max(per, key=lambda c: per[c]["avg_us"])
    ach = per[dom]["alg_bytes"] / (per[dom]["avg_us"] * 1e-6) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mcell-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": runs["nc"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (exact PEC cavity mode sampled on the Yee grids)",
        "config": {"workload": f"NC scheme, 2D TM PEC cavity N={n}, mode {k}, CFL {cfl}, {steps} steps", "n": n},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                     "kernels": "k_nc_e (Ez update) / k_nc_h (Hx and Hy updates)",
                     "avg_us": round(per[dom]["avg_us"], 3), "alg_bytes_per_launch": per[dom]["alg_bytes"],
                     "per_kernel_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()}},
        "runs": runs,
        "error_ratio_nc_over_c4": runs["nc"]["l2_vs_exact"] / runs["c4"]["l2_vs_exact"],
    }
    print(json.dumps(line), flush=True)


def bench_source(args):
    """The 2D step with a current Jz (c4m_step_source) on the driven cavity
    (N = 2048, CFL 0.5; the source arrays of one instant, resident on the
    device and reused every step), next to the plain step of the same
    problem: throughput, and the source correction's roofline (one launch
    group per field component: its right-hand side and the Chebyshev
    applications of M, against the compulsory bytes of the group)."""
    import torch
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd import _lib as L
    from workloads.driven import DrivenTM
    n, cfl = args.n, args.cfl
    ht = cfl / n
    steps = args.steps if args.steps is not None else 200
    drv = DrivenTM()
    init = drv.fields(n, 0.0, ht / 2)
    st = torch.cuda.Stream()
    data = dict(drv.step1_data(n, 0.25))
    data.update(drv.step2_data(n, 0.25))

    def on_dev(v):
        if isinstance(v, list):
            return [[torch.as_tensor(a).to("cuda") for a in w] for w in v]
        return torch.as_tensor(v).to("cuda").contiguous()

    with torch.cuda.stream(st):
        dev = {k: on_dev(v) for k, v in data.items()}
    torch.cuda.synchronize()
    runs = {}
    for mode in ("source", "plain"):
        p = Problem(2, n, cfl, stream=st)
        for name in p.fields():
            p.set(name, init[name])
        go = (lambda k: [p.step_source(dev) for _ in range(k)]) if mode == "source" else p.step
        go(args.warmup)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        go(steps)
        ev1.record(st)
        torch.cuda.synchronize()
        el = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
        runs[mode] = {"ms_per_step": round(el * 1e3 / steps, 5), "mcell_steps_per_s": round(n * n * steps / el / 1e6, 2)}
        p.close()
    # per-class averages from a separate profiled run (events around every launch group)
    p = Problem(2, n, cfl, stream=st, flags=L.FLAG_PROFILE)
    for name in p.fields():
        p.set(name, init[name])
    for _ in range(args.warmup):
        p.step_source(dev)
    w0 = p.info()
    for _ in range(min(steps, args.profile_steps)):
        p.step_source(dev)
    inf = p.info()
    per = {}
    for ci, cname in enumerate(L.KERNEL_CLASSES):
        cnt = inf["kernel_launches"][ci] - w0["kernel_launches"][ci]
        if cnt:
            per[cname] = {"avg_us": 1e3 * (inf["kernel_ms"][ci] - w0["kernel_ms"][ci]) / cnt,
                          "alg_bytes": inf["kernel_alg_bytes"][ci]}
    p.close()
    src = per["other"]
    ach = src["alg_bytes"] / (src["avg_us"] * 1e-6) / 1e9
    line = {
        "metric": "sourced 2D step throughput", "value": runs["source"]["mcell_steps_per_s"], "unit": "Mcell-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": runs["source"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (the driven-cavity current and wall data of one instant, resident and reused every step)",
        "config": {"workload": f"2D TM PEC cavity driven by a current Jz, N={n}, CFL {cfl}", "n": n},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "other",
                     "kernels": "k_src_tile (one launch per field component: its source right-hand side and K applications of M on an LDS window, then the update)",
                     "avg_us": round(src["avg_us"], 3), "alg_bytes_per_launch": src["alg_bytes"],
                     "per_class_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()}},
        "runs": runs,
        "source_overhead_ms_per_step": round(runs["source"]["ms_per_step"] - runs["plain"]["ms_per_step"], 5),
    }
    print(json.dumps(line), flush=True)


def bench_sweep(args):
    """Refinement sweep of the 2D TM cavity: N = 128 .. 2048, mode (4, 3),
    CFL 0.5, T = 1 (2N steps each): L2 error against the exact mode, the
    observed order between successive N, and the throughput of each run."""
    import math
    import torch
    from paper_2306_17263_amd import Problem
    ns = (128, 256, 512, 1024, 2048)
    k = (4, 3)
    cfl = 0.5
    names = ["ez", "hx", "hy"]
    st = torch.cuda.Stream()
    runs = []
    total_cells, total_s = 0.0, 0.0
    for n in ns:
        ht = cfl / n
        steps = int(round(1.0 / ht))
        init = exact_fields(n, k, 0.0, ht / 2)
        p = Problem(2, n, cfl, stream=st, closure=args.closure, lap_mode=args.lap, precision=args.precision)

        def load():
            for name in p.fields():
                p.set(name, init[name])

        load()
        p.step(min(args.warmup, steps))
        load()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(st)
        p.step(steps)
        ev1.record(st)
        torch.cuda.synchronize()
        elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
        ex = exact_fields(n, k, steps * ht, (steps + 0.5) * ht)
        err = rel_l2({x: p.get(x) for x in names}, ex, names)
        p.close()
        runs.append({"n": n, "steps": steps, "l2_vs_exact": err, "seconds": round(elapsed, 5),
                     "mcell_steps_per_s": round(n * n * steps / elapsed / 1e6, 2)})
        total_cells += n * n * steps
        total_s += elapsed
    for a, b in zip(runs, runs[1:]):
        b["observed_order"] = round(math.log2(a["l2_vs_exact"] / b["l2_vs_exact"]), 3)
    line = {
        "metric": "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline",
        "value": round(total_cells / total_s / 1e6, 2), "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": sum(r["steps"] for r in runs), "warmup": args.warmup,
        "ms_per_step": round(total_s * 1e3 / sum(r["steps"] for r in runs), 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (exact PEC cavity mode sampled on the Yee grids)",
        "config": {"workload": f"2D TM PEC cavity refinement sweep N=128..2048, mode (4, 3), CFL 0.5, T=1, "
                               f"{args.closure} closure, {args.lap} Laplacian, {args.precision}"},
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


MFMA_F64_PEAK_TFLOPS = 78.6


def transform_flops(dim: int, n: int) -> dict:
    """Algorithmic flops of one launch group of the transform solve (a dense
    product per axis forward and back, 2 flops per multiply-add): 2D solve_e
    = Ez, solve_h = Hx and Hy; 3D one component of either kind."""
    def solve(sizes):
        cells = 1
        for v in sizes:
            cells *= v
        return 2.0 * cells * 2 * sum(sizes)        # forward and inverse along every axis
    if dim == 2:
        return {"solve_e": solve((n - 1, n - 1)), "solve_h": 2 * solve((n - 1, n))}
    return {"solve_e": solve((n, n - 1, n - 1)), "solve_h": solve((n - 1, n, n))}


def transform_roofline(dim: int, n: int, per: dict) -> dict:
    fl = transform_flops(dim, n)
    dom = max(fl, key=lambda c: per[c]["avg_us"] * per[c]["launches"])
    ach = fl[dom] / (per[dom]["avg_us"] * 1e-6) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 2), "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / MFMA_F64_PEAK_TFLOPS, 4), "traffic": None, "kernel": dom,
            "kernels": "k_gemm_f64 (FP64 MFMA 16x16x4 tiles): 4 products per 2D component, 6 per 3D one",
            "flops_per_launch_group": fl[dom], "avg_us": round(per[dom]["avg_us"], 3),
            "note": "2D solve classes also hold the right-hand-side kernel of the component",
            "per_kernel_avg_us": {c: round(v["avg_us"], 3) for c, v in per.items()}}


def bench_serve(args):
    """Serving form: Poisson arrivals (seed 17263) of mixed 2D (N 64..1024)
    and 3D (N 32..128) cavity solves of 100..2000 steps, admitted by HBM
    footprint into the continuous-batching loop.  Two runs of the same mix:
      * the workload's rate, 200 requests/s, for --serve-limit seconds (the
        offered work is several times one GPU's capacity, so the completed
        throughput is the capacity and latency is queue-dominated);
      * all --serve-count requests at a sub-saturation rate, 70 % of the
        capacity the first run measured (in requests/s of this mix).
    The loop runs on several streams (the 2D cohort, the 3D requests, the
    set-up of new requests); the process asks HIP for 8 hardware queues so
    that set-up copies do not queue behind another stream's kernels."""
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_queues)   # read when HIP initialises (not yet here)
    import torch
    from paper_2306_17263_amd.serve import DeviceBackend, Server, requests_from_mix
    from workloads import serving_arrivals
    count = args.serve_count
    free, total = torch.cuda.mem_get_info()
    budget = int(0.5 * free)
    settings = dict(closure=args.closure, lap_mode=args.lap, precision=args.precision)
    runs = {}
    mix = serving_arrivals(count=count, seed=17263, rate=200.0)
    work_per_req = sum(m["n"] ** m["dim"] * m["steps"] for m in mix) / count

    def one(label, rate, limit):
        reqs = requests_from_mix(serving_arrivals(count=count, seed=17263, rate=rate))
        print(f"serve run {label}: {count} requests at {rate:.3f}/s, limit {limit}", file=sys.stderr, flush=True)
        be = DeviceBackend(settings=settings, chunk=args.serve_chunk, n_side_streams=args.serve_streams)
        out = Server(be, hbm_budget=budget, chunk=args.serve_chunk, chunk_3d=args.serve_chunk3,
                     max_active=args.serve_active).run(
            reqs, time_limit=limit, progress=lambda t: print(f"  {label}: {t}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        d2 = [r for r in out["done"] if r.dim == 2]
        d3 = [r for r in out["done"] if r.dim == 3]
        pct = lambda rs, q: round(float(np.percentile([r.t_done - r.t_arrive for r in rs], q)), 4) if rs else None
        runs[label] = {"rate_per_s": round(rate, 4), "requests": len(reqs), "completed": out["completed"],
                       "time_limit_s": limit,
                       "p50_latency_s": round(out["p50_latency_s"], 4),
                       "p99_latency_s": round(out["p99_latency_s"], 4),
                       "p50_p99_2d_s": [pct(d2, 50), pct(d2, 99)], "p50_p99_3d_s": [pct(d3, 50), pct(d3, 99)],
                       "Mcell_steps_per_s": round(out["cell_steps_per_s"] / 1e6, 2),
                       "executed_Mcell_steps_per_s": round(out["executed_cell_steps_per_s"] / 1e6, 2),
                       "not_finished": out["queued_or_active_at_end"],
                       "wall_s": round(out["wall_s"], 3), "chunks": out["chunks"],
                       "peak_hbm_GB": round(out["peak_hbm_bytes"] / 1e9, 3),
                       "host_s": {a: round(v, 3) for a, v in be.host_s.items()}, "batch_reforms": be.reforms}
        print(json.dumps({label: runs[label]}), file=sys.stderr, flush=True)
        return out

    out = one("rate_200_per_s", 200.0, args.serve_limit)
    capacity = out["executed_cell_steps_per_s"]
    sub_rate = args.serve_rate if args.serve_rate else 0.7 * capacity / work_per_req
    if not args.serve_skip_full:
        one("sub_saturation_full_mix", sub_rate, None)
    line = {
        "metric": METRIC,
        "value": runs["rate_200_per_s"]["executed_Mcell_steps_per_s"], "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded Poisson arrivals of exact cavity modes)",
        "config": {"workload": f"serving: {count}-request mix (50% 2D N 64..1024, 50% 3D N 32..128, "
                               f"100..2000 steps), HBM budget {budget / 1e9:.1f} GB, chunk {args.serve_chunk}",
                   "budget_bytes": budget, "offered_cell_steps_per_request": work_per_req},
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
