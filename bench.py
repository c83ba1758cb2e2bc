"""Throughput benchmark of the compact fourth-order Yee stepper on one MI355X.

Default workload: 2D TM PEC unit-square cavity, N = 2048, mode (k, l) = (4, 3),
CFL 0.5, FP64, PAPER closure with the carried Laplacian; one bench step is
one time step (Step 1 + Step 2) of that problem, and the default K = 4096
steps covers T = 1.  The fields are resident in HBM before the timed region.

Prints ONE JSON line with the metric, the roofline block of the dominant
kernel (per-kernel HIP-event timing on the problem's stream, in a profiled
pass of the same steps right after the timed region) and the CPU baseline
(the oracle on the host cores over a bounded sample of the same workload,
also used as a full-size parity check of the device result).
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_17263_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
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
    if not ent or ent.get("source_hash") != kernel_source_hash():
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


def traffic_key(n, args):
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
    for cls, pat in CLASS_PATTERNS.items():
        rx = re.compile(pat)
        fb = sum(v for name, v in fetch.items() if rx.search(name)) * 1024.0 / scale_f
        wb = sum(v for name, v in write.items() if rx.search(name)) * 1024.0 / scale_w
        if fb or wb:
            out[cls] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                        "copy_scale": {"fetch": scale_f, "write": scale_w},
                        "source_hash": kernel_source_hash()}
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
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--mode", type=str, default="4,3")
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--closure", default="paper")
    ap.add_argument("--lap", default="tracked")
    ap.add_argument("--profile-steps", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="2d", choices=["2d", "batch", "3d", "serve", "sweep"],
                    help="2d: the N=2048 refinement-sweep cavity (default); batch: 512 seeded 2D "
                         "cavities of uneven N; 3d: the cube cavity")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refined"])
    ap.add_argument("--solver", default="chebyshev", choices=["chebyshev", "pcg"],
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
                   "solver": f"chebyshev x{sweeps}" if args.solver == "chebyshev" else "pcg"},
        "l2_vs_exact": l2_exact,
        "parity_sample": parity,
        **({"pcg": pcg_stats} if pcg_stats else {}),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _cpu_cores():
    return len(os.sched_getaffinity(0))


def bench_batch(args):
    """Batched form: seeded mix of independent 2D TM cavities, N uniform in
    64..768, modes (k, l) in 1..8, amplitude U(0.5, 2), CFL 0.5, 200 steps
    each, one persistent launch per phase and a HIP graph per step, launch
    shape from the autotuner."""
    import torch
    from paper_2306_17263_amd import Batch, Problem, autotune
    from workloads import batch_mix, mode_fields
    specs = batch_mix(count=args.count)
    steps = args.steps if args.steps is not None else 200
    st = torch.cuda.Stream()
    settings = dict(closure=args.closure, lap_mode=args.lap, precision=args.precision)
    tuned = autotune.tune_batch([{"n": s["n"]} for s in specs], steps=2, **settings)
    b = Batch(specs, stream=st, tile_x=tuned["tile_x"], tile_y=tuned["tile_y"], **settings)
    inits = []
    for p, s in zip(b.problems, specs):
        h = 1.0 / s["n"]
        init = mode_fields(2, s["n"], s["k"], 0.0, s["r"] * h / 2, amp=s["amp"])
        inits.append(init)
        for name in p.fields():
            p.set(name, init[name])
    b.step(args.warmup)
    for p, init in zip(b.problems, inits):
        for name in p.fields():
            p.set(name, init[name])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    b.step(steps)
    ev1.record(st)
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3)
    cells = sum(s["n"] ** 2 for s in specs)
    value = cells * steps / elapsed / 1e6
    # accuracy of every problem against its exact mode at the final time
    names = ["ez", "hx", "hy"]
    errs = []
    for p, s in zip(b.problems, specs):
        h = 1.0 / s["n"]
        ht = s["r"] * h
        ex = mode_fields(2, s["n"], s["k"], steps * ht, (steps + 0.5) * ht, amp=s["amp"], with_laplacian=False)
        errs.append(rel_l2({a: p.get(a) for a in names}, ex, names))
    # the plain FP64 stepper: the same problems one after another through the
    # single-problem path (created and loaded before the clock starts)
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
    errs_plain = []
    for q, s in zip(singles, specs):
        ht = s["r"] / s["n"]
        ex = mode_fields(2, s["n"], s["k"], steps * ht, (steps + 0.5) * ht, amp=s["amp"], with_laplacian=False)
        errs_plain.append(rel_l2({a: q.get(a) for a in names}, ex, names))
        q.close()
    err_ratio = max(e / f for e, f in zip(errs, errs_plain))
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        sub = sorted(range(len(specs)), key=lambda i: specs[i]["n"])[:3]
        parity = []
        for i in sub:
            s = specs[i]
            o = oracle.OracleProblem(2, s["n"], s["r"], 1.0)
            for name in o.fields():
                o.set(name, inits[i][name])
            o.step(steps)
            parity.append({"n": s["n"], "rel_l2_vs_oracle":
                           rel_l2({a: b.problems[i].get(a) for a in names}, {a: o.get(a) for a in names}, names)})
        rng = np.random.default_rng(2306)
        sample = sorted(rng.choice(len(specs), 32, replace=False).tolist())
        t2 = time.perf_counter()
        done = 0
        for i in sample:
            s = specs[i]
            o = oracle.OracleProblem(2, s["n"], s["r"], 1.0)
            for name in o.fields():
                o.set(name, inits[i][name])
            o.step(2)
            done += s["n"] ** 2 * 2
            if time.perf_counter() - t2 > args.cpu_seconds:
                break
        spent = time.perf_counter() - t2
        cpu = {"value": round(done / spent / 1e6, 3), "unit": "Mcell-steps/s", "cores": _cpu_cores(), "kind": "oracle",
               "sample": f"2 steps of each of up to 32 seeded problems of the mix ({spent:.1f} s)"}
    b.close()
    line = {
        "metric": "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline",
        "value": round(value, 2), "unit": "Mcell-steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded exact PEC cavity modes)",
        "config": {"workload": f"batched: {len(specs)} 2D TM cavities, N uniform 64..768 (seed 2306), "
                               f"modes 1..8, CFL 0.5, {steps} steps each, {args.precision}",
                   "problems": len(specs), "cells_per_step": cells, "tile_x": tuned["tile_x"],
                   "tile_y": tuned["tile_y"], "autotune_timings_s": tuned["timings"]},
        "l2_vs_exact": {"max": max(errs), "median": float(np.median(errs))},
        "plain_fp64_sequential_s": round(seq, 4), "speedup_vs_plain_fp64_sequential": round(seq / elapsed, 3),
        "l2_vs_exact_plain_fp64": {"max": max(errs_plain), "median": float(np.median(errs_plain))},
        "max_l2_ratio_vs_plain_fp64": err_ratio,
        "parity_sample": parity,
        "step_frac": round(88.0 * value * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_3d(args):
    """3D PEC cube cavity, mode (2,3,4), CFL 0.4, T = 0.5."""
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
    p = Problem(3, n, r, stream=st, **settings)
    for name in p.fields():
        p.set(name, init[name])
    p.step(min(args.warmup, 4))
    for name in p.fields():
        p.set(name, init[name])
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
    p.close()
    pp = Problem(3, n, r, stream=st, flags=L.FLAG_PROFILE, **settings)
    for name in pp.fields():
        pp.set(name, init[name])
    pp.step(2)
    inf = pp.info()
    pp.close()
    per = {c: 1e3 * inf["kernel_ms"][i] / inf["kernel_launches"][i] for i, c in enumerate(L.KERNEL_CLASSES)
           if inf["kernel_launches"][i]}
    line = {
        "metric": "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline",
        "value": round(value, 2), "unit": "Mcell-steps/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 4),
        "ms_per_step": round(elapsed * 1e3 / steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (exact PEC cube-cavity mode)",
        "config": {"workload": f"3D PEC cube cavity N={n}, mode (2,3,4), CFL 0.4, T=0.5 ({steps} steps), "
                               f"{args.closure} closure, {args.lap} Laplacian, {args.precision}", "n": n},
        "l2_vs_exact": l2,
        "per_class_avg_us": {c: round(v, 1) for c, v in per.items()},
        "step_frac": round(192.0 * value * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
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


def bench_serve(args):
    """Serving form: Poisson arrivals (seed 17263) of mixed 2D (N 64..1024)
    and 3D (N 32..128) cavity solves of 100..2000 steps, admitted by HBM
    footprint into a continuous-batching loop.  Two runs: the arrival rate of
    the workload (200/s, first --count requests; the offered work is far
    above one GPU's capacity, so latency is queue-dominated) and a rate at
    about 70 % of the capacity measured in the first run."""
    import torch
    from paper_2306_17263_amd.serve import DeviceBackend, Server, requests_from_mix
    from workloads import serving_arrivals
    count = args.count if args.count != 512 else 48
    free, total = torch.cuda.mem_get_info()
    budget = int(0.5 * free)
    runs = {}
    rate = 200.0
    for label in ("rate_200_per_s", "sub_saturation"):
        mix = serving_arrivals(count=count, seed=17263, rate=rate)
        reqs = requests_from_mix(mix)
        be = DeviceBackend(settings=dict(closure=args.closure, lap_mode=args.lap, precision=args.precision))
        out = Server(be, hbm_budget=budget, chunk=100).run(reqs)
        work = sum(r.cells * r.steps for r in reqs)
        runs[label] = {"rate_per_s": round(rate, 3), "requests": len(reqs), "completed": out["completed"],
                       "p50_latency_s": round(out["p50_latency_s"], 4),
                       "p99_latency_s": round(out["p99_latency_s"], 4),
                       "Mcell_steps_per_s": round(out["cell_steps_per_s"] / 1e6, 2),
                       "wall_s": round(out["wall_s"], 3), "ticks": out["ticks"],
                       "peak_hbm_GB": round(out["peak_hbm_bytes"] / 1e9, 3)}
        capacity = out["cell_steps_per_s"]
        rate = 0.7 * capacity / (work / len(reqs))
    line = {
        "metric": "Mcell-steps/s at fixed L2 error vs FP64 oracle + % HBM roofline; p50/p99 latency",
        "value": runs["rate_200_per_s"]["Mcell_steps_per_s"], "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded Poisson arrivals of exact cavity modes)",
        "config": {"workload": f"serving: first {count} requests of the 200/s mix (50% 2D N 64..1024, 50% 3D "
                               f"N 32..128, 100..2000 steps), HBM budget {budget / 1e9:.1f} GB, chunk 100",
                   "budget_bytes": budget},
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
