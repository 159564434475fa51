#!/usr/bin/env python3
"""Throughput of the generalised 'abc' set-projection iteration on one MI355X.

A step is one full iteration of the hot path over every diffraction pattern
of the workload: divide (the pending update, forward DFT, relaxed modulus
projection, inverse DFT), concur (object and probe overlap consensus in
float64) and the metric finalisation.  The metric is diffraction-pattern
projections per second, J * steps / time, with every input resident in HBM
before the timed region starts.

Default workload: scan_n128 -- object 1024 x 1024, N = 128, J = 1024
positions (32 x 32 raster, step 28, +-2 jitter), Poisson data at 1e6 photons
per pattern, blind RAAR (beta = 0.75), float32 exit waves with float64
overlap sums.  Inputs are seeded and synthetic (ptysynth).

The roofline figure is for the kernel with the largest share of the step,
timed with HIP events on the scan's stream over the timed region itself.

  python bench.py [--steps K] [--warmup W] [--workload scan_n128|large_n256|tiny_n32]
  python bench.py --summarize-pmc FETCH_CSV WRITE_CSV   (writes the traffic file under profiles/)
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
KERNEL_NAMES = {
    "divide": "divide_fused_kernel",
    "divide_cols": "cols256_kernel",
    "divide_rows_inv": "rows256_inv_kernel",
    "object": "object_lds_kernel",
    "probe": "probe_partial_kernel",
    "final": "probe_final_kernel",
}


def kernel_name(cls: str, n: int) -> str:
    """The HIP kernel behind a kernel class at pattern size n."""
    if n == 256 and cls == "divide":
        return "rows256_fwd_kernel"
    if n == 256 and cls == "object":
        return "object_update_kernel"
    return KERNEL_NAMES[cls]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{kernel}_{workload}.json")
# Kernel durations come from HIP events around the launches of every 16th
# iteration of the timed region (every iteration of short runs, so that at
# least eight are timed): an event pair around every launch would add about
# 29 us per N = 128 iteration (13 %) to the throughput it measures.
PROFILE_EVERY = 16


def profile_every(steps: int) -> int:
    return max(1, min(PROFILE_EVERY, steps // 8))


def sampled_iterations(k0: int, steps: int, every: int) -> int:
    """Iterations k0 .. k0+steps-1 whose launches the sampled event timing covers."""
    return sum(1 for k in range(k0, k0 + steps) if k % every == 0)


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2311_11466_amd", "csrc", f)
                  for f in ("divide.hip", "divide_fused.hpp", "divide_ops.hpp", "divide_n32.hip", "divide_n64.hip",
                            "divide_n128.hip", "concur.hip", "common.hpp", "params.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, n: int, J: int, abc, blind: bool, storage: str, full_metrics=True):
    """HBM bytes one launch of a kernel class must move (roofline numerator).

    Per pattern pixel: divide reads x_{k-1}, y_{k-1} (when needed), sqrt(I)
    (4 B) and writes x_k, y_k; the N = 256 column pass reads and writes its
    float32 intermediate (16 B) and reads sqrt(I); the row passes read or write
    the intermediate (8 B) besides the exit waves; the object and probe kernels
    read y once each.  Object/probe gathers and the float64 partial sums are
    not counted (they are cache-resident or small).
    """
    from paper_2311_11466_amd import uses_blend_form
    a, b, _ = abc
    e = 4 if storage == "fp16" else 8
    rx = e if (abs(1 - a) > 0 or full_metrics) else 0
    ry = e if (abs(a * (1 - b)) > 0 or full_metrics) else 0
    nn = n * n * J
    if kind == "divide":
        if uses_blend_form(n, a, b, full_metrics):
            return (e + 4 + e + e) * nn             # w_{k-1}, sqrt(I) in; w_k, y_k out
        if n == 256:
            return (rx + ry + rx + 8) * nn          # rows forward: x, y in; x out; intermediate out
        return (rx + ry + 4 + rx + e) * nn
    if kind == "divide_cols":
        return (8 + 4 + 8) * nn
    if kind == "divide_rows_inv":
        return (8 + e) * nn
    if kind in ("object", "probe"):
        return e * nn
    return 0


def make_workload(name: str):
    import numpy as np
    from ptysynth import make_scan
    scan = make_scan(name, intensity_dtype=np.float32)
    return scan


def run_cpu_baseline(scan, abc, n_iter: int):
    """The FP64 oracle, as it stands, on the same scan for n_iter iterations."""
    import numpy as np
    from oracle import pty_oracle as po
    amp = np.sqrt(scan.intensity.astype(np.float64))
    st = po.init_state(scan.obj0, scan.probe0, scan.pos)
    t0 = time.perf_counter()
    po.run(st, amp, scan.pos, *abc, n_iter, blind=True)
    dt = time.perf_counter() - t0
    return scan.n_pos * n_iter / dt, dt


def load_traffic(kernel: str, workload: str):
    path = TRAFFIC_FILE.format(kernel=kernel, workload=workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None      # the kernel changed since the counters were taken
    return t.get("bytes_per_launch")


def bench(args):
    import numpy as np
    import torch
    import paper_2311_11466_amd as pk

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    scan = make_workload(args.workload)
    abc = pk.preset(args.algorithm, args.param)
    cfg = scan.config
    full_metrics = args.metrics == "all"
    print(f"# workload {cfg.name}: object {cfg.obj_h}x{cfg.obj_w}, N={cfg.n}, J={scan.n_pos}", file=sys.stderr,
          flush=True)
    g = pk.Scan(torch.as_tensor(scan.pos).to(dev), torch.as_tensor(scan.intensity).to(dev),
                torch.as_tensor(scan.obj0.astype(np.complex64)).to(dev),
                torch.as_tensor(scan.probe0.astype(np.complex64)).to(dev),
                storage=args.storage, blind=True, device=dev, full_metrics=full_metrics)
    g.set_algorithm(*abc)
    g.set_concur_sweeps(args.concur_sweeps)
    sched = None
    if args.schedule == "linear":
        # the preset's parameter (beta or lambda) moves linearly from --param to
        # --param-end over warm-up and timed iterations
        n_all = args.warmup + args.steps
        sched = [pk.preset(args.algorithm, args.param + (args.param_end - args.param) * i / max(n_all - 1, 1))
                 for i in range(n_all)]
        g.iterate_schedule(sched[:args.warmup])
    else:
        g.iterate(args.warmup)
    torch.cuda.synchronize()
    every = profile_every(args.steps)
    n_sampled = sampled_iterations(g.iteration, args.steps, every)
    g.profile(True, every=every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if sched is not None:
        g.iterate_schedule(sched[args.warmup:])
    else:
        g.iterate(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    dt = t1 - t0
    m = g.metrics(allow_diverged=True)
    print(f"# timed {args.steps} steps in {dt * 1e3:.2f} ms; last metrics {m}", file=sys.stderr, flush=True)

    kernels = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_us = ms / cnt * 1e3
        nbytes = algorithmic_bytes(k, cfg.n, scan.n_pos, abc, True, args.storage, full_metrics)
        kernels[k] = {"avg_us": round(avg_us, 3), "launches": cnt,
                      "share": round(ms / n_sampled * args.steps / (dt * 1e3), 4),
                      "algorithmic_bytes": nbytes,
                      "GBs": round(nbytes / (avg_us * 1e-6) / 1e9, 1) if nbytes else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    d = kernels[dom]
    traffic = load_traffic(dom, cfg.name)
    roofline = {"bound": "hbm", "achieved": d["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["GBs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name(dom, cfg.n), "avg_us": d["avg_us"],
                "algorithmic_bytes_per_launch": d["algorithmic_bytes"]}

    if args.copy_probe:
        # a plain elementwise kernel of known traffic (reads 2 B, writes B bytes), for
        # scaling the rocprofv3 FETCH_SIZE / WRITE_SIZE counters
        nf = args.copy_probe_bytes // 4
        a = torch.ones(nf, dtype=torch.float32, device=dev)
        b = torch.ones(nf, dtype=torch.float32, device=dev)
        c = torch.empty(nf, dtype=torch.float32, device=dev)
        for _ in range(3):
            torch.add(a, b, out=c)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu = 3 if cfg.n <= 128 else 1        # about 3 s (N = 128) or 18 s (N = 256) of host work
        rate, cpu_dt = run_cpu_baseline(scan, abc, n_cpu)
        cpu = {"value": round(rate, 2), "unit": "projections/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_cpu} iterations of the full {cfg.name} workload ({scan.n_pos} patterns), "
                         f"FP64 NumPy oracle, single thread, {cpu_dt:.1f} s"}
    value = scan.n_pos * args.steps / dt
    line = {
        "metric": "diffraction-pattern projections/s (P_D+P_C) at 1 GPU",
        "value": round(value, 1),
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if args.storage == "fp32" else "fp16-storage/fp32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "object": [cfg.obj_h, cfg.obj_w], "n": cfg.n, "positions": scan.n_pos,
                   "algorithm": f"{args.algorithm}({args.param})" if args.algorithm in ("RAAR", "RRR", "TLAMBDA")
                   else args.algorithm,
                   "abc": list(abc), "blind": True, "storage": args.storage, "accumulate": "fp64",
                   "metrics": ("fourier, consistency and change errors every iteration" if full_metrics
                               else "fourier error every iteration"),
                   "exit_wave_state": "w = (1-a) x + a(1-b) y" if pk.uses_blend_form(cfg.n, abc[0], abc[1],
                                                                                     full_metrics) else "x",
                   "concur_sweeps": args.concur_sweeps,
                   "schedule": (f"{args.algorithm} parameter linear {args.param} -> {args.param_end}"
                                if sched is not None else "constant"),
                   "photons": cfg.photons, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "metrics_last": m,
    }
    g.close()
    print(json.dumps(line), flush=True)


def _make_request(i):
    """Worker: one request of the served mixed load (ptysynth recipe, seeded by i)."""
    import numpy as np
    from ptysynth import make_request, make_scan
    from paper_2311_11466_amd.serve import request_from_scan
    cfg, algo, prm = make_request(i)
    sc = make_scan(cfg, intensity_dtype=np.float32)
    return request_from_scan(i, sc, algo, prm, max_iter=200, tol=1e-3)


def bench_served(args):
    """Served mixed load: Poisson arrivals at a fraction of the closed-loop capacity."""
    import multiprocessing as mp
    import numpy as np
    import torch
    from paper_2311_11466_amd.serve import Server, poisson_arrivals
    torch.cuda.set_device(0)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        reqs = pool.map(_make_request, range(args.requests))
    print(f"# generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s on {workers} cores",
          file=sys.stderr, flush=True)
    warm = Server(budget_bytes=args.budget_gb * 1e9, max_slots=args.slots, chunk=10)
    warm.run([reqs[0]])
    for r in reqs:
        r.arrival = 0.0
    closed = Server(budget_bytes=args.budget_gb * 1e9, max_slots=args.slots, chunk=10).run(reqs)
    capacity = len(reqs) / closed.wall
    arr = poisson_arrivals(len(reqs), args.rate_factor * capacity, seed=501)
    for r, t in zip(reqs, arr):
        r.arrival = float(t)
    opened = Server(budget_bytes=args.budget_gb * 1e9, max_slots=args.slots, chunk=10).run(reqs)
    s = opened.summary()
    line = {
        "metric": "served mixed load: p50/p99 latency and aggregate projections/s at 1 GPU",
        "value": round(s["projections_per_s"], 1), "unit": "projections/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic",
        "p50_latency_s": round(s["p50_latency_s"], 4), "p99_latency_s": round(s["p99_latency_s"], 4),
        "closed_loop": {"requests_per_s": round(capacity, 3),
                        "projections_per_s": round(closed.summary()["projections_per_s"], 1)},
        "config": {"workload": "served", "requests": len(reqs), "arrival_rate_per_s": round(args.rate_factor * capacity, 3),
                   "rate_factor": args.rate_factor, "budget_gb": args.budget_gb, "slots": args.slots,
                   "chunk": 10, "max_iter": 200, "tol_fourier_err": 1e-3,
                   "n_mix": {str(n): sum(r.n == n for r in reqs) for n in (64, 128, 256)},
                   "peak_active": s["peak_active"], "peak_workspace_gb": round(s["peak_workspace_bytes"] / 1e9, 2)},
        "iterations": [r.iterations for r in opened.results],
    }
    print(json.dumps(line), flush=True)


def bench_sp(args):
    """Sequential projections on the same scan: one step = one SP iteration
    (every position once, in ascending order, batched by dependency level)."""
    import numpy as np
    import torch
    import paper_2311_11466_amd as pk
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    scan = make_workload(args.workload)
    cfg = scan.config
    g = pk.Scan(torch.as_tensor(scan.pos).to(dev), torch.as_tensor(scan.intensity).to(dev),
                torch.as_tensor(scan.obj0.astype(np.complex64)).to(dev),
                torch.as_tensor(scan.probe0.astype(np.complex64)).to(dev), blind=True, device=dev)
    from paper_2311_11466_amd.sp import disjoint_order
    order = disjoint_order(scan.pos, cfg.n) if args.sp_order == "colour" else None
    nb = 0
    for _ in range(args.warmup):
        nb = g.sp_iterate(order, args.sp_max_batch, args.sp_alpha, args.sp_beta)
    torch.cuda.synchronize()
    every = profile_every(args.steps)
    n_sampled = sampled_iterations(g.iteration, args.steps, every)
    g.profile(True, every=every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sp_iterate(order, args.sp_max_batch, args.sp_alpha, args.sp_beta)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = g.profile_read()
    m = g.metrics(allow_diverged=True)
    g.close()
    nn = cfg.n * cfg.n
    per_batch = scan.n_pos / max(nb, 1)
    bytes_per = {"divide": 20 * nn * per_batch, "probe": 8 * nn * per_batch + 16 * nn}
    names = {"divide": "divide_fused_kernel (sequential-projection mode)", "probe": "sp_probe_kernel"}
    kernels = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_us = ms / cnt * 1e3
        b = bytes_per.get(k)
        kernels[names.get(k, k)] = {"avg_us": round(avg_us, 3), "launches": cnt,
                                    "share": round(ms / n_sampled * args.steps / (dt * 1e3), 4),
                                    "algorithmic_bytes": round(b) if b else None,
                                    "GBs": round(b / (avg_us * 1e-6) / 1e9, 1) if b else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    d = kernels[dom]
    line = {
        "metric": "diffraction-pattern projections/s (sequential projections) at 1 GPU",
        "value": round(scan.n_pos * args.steps / dt, 1),
        "unit": "projections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": cfg.name, "method": "sequential projections", "positions": scan.n_pos, "n": cfg.n,
                   "order": "colour classes of the overlap graph" if order is not None else "ascending",
                   "batches_per_iteration": nb, "max_batch": args.sp_max_batch,
                   "alpha": args.sp_alpha, "beta": args.sp_beta, "blind": True},
        "roofline": {"bound": "hbm", "achieved": d["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(d["GBs"] / HBM_PEAK_GBS, 4) if d["GBs"] else None, "traffic": None,
                     "kernel": dom, "avg_us": d["avg_us"]},
        "kernels": kernels,
        "metrics_last": m,
    }
    print(json.dumps(line), flush=True)


def bench_compare(args):
    """Algorithm comparison (error lines of the presets, big and small probe).

    args.steps iterations per algorithm from the standard start; per algorithm
    the mean object error (against the truth, global complex scale removed) and
    Fourier error over the last 20 iterations, the ranking by object error and
    the uninstrumented time per iteration.  Full curves go to --curves-out.
    """
    import numpy as np
    import torch
    from ptysynth import make_scan, comparison_config
    from paper_2311_11466_amd.compare import ALGORITHMS, error_lines, summary
    torch.cuda.set_device(0)
    result, curves = {}, {}
    for probe in ("big", "small"):
        cfg = comparison_config(probe)
        sc = make_scan(cfg, intensity_dtype=np.float32)
        t0 = time.perf_counter()
        algs = list(ALGORITHMS) + [("TLAMBDA", lam) for lam in (0.3, 0.7, 0.9)] + [("RAAR", 0.9)]
        lines = error_lines(sc.pos, sc.intensity, sc.obj0, sc.probe0, sc.obj_true, sc.metric_box(),
                            algorithms=algs, n_iter=args.steps, sweeps=args.concur_sweeps)
        print(f"# {cfg.name}: {len(lines)} algorithms x {args.steps} iterations in "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        result[probe] = summary(lines)
        result[probe]["config"] = {"object": [cfg.obj_h, cfg.obj_w], "n": cfg.n, "positions": sc.n_pos,
                                   "probe_radius": cfg.probe_radius, "step": cfg.step, "photons": cfg.photons,
                                   "error_box": list(sc.metric_box())}
        curves[probe] = lines
    line = {
        "metric": "error lines of the presets: object error vs truth and Fourier error per iteration",
        "config": {"workload": "compare (big and small probe)", "iterations": args.steps,
                   "concur_sweeps": args.concur_sweeps, "storage": "fp32", "blind": True},
        "data": "synthetic",
        "big": result["big"],
        "small": result["small"],
    }
    if args.curves_out:
        with open(args.curves_out, "w") as fh:
            json.dump(curves, fh)
    print(json.dumps(line), flush=True)


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int):
    """Turn two rocprofv3 --pmc counter CSVs into the traffic file bench.py reads.

    FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by the
    ratio of known bytes to the same counter's reading on the calibration
    kernel (torch's elementwise add of two copy_bytes arrays into a third:
    2 * copy_bytes read, copy_bytes written).
    """
    import csv
    import statistics

    def read(path, counter):
        rows = {}
        files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True) \
            if os.path.isdir(path) else [path]
        for f in files:
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") != counter:
                        continue
                    rows.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return rows
    fetch = read(fetch_csv, "FETCH_SIZE")
    write = read(write_csv, "WRITE_SIZE")

    def pick(rows, key):
        vals = [v for k, vs in rows.items() if key in k for v in vs]
        return statistics.median(vals) if vals else None
    copy_key = "CUDAFunctor_add"
    f_copy = pick(fetch, copy_key)
    w_copy = pick(write, copy_key)
    f_scale = 2 * copy_bytes / (f_copy * 1024) if f_copy else None
    w_scale = copy_bytes / (w_copy * 1024) if w_copy else None
    src_hash = kernel_source_hash()
    from ptysynth.scans import CONFIGS
    n = CONFIGS[workload].n
    for cls in KERNEL_NAMES:
        kname = kernel_name(cls, n)
        f = pick(fetch, kname)
        w = pick(write, kname)
        if f is None or w is None or f_scale is None or w_scale is None:
            continue
        out = {"kernel": kname, "workload": workload, "source_hash": src_hash,
               "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
               "copy_bytes": copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
               "fetch_scale": f_scale, "write_scale": w_scale,
               "bytes_per_launch": round(f * 1024 * f_scale + w * 1024 * w_scale)}
        path = TRAFFIC_FILE.format(kernel=cls, workload=workload)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", path, out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="scan_n128",
                    choices=["scan_n128", "large_n256", "tiny_n32", "served", "compare"])
    ap.add_argument("--curves-out", default=None, help="compare: write the full error lines here (JSON)")
    ap.add_argument("--method", default="abc", choices=["abc", "sp"],
                    help="abc: the generalised iteration; sp: sequential projections")
    ap.add_argument("--sp-max-batch", type=int, default=0)
    ap.add_argument("--sp-order", default="colour", choices=["colour", "ascending"])
    ap.add_argument("--sp-alpha", type=float, default=1.0)
    ap.add_argument("--sp-beta", type=float, default=1.0)
    ap.add_argument("--concur-sweeps", type=int, default=1, help="(object, probe) sweeps per concur step")
    ap.add_argument("--schedule", default="constant", choices=["constant", "linear"],
                    help="linear: the preset parameter moves from --param to --param-end")
    ap.add_argument("--param-end", type=float, default=0.3)
    ap.add_argument("--metrics", default="all", choices=["all", "fourier"],
                    help="all: Fourier, consistency and change errors every iteration; "
                         "fourier: the Fourier error only (N <= 64: enables the blend form)")
    ap.add_argument("--requests", type=int, default=256, help="served: number of requests")
    ap.add_argument("--rate-factor", type=float, default=0.7, help="served: arrival rate / closed-loop capacity")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="served: HBM budget")
    ap.add_argument("--slots", type=int, default=32, help="served: concurrent scans")
    ap.add_argument("--algorithm", default="RAAR")
    ap.add_argument("--param", type=float, default=0.75)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run an elementwise add of known traffic (counter calibration)")
    ap.add_argument("--copy-probe-bytes", type=int, default=1 << 30)
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, args.copy_probe_bytes)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the whole scan runs on a single MI355X "
              "(sharding across GPUs is designed, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "served":
        bench_served(args)
    elif args.workload == "compare":
        bench_compare(args)
    elif args.method == "sp":
        bench_sp(args)
    else:
        bench(args)


if __name__ == "__main__":
    main()
