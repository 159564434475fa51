#!/usr/bin/env python3
"""Throughput of the generalised 'abc' set-projection iteration on one MI355X.

A step is one full iteration of the hot path over every diffraction pattern
of the workload: divide (the pending update, forward DFT, relaxed modulus
projection, inverse DFT), concur (object and probe overlap consensus in
float64) and the metric finalisation.  The metric is diffraction-pattern
projections per second, J * steps / time, with every input resident in HBM
before the timed region starts.

Default workload: large_n256 -- object 4096 x 4096, N = 256, J = 4096
positions (64 x 64 raster, step 56, +-3 jitter), Poisson data at 1e4 photons
per pattern, blind RAAR (beta = 0.75), float32 exit waves with float64
overlap sums, all three metrics every iteration.  scan_n128 (object 1024^2,
N = 128, J = 1024, 1e6 photons) is measured beside it.  Inputs are seeded
and synthetic (ptysynth).

Timing: the timed region holds only the iterations (no per-kernel events);
kernel durations come from a second pass of the same iterations with a HIP
event pair on the scan's stream around every launch.  The roofline line is
the divide (the dominant kernel; at N = 256 its three passes together) at its
algorithmic bytes: read x, y and sqrt(I), write x and y, 36 B per pattern
pixel in float32; the whole iteration's fraction at 52 B per pattern pixel
(blind) is given beside it.  `traffic` is the divide's measured HBM bytes per
iteration from rocprofv3 FETCH_SIZE / WRITE_SIZE counters (profiles/), null
if the kernel sources or the run settings differ from those the counters were
taken with.  The CPU baseline is the FP64 oracle on a bounded sample of the
same workload, on one core and on 16 (one single-threaded copy per core).

  python bench.py [--steps K] [--warmup W] [--workload large_n256|scan_n128|tiny_n32|served|compare]
                  [--storage fp16] [--metrics fourier] [--method sp] [--also none]
  python bench.py --workload X --storage S --summarize-pmc FETCH_DIR WRITE_DIR
                  (writes the traffic files under profiles/)
  python bench.py --summarize-ktrace STATS_CSV TITLE COMMAND
                  (a markdown summary of a rocprofv3 kernel_stats.csv)
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
DIVIDE_CLASSES = ("divide", "divide_cols", "divide_rows_inv")


def kernel_name(cls: str, n: int) -> str:
    """The HIP kernel behind a kernel class at pattern size n."""
    if n == 256 and cls == "divide":
        return "rows256_fwd_kernel"
    if n == 256 and cls == "object":
        return "object_update_kernel"
    return KERNEL_NAMES[cls]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{kernel}_{workload}_{storage}.json")
PROFILE_STEPS = 50       # iterations of the kernel-timing pass (at most)

KERNEL_SOURCES = [os.path.join(ROOT, "paper_2311_11466_amd", "csrc", f)
                  for f in ("divide.hip", "divide_fused.hpp", "divide_ops.hpp", "divide_n32.hip", "divide_n64.hip",
                            "divide_n128.hip", "concur.hip", "common.hpp", "params.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, n: int, J: int, abc, blind: bool, storage: str, full_metrics: bool, form: str):
    """Algorithmic HBM bytes of one iteration's kernel class (roofline numerator).

    Per pattern pixel, with e the exit-wave element size (8 B float32, 4 B
    float16): the divide reads x_{k-1} (when 1-a != 0 or the metrics need it),
    y_{k-1} (when a(1-b) != 0 or the metrics need it) and sqrt(I) (4 B), and
    writes x_k (same condition as its read) and y_k; in the blend form
    (form "w") it reads w_{k-1} and sqrt(I) and writes w_k and y_k.  The
    object and probe steps read y once each (the probe step only when blind).
    Object and probe gathers and the float64 partial sums are cache-resident
    or small and are not counted; neither is the float32 intermediate of the
    N = 256 passes (traffic the method does not need).
    """
    a, b, _ = abc
    e = 4 if storage == "fp16" else 8
    nn = n * n * J
    if kind == "divide":
        if form == "w":
            return (e + 4 + e + e) * nn
        rx = e if (abs(1 - a) > 0 or full_metrics) else 0
        ry = e if (abs(a * (1 - b)) > 0 or full_metrics) else 0
        return (rx + ry + 4 + rx + e) * nn
    if kind == "object":
        return e * nn
    if kind == "probe":
        return e * nn if blind else 0
    return 0


def make_workload(name: str):
    import numpy as np
    from ptysynth import make_scan
    return make_scan(name, intensity_dtype=np.float32)


# --------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands
# --------------------------------------------------------------------------
def cpu_sample(scan, max_patterns: int):
    """A bounded sample of the workload for the oracle: the whole scan if it has
    at most max_patterns patterns, else the leading square block of the raster
    (its object cropped to the block's windows).  Returns (pos, amp, obj0,
    probe0, description)."""
    import numpy as np
    cfg = scan.config
    pos = np.asarray(scan.pos)
    amp = np.sqrt(scan.intensity.astype(np.float64))
    if scan.n_pos <= max_patterns:
        return pos, amp, scan.obj0, scan.probe0, f"the whole {cfg.name} scan ({scan.n_pos} patterns)"
    rows, cols = cfg.raster
    side = int(np.sqrt(max_patterns))
    idx = np.array([r * cols + c for r in range(side) for c in range(side)])
    sub = pos[idx]
    r0, c0 = sub.min(axis=0)
    r1, c1 = sub.max(axis=0) + scan.n
    return (sub - [r0, c0], amp[idx], scan.obj0[r0:r1, c0:c1].copy(), scan.probe0,
            f"the leading {side} x {side} block of the {cfg.name} raster ({len(idx)} of {scan.n_pos} patterns "
            f"of {scan.n}^2, object cropped to {r1 - r0} x {c1 - c0})")


def _oracle_worker(path, abc, n_iter):
    """One oracle run of the sample stored at path (a file this benchmark wrote);
    returns its wall time."""
    import numpy as np
    from oracle import pty_oracle as po
    with np.load(path) as d:
        pos, amp, obj0, probe0 = d["pos"], d["amp"], d["obj0"], d["probe0"]
    st = po.init_state(obj0, probe0, pos)
    t0 = time.perf_counter()
    po.run(st, amp, pos, *abc, n_iter, blind=True)
    return time.perf_counter() - t0


def run_cpu_baseline(scan, abc, max_patterns: int, n_iter: int):
    """The oracle on one host core, and as one copy per core on all of them
    (aggregate projections/s of independent runs of the same sample)."""
    import multiprocessing as mp
    import tempfile
    import numpy as np
    pos, amp, obj0, probe0, what = cpu_sample(scan, max_patterns)
    fd, path = tempfile.mkstemp(suffix=".npz", dir="/tmp")
    os.close(fd)
    try:
        np.savez(path, pos=pos, amp=amp, obj0=obj0, probe0=probe0)
        t1 = _oracle_worker(path, abc, n_iter)
        one = len(pos) * n_iter / t1
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            times = pool.starmap(_oracle_worker, [(path, abc, n_iter)] * cores)
        wall = time.perf_counter() - t0
        allc = cores * len(pos) * n_iter / max(max(times), 1e-9)
    finally:
        os.unlink(path)
    return {"value": round(allc, 2), "unit": "projections/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_iter} iterations of {what}, FP64 NumPy oracle, one single-threaded copy per core "
                      f"on {cores} cores ({wall:.1f} s wall; slowest copy {max(times):.1f} s)",
            "one_core": round(one, 2), "one_core_s": round(t1, 1)}


def traffic_run(args) -> dict:
    """The settings that decide which kernel variant runs (its traffic)."""
    return {"storage": args.storage, "algorithm": args.algorithm, "param": args.param, "metrics": args.metrics,
            "concur_sweeps": args.concur_sweeps, "schedule": args.schedule}


def load_traffic(cls: str, workload: str, run: dict):
    path = TRAFFIC_FILE.format(kernel=cls, workload=workload, storage=run["storage"])
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None      # the kernel changed since the counters were taken
    if t.get("run") != run:
        return None      # counters of another kernel variant
    return t.get("bytes_per_launch")


def measure(args, workload: str, steps: int, warmup: int):
    """Create the scan, run warm-up, the timed region and the kernel-timing
    pass.  Returns the measurement record (no CPU baseline)."""
    import numpy as np
    import torch
    import paper_2311_11466_amd as pk

    dev = torch.device("cuda", 0)
    scan = make_workload(workload)
    cfg = scan.config
    full_metrics = args.metrics == "all"
    print(f"# workload {cfg.name}: object {cfg.obj_h}x{cfg.obj_w}, N={cfg.n}, J={scan.n_pos}", file=sys.stderr,
          flush=True)
    g = pk.Scan(torch.as_tensor(scan.pos).to(dev), torch.as_tensor(scan.intensity).to(dev),
                torch.as_tensor(scan.obj0.astype(np.complex64)).to(dev),
                torch.as_tensor(scan.probe0.astype(np.complex64)).to(dev),
                storage=args.storage, blind=True, device=dev, full_metrics=full_metrics)
    g.set_algorithm_named(args.algorithm, args.param)
    abc = pk.algorithm_abc(args.algorithm, args.param)
    g.set_concur_sweeps(args.concur_sweeps)
    sched = None
    n_prof = min(steps, PROFILE_STEPS)
    if args.schedule == "linear":
        # the preset's parameter (beta or lambda) moves linearly from --param to
        # --param-end over warm-up and timed iterations; the kernel pass repeats
        # the timed part of the schedule
        n_all = warmup + steps
        sched = [pk.algorithm_abc(args.algorithm, args.param + (args.param_end - args.param) * i / max(n_all - 1, 1))
                 for i in range(n_all)]
        g.iterate_schedule(sched[:warmup])
    else:
        g.iterate(warmup)
    form = g.state_form()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if sched is not None:
        g.iterate_schedule(sched[warmup:])
    else:
        g.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m = g.metrics(allow_diverged=True)
    print(f"# timed {steps} steps in {dt * 1e3:.2f} ms; last metrics {m}", file=sys.stderr, flush=True)
    # kernel-timing pass: the same iterations with an event pair around every launch
    g.profile(True, every=1)
    if sched is not None:
        g.iterate_schedule(sched[warmup:warmup + n_prof])
    else:
        g.iterate(n_prof)
    prof = g.profile_read()
    g.profile(False)
    g.close()

    kernels = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        per_iter_us = ms / n_prof * 1e3
        kernels[k] = {"kernel": kernel_name(k, cfg.n), "avg_us": round(ms / cnt * 1e3, 3), "launches": cnt,
                      "us_per_iteration": round(per_iter_us, 3),
                      "share": round(per_iter_us / (dt / steps * 1e6), 4)}
    units = {}
    div = [k for k in DIVIDE_CLASSES if k in kernels]
    div_us = sum(kernels[k]["us_per_iteration"] for k in div)
    units["divide"] = (div_us, algorithmic_bytes("divide", cfg.n, scan.n_pos, abc, True, args.storage,
                                                 full_metrics, form))
    for k in ("object", "probe"):
        if k in kernels:
            units[k] = (kernels[k]["us_per_iteration"],
                        algorithmic_bytes(k, cfg.n, scan.n_pos, abc, True, args.storage, full_metrics, form))
    for k, (us, nbytes) in units.items():
        rec = kernels.setdefault(k, {})
        if k == "divide" and len(div) > 1:
            rec = kernels["divide_all_passes"] = {"kernels": [kernels[c]["kernel"] for c in div],
                                                  "us_per_iteration": round(us, 3)}
        rec["algorithmic_bytes"] = nbytes
        rec["GBs"] = round(nbytes / (us * 1e-6) / 1e9, 1) if nbytes else None
        rec["frac"] = round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if nbytes else None
    traffic = [load_traffic(c, cfg.name, traffic_run(args)) for c in div]
    d_us, d_bytes = units["divide"]
    roofline = {"bound": "hbm", "achieved": round(d_bytes / (d_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d_bytes / (d_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": (sum(traffic) if all(t is not None for t in traffic) else None),
                "kernel": " + ".join(kernel_name(c, cfg.n) for c in div), "avg_us": round(d_us, 3),
                "algorithmic_bytes_per_launch": d_bytes}
    it_bytes = sum(v[1] for v in units.values())
    ms_step = dt / steps * 1e3
    iteration = {"algorithmic_bytes": it_bytes, "ms": round(ms_step, 4),
                 "achieved_GBs": round(it_bytes / (ms_step * 1e-3) / 1e9, 1),
                 "frac": round(it_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return {"scan": scan, "cfg": cfg, "abc": abc, "form": form, "full_metrics": full_metrics, "sched": sched,
            "dt": dt, "steps": steps, "value": scan.n_pos * steps / dt, "ms_per_step": ms_step,
            "roofline": roofline, "iteration_roofline": iteration, "kernels": kernels, "metrics_last": m,
            "profile_steps": n_prof}


def bench(args):
    import torch
    torch.cuda.set_device(0)
    r = measure(args, args.workload, args.steps, args.warmup)
    scan, cfg, abc = r["scan"], r["cfg"], r["abc"]
    also = {}
    if args.also and args.also != args.workload:
        o = measure(args, args.also, args.also_steps, args.warmup)
        also[args.also] = {"value": round(o["value"], 1), "unit": "projections/s", "steps": o["steps"],
                           "ms_per_step": round(o["ms_per_step"], 4), "roofline": o["roofline"],
                           "iteration_roofline": o["iteration_roofline"],
                           "config": {"object": [o["cfg"].obj_h, o["cfg"].obj_w], "n": o["cfg"].n,
                                      "positions": o["scan"].n_pos}}
        del o
    if args.copy_probe:
        # a plain elementwise kernel of known traffic (reads 2 B, writes B bytes), for
        # scaling the rocprofv3 FETCH_SIZE / WRITE_SIZE counters
        nf = args.copy_probe_bytes // 4
        a = torch.ones(nf, dtype=torch.float32, device="cuda")
        b = torch.ones(nf, dtype=torch.float32, device="cuda")
        c = torch.empty(nf, dtype=torch.float32, device="cuda")
        for _ in range(3):
            torch.add(a, b, out=c)
        torch.cuda.synchronize()
        del a, b, c
    cpu = None
    if not args.no_cpu_baseline:
        if cfg.n >= 256:
            cpu = run_cpu_baseline(scan, abc, max_patterns=256, n_iter=6)
        else:
            cpu = run_cpu_baseline(scan, abc, max_patterns=1024, n_iter=3 if cfg.n >= 128 else 20)
    line = {
        "metric": "diffraction-pattern projections/s (P_D+P_C) at 1 GPU",
        "value": round(r["value"], 1),
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if args.storage == "fp32" else "fp16-storage/fp32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "object": [cfg.obj_h, cfg.obj_w], "n": cfg.n, "positions": scan.n_pos,
                   "algorithm": f"{args.algorithm}({args.param})" if args.algorithm in ("RAAR", "RRR", "TLAMBDA")
                   else args.algorithm,
                   "abc": list(abc), "blind": True, "storage": args.storage, "accumulate": "fp64",
                   "metrics": ("fourier, consistency and change errors every iteration" if r["full_metrics"]
                               else "fourier error every iteration"),
                   "exit_wave_state": "w = (1-a) x + a(1-b) y" if r["form"] == "w" else "x",
                   "concur_sweeps": args.concur_sweeps,
                   "schedule": (f"{args.algorithm} parameter linear {args.param} -> {args.param_end}"
                                if r["sched"] is not None else "constant"),
                   "photons": cfg.photons, "parallelism": "single GPU"},
        "roofline": r["roofline"],
        "iteration_roofline": r["iteration_roofline"],
        "cpu_baseline": cpu,
        "kernels": r["kernels"],
        "kernel_timing": f"HIP events around every launch in a separate pass of {r['profile_steps']} iterations",
        "metrics_last": r["metrics_last"],
        "also": also,
    }
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
    from paper_2311_11466_amd.sp import colour_classes, disjoint_order
    order = disjoint_order(scan.pos, cfg.n) if args.sp_order == "colour" else None
    if args.sp_beta is None:
        # the probe steps of a batch are summed: with beta = 1 a batch of b
        # windows moves the probe b single steps at once, which diverges for
        # the colour batches (the oracle's iteration as well); 1 / (mean batch
        # size) makes a batch's summed step about one step.  The ascending
        # order's batches hold a few windows: beta = 1.
        n_col = int(colour_classes(scan.pos, cfg.n).max()) + 1
        args.sp_beta = n_col / scan.n_pos if args.sp_order == "colour" else 1.0
    nb = 0
    for _ in range(args.warmup):
        nb = g.sp_iterate(order, args.sp_max_batch, args.sp_alpha, args.sp_beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sp_iterate(order, args.sp_max_batch, args.sp_alpha, args.sp_beta)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m = g.metrics(allow_diverged=True)
    # kernel-timing pass: the same iterations with an event pair around every launch
    n_sampled = min(args.steps, PROFILE_STEPS)
    g.profile(True, every=1)
    for _ in range(n_sampled):
        g.sp_iterate(order, args.sp_max_batch, args.sp_alpha, args.sp_beta)
    prof = g.profile_read()
    g.profile(False)
    g.close()
    nn = cfg.n * cfg.n
    per_batch = scan.n_pos / max(nb, 1)
    # per batch member pixel: sqrt(I) 4, object window read 8 and written 8,
    # probe step written 8; the probe kernel reads the steps and the probe and
    # writes the probe
    bytes_per = {"divide": 28 * nn * per_batch, "probe": 8 * nn * per_batch + 16 * nn}
    names = {"divide": ("sp256_rows_fwd_kernel + sp256_cols_kernel + sp256_rows_inv_kernel" if cfg.n == 256
                        else "divide_fused_kernel (sequential-projection mode)"), "probe": "sp_probe_kernel"}
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


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int, run: dict):
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
        out = {"kernel": kname, "workload": workload, "run": run, "source_hash": src_hash,
               "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
               "copy_bytes": copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
               "fetch_scale": f_scale, "write_scale": w_scale,
               "bytes_per_launch": round(f * 1024 * f_scale + w * 1024 * w_scale)}
        path = TRAFFIC_FILE.format(kernel=cls, workload=workload, storage=run["storage"])
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", path, out)


def summarize_ktrace(stats_csv: str, title: str, command: str):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = [f"# Kernel trace: {title}", "", "Command (after `cd /tmp && export TMPDIR=/tmp`; `<repo>` is the repository root):",
           "", "```", command, "```", "", "Durations from `kernel_stats.csv`:", "",
           "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share |", "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"] if len(r["Name"]) < 90 else r["Name"][:87] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / total:.1f} % |")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large_n256",
                    choices=["large_n256", "scan_n128", "tiny_n32", "served", "compare"])
    ap.add_argument("--also", default="scan_n128", choices=["scan_n128", "large_n256", "tiny_n32", "none"],
                    help="a second workload measured in the same run and reported under 'also'")
    ap.add_argument("--also-steps", type=int, default=100)
    ap.add_argument("--curves-out", default=None, help="compare: write the full error lines here (JSON)")
    ap.add_argument("--method", default="abc", choices=["abc", "sp"],
                    help="abc: the generalised iteration; sp: sequential projections")
    ap.add_argument("--sp-max-batch", type=int, default=0)
    ap.add_argument("--sp-order", default="colour", choices=["colour", "ascending"])
    ap.add_argument("--sp-alpha", type=float, default=1.0)
    ap.add_argument("--sp-beta", type=float, default=None,
                    help="SP probe step size (default: 1 / mean batch size for the colour order, else 1)")
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
    ap.add_argument("--summarize-ktrace", nargs=3, metavar=("STATS_CSV", "TITLE", "COMMAND"),
                    help="print a markdown summary of a rocprofv3 kernel_stats.csv")
    args = ap.parse_args()
    if args.also == "none":
        args.also = None
    if args.summarize_ktrace:
        summarize_ktrace(*args.summarize_ktrace)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, args.copy_probe_bytes,
                      traffic_run(args))
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
