"""Served form: continuous batching of many reconstructions on one GPU.

Requests (a scan plus an algorithm) arrive over time.  The server admits a
request when a slot is free and its exact device workspace
(`pty_workspace_bytes`) fits in the remaining HBM budget, keeps every admitted
scan's state resident on the device, and advances all admitted scans together
on one stream: each tick runs up to `chunk` iterations of every scan through
`pty_iterate_many`, whose grouped launches run each kernel once for up to
eight scans of the same pattern size, so small scans share the GPU instead of
queueing behind each other.  After a tick (one synchronisation for all scans)
a scan whose Fourier error is below its tolerance, or that has run its
iteration limit, completes: its object and probe are copied out, its
workspace is released, and the next waiting request can take the slot.  The
completion decision is taken only every `chunk` iterations, so a request's
result does not depend on what else shares the GPU.

All arithmetic runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

from . import Scan, iterate_many, workspace_bytes


@dataclass
class Request:
    rid: int
    pos: np.ndarray                 # int32 [J, 2]
    intensity: np.ndarray           # float32 [J, N, N]
    obj0: np.ndarray                # complex64 [H, W]
    probe0: np.ndarray              # complex64 [N, N]
    algorithm: str                  # a named algorithm of the library (DC, AR, DR, SF, RAAR, RRR, TLAMBDA)
    param: float                    # its beta or lambda
    max_iter: int = 200
    tol: float = 1e-3               # completes once the Fourier error is below this
    arrival: float = 0.0            # seconds after the server starts
    storage: str = "fp32"

    @property
    def n(self) -> int:
        return int(self.intensity.shape[-1])

    @property
    def n_pos(self) -> int:
        return int(self.intensity.shape[0])

    def workspace(self) -> int:
        h, w = self.obj0.shape
        return workspace_bytes(self.n, self.n_pos, h, w, self.storage)


@dataclass
class Result:
    rid: int
    obj: np.ndarray
    probe: np.ndarray
    iterations: int
    fourier_err: float
    arrival: float
    admitted: float
    done: float
    projections: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Active:
    req: Request
    scan: Scan
    stream: object
    admitted: float
    ws: int


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    wall: float = 0.0
    ticks: int = 0
    peak_active: int = 0
    peak_bytes: int = 0

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        proj = sum(r.projections for r in self.results)
        return {
            "requests": len(self.results),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "projections_per_s": proj / self.wall if self.wall > 0 else 0.0,
            "wall_s": self.wall,
            "ticks": self.ticks,
            "peak_active": self.peak_active,
            "peak_workspace_bytes": self.peak_bytes,
        }


class Server:
    """Continuous-batching scheduler for scans on one GPU."""

    def __init__(self, budget_bytes: float = 200e9, max_slots: int = 32, chunk: int = 10,
                 device=None, clock=time.perf_counter):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.clock = clock
        self.stream = torch.cuda.Stream(device=self.device)   # all scans' work; default priority

    def _admit(self, req: Request, now: float) -> _Active:
        torch = self.torch
        stream = self.stream
        with torch.cuda.stream(stream):
            dev = self.device
            scan = Scan(torch.as_tensor(req.pos).to(dev, non_blocking=False),
                        torch.as_tensor(req.intensity).to(dev),
                        torch.as_tensor(req.obj0).to(dev), torch.as_tensor(req.probe0).to(dev),
                        storage=req.storage, blind=True, device=dev, stream=stream,
                        full_metrics=False)   # completion reads the Fourier error only
        scan.set_algorithm_named(req.algorithm, req.param)
        return _Active(req, scan, stream, now, scan.workspace_bytes)

    def _finish(self, a: _Active, now: float, ef: float) -> Result:
        obj = a.scan.object().cpu().numpy()
        prb = a.scan.probe().cpu().numpy()
        it = a.scan.iteration
        a.scan.close()
        return Result(a.req.rid, obj, prb, it, ef, a.req.arrival, a.admitted, now,
                      a.req.n_pos * it)

    def run(self, requests: Sequence[Request]) -> ServeStats:
        """Serve all requests (each becomes visible at its arrival time)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if r.workspace() > self.budget:
                raise ValueError(f"request {r.rid} needs more than the whole HBM budget")
        active: list = []
        used = 0
        stats = ServeStats()
        t0 = self.clock()
        qi = 0
        while qi < len(pending) or active:
            now = self.clock() - t0
            # admit, in arrival order, whatever has arrived and fits
            while qi < len(pending) and pending[qi].arrival <= now and len(active) < self.max_slots:
                need = pending[qi].workspace()
                if used + need > self.budget:
                    break
                active.append(self._admit(pending[qi], now))
                used += need
                qi += 1
            stats.peak_active = max(stats.peak_active, len(active))
            stats.peak_bytes = max(stats.peak_bytes, used)
            if not active:
                # idle until the next arrival
                wait = pending[qi].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            # one tick: every active scan advances, interleaved, to the nearest
            # checkpoint of any of them; a scan is tested only at its own
            # checkpoints (multiples of chunk, or its iteration limit)
            its = [a.scan.iteration for a in active]
            n = min(min(self.chunk - it % self.chunk, a.req.max_iter - it) for a, it in zip(active, its))
            iterate_many([a.scan for a in active], n)
            stats.ticks += 1
            self.stream.synchronize()                     # one wait for every scan of the tick
            still = []
            for a, it in zip(active, its):
                it += n
                if it % self.chunk != 0 and it < a.req.max_iter:
                    still.append(a)
                    continue
                m = a.scan.metrics(allow_diverged=True)   # already complete
                ef = m["fourier_err"]
                done = it >= a.req.max_iter or not np.isfinite(ef) or ef < a.req.tol
                if done:
                    stats.results.append(self._finish(a, self.clock() - t0, ef))
                    used -= a.ws
                else:
                    still.append(a)
            active = still
        stats.wall = self.clock() - t0
        stats.results.sort(key=lambda r: r.rid)
        return stats


def request_from_scan(rid: int, scan, algorithm: str, param: float, arrival: float = 0.0,
                      max_iter: int = 200, tol: float = 1e-3, storage: str = "fp32") -> Request:
    """Build a Request from a ptysynth Scan."""
    return Request(rid, scan.pos.astype(np.int32), scan.intensity.astype(np.float32),
                   scan.obj0.astype(np.complex64), scan.probe0.astype(np.complex64),
                   algorithm, float(param), max_iter, tol, arrival, storage)


def poisson_arrivals(n: int, rate: float, seed: int = 501) -> np.ndarray:
    """Arrival times of n requests at `rate` per second (exponential gaps, seeded)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


__all__ = ["Request", "Result", "Server", "ServeStats", "request_from_scan", "poisson_arrivals"]
