"""Algorithm comparison: the error lines of the paper's Figs. 7-8.

Every preset of the generalised iteration (DC, AR, DR, SF, RAAR, RRR, T_lambda)
runs from the same start on the same scan; after each iteration the Fourier
error (from the library's metric history) and the object error against the
ground truth inside a box (``Scan.object_error``: global complex scale
removed) are recorded.  A second, uninstrumented run of each algorithm gives
its time per iteration.  All arithmetic runs in the HIP library; this module
only drives it.
"""
from __future__ import annotations

import time
from typing import Sequence

import numpy as np

from . import Scan, algorithm_abc

ALGORITHMS = (("DC", 0.0), ("AR", 0.0), ("DR", 0.0), ("SF", 0.0), ("RAAR", 0.75), ("RRR", 0.5),
              ("TLAMBDA", 0.5))


def label(name: str, param: float) -> str:
    return f"{name}({param:g})" if name in ("RAAR", "RRR", "TLAMBDA") else name


def error_lines(pos, intensity, obj0, probe0, truth, box, algorithms: Sequence = ALGORITHMS,
                n_iter: int = 300, sweeps: int = 1, storage: str = "fp32", device=None,
                timed: bool = True) -> dict:
    """Error lines of each algorithm.

    pos: int32 [J, 2]; intensity: float32 [J, N, N]; obj0, probe0: complex64
    start; truth: the true object (complex, [H, W]); box: (r0, r1, c0, c1) of
    the error area.  Returns {label: {"abc", "fourier_err", "object_err",
    "ms_per_iteration"}}.
    """
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    r0, r1, c0, c1 = box
    t_box = torch.as_tensor(np.ascontiguousarray(truth[r0:r1, c0:c1]).astype(np.complex64)).to(dev)
    args = (torch.as_tensor(np.asarray(pos, np.int32)).to(dev),
            torch.as_tensor(np.asarray(intensity, np.float32)).to(dev),
            torch.as_tensor(np.asarray(obj0, np.complex64)).to(dev),
            torch.as_tensor(np.asarray(probe0, np.complex64)).to(dev))
    out = {}
    for name, prm in algorithms:
        abc = algorithm_abc(name, prm)
        g = Scan(*args, storage=storage, blind=True, device=dev, full_metrics=False)
        g.set_algorithm_named(name, prm)
        g.set_concur_sweeps(sweeps)
        eo = []
        for _ in range(n_iter):
            g.iterate(1)
            eo.append(g.object_error(t_box, r0, c0))
        ef = [m["fourier_err"] for m in g.metric_history()]
        g.close()
        ms = None
        if timed:
            g = Scan(*args, storage=storage, blind=True, device=dev, full_metrics=False)
            g.set_algorithm_named(name, prm)
            g.set_concur_sweeps(sweeps)
            g.iterate(5)
            g.synchronize()
            t0 = time.perf_counter()
            g.iterate(n_iter)
            g.synchronize()
            ms = (time.perf_counter() - t0) / n_iter * 1e3
            g.close()
        out[label(name, prm)] = {"abc": list(abc), "fourier_err": ef, "object_err": eo, "ms_per_iteration": ms}
    return out


def summary(lines: dict, last: int = 20) -> dict:
    """Per algorithm the mean object and Fourier error over the last `last`
    iterations, and the algorithms ranked by that object error (best first)."""
    rows = {k: {"object_err": float(np.mean(v["object_err"][-last:])),
                "fourier_err": float(np.mean(v["fourier_err"][-last:])),
                "ms_per_iteration": v["ms_per_iteration"]} for k, v in lines.items()}
    return {"final": rows, "ranking": sorted(rows, key=lambda k: rows[k]["object_err"])}


__all__ = ["ALGORITHMS", "error_lines", "summary", "label"]
