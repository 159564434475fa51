"""Checkpoint and resume reproduce an uninterrupted run bit for bit, for every
named algorithm, pattern size, storage and metric setting (GPU).

A scan runs different divide prologue modes over its life: the first
iteration, the steady state (which buffers are read and written depends on
the algorithm, the metrics and the storage), and the first iteration after
pty_set_state, which starts from a materialised x.  Each mode is its own
kernel instantiation; resuming matches only if every instantiation rounds
every value the same way.  With float16 storage a checkpoint holds x_k as
stored (rounded to float16), so every prologue uses x_k in that form too.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_scan
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu

_SCANS = {}


def get_scan(name):
    if name not in _SCANS:
        if name == "tiny_n32":
            _SCANS[name] = make_scan("tiny_n32")
        elif name == "p64":
            _SCANS[name] = make_scan(small_config("p64", 64, 5, 24, jitter=2, photons=1e6, seed=31))
        elif name == "p128":
            _SCANS[name] = make_scan(small_config("p128", 128, 4, 40, jitter=2, photons=1e6, seed=41))
        else:
            _SCANS[name] = make_scan(small_config("p256", 256, 3, 80, jitter=3, photons=1e5, seed=51))
    return _SCANS[name]


PRESETS = [("DC", 0.0), ("AR", 0.0), ("DR", 0.0), ("SF", 0.0), ("RAAR", 0.75), ("RRR", 0.5), ("TLAMBDA", 0.5)]


def _run(scan, storage, full, algo, prm, n, state=None):
    g = gpu_scan(scan, storage=storage, full_metrics=full)
    if state is not None:
        g.set_state(*state)
    g.set_algorithm_named(algo, prm)
    g.iterate(n)
    st = g.get_state()
    g.close()
    return st


@pytest.mark.parametrize("full", [True, False], ids=["all_metrics", "fourier_only"])
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
@pytest.mark.parametrize("cfg", ["tiny_n32", "p64", "p128", "p256"])
def test_resume_every_preset(cfg, storage, full):
    scan = get_scan(cfg)
    for algo, prm in PRESETS:
        print(f"case: resume {cfg} {storage} full_metrics={full} {algo}({prm})", flush=True)
        sys.stdout.flush()
        ref = [t.cpu().numpy() for t in _run(scan, storage, full, algo, prm, 4)]
        ck = _run(scan, storage, full, algo, prm, 2)
        got = [t.cpu().numpy() for t in _run(scan, storage, full, algo, prm, 2, state=ck)]
        for name, r, q in zip("xyop", ref, got):
            assert np.array_equal(r.view(np.uint32), q.view(np.uint32)), (algo, name)
