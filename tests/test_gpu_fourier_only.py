"""GPU parity without full metrics (only the Fourier error every iteration).

The divide prologue then reads and writes only what (a, b, c) needs: DC and AR
(a = b = 1) form x = P S_j O and read nothing, SF (a = 1) reads y, RAAR reads
x and y (and forms the other two metrics since it reads their inputs anyway).
Each is its own kernel instantiation; at N = 128 they run with the split
exchanges, at N = 256 as three passes.  Two iterations from an identical state
(the second runs the pending form) against two oracle iterations; bound: 20 x
the oracle's own change under a 1e-7 perturbation of the start (at least
1e-5), since the second concur divides by overlap sums that are small at the
edge of the scanned area.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import (amp32, covered_mask, gpu_scan, oracle_state_after, rel_l2, round_state, to_dev,
                         trajectory_bound, PERTURB)
from oracle import pty_oracle as po
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu

TOL = 1e-5
_SCANS = {}


def get_scan(name):
    if name not in _SCANS:
        if name == "p64":
            _SCANS[name] = make_scan(small_config("p64", 64, 5, 24, jitter=2, photons=1e6, seed=31))
        elif name == "p128":
            _SCANS[name] = make_scan(small_config("p128", 128, 4, 40, jitter=2, photons=1e6, seed=41))
        elif name == "p256":
            _SCANS[name] = make_scan(small_config("p256", 256, 3, 80, jitter=3, photons=1e5, seed=51))
        else:
            raise KeyError(name)
    return _SCANS[name]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg", ["p64", "p128", "p256"])
@pytest.mark.parametrize("name,param", [("DC", 0.0), ("AR", 0.0), ("SF", 0.0), ("RAAR", 0.75)])
def test_fourier_only_two_steps(cfg, name, param):
    scan = get_scan(cfg)
    abc = po.preset(name, param)
    say("case: Fourier-only metrics, two steps", cfg, name, abc)
    st = round_state(oracle_state_after(scan, 2, po.preset("RAAR", 0.75)))
    g = gpu_scan(scan, full_metrics=False)
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))
    g.set_algorithm(*abc)
    g.iterate(2)
    x2, y1, o2, p2 = (t.cpu().numpy() for t in g.get_state())
    hist = g.metric_history()
    g.close()
    amp = amp32(scan)
    cov = covered_mask(scan)

    def two(x_start):
        s0 = po.State(x_start, st.obj, st.probe, st.k)
        s1, i0 = po.step(s0, amp, scan.pos, *abc)
        s2, i1 = po.step(s1, amp, scan.pos, *abc)
        return s2, i0, i1

    s2, i0, i1 = two(st.x)
    errs = {"y": rel_l2(y1, i1["y"]), "x": rel_l2(x2, s2.x), "obj": rel_l2(o2, s2.obj, cov),
            "probe": rel_l2(p2, s2.probe)}
    rng = np.random.default_rng(1)
    q2, _, qi = two(st.x * (1 + PERTURB * rng.standard_normal(st.x.shape)))
    drift = {"y": rel_l2(qi["y"], i1["y"]), "x": rel_l2(q2.x, s2.x), "obj": rel_l2(q2.obj, s2.obj, cov),
             "probe": rel_l2(q2.probe, s2.probe)}
    tol = {k: float(trajectory_bound(v, 2)) for k, v in drift.items()}
    say("  errors", {k: f"{v:.2e}" for k, v in errs.items()}, "bounds", {k: f"{v:.2e}" for k, v in tol.items()})
    assert all(errs[k] <= tol[k] for k in errs), (errs, tol)
    assert np.array_equal(o2[~cov], s2.obj[~cov].astype(np.complex64))
    assert len(hist) == 2
    for m, info in zip(hist, (i0, i1)):
        ef = info["metrics"]["fourier_err"]
        assert abs(m["fourier_err"] - ef) <= 1e-4 * ef, (m["fourier_err"], ef)
