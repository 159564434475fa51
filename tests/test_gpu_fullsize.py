"""GPU parity at full workload sizes, in the launch configuration bench.py times.

scan_n128 (1024 patterns, N = 128, object 1024^2): a complete FP64 oracle
iteration from the same float32 state (a few seconds on the host).

large_n256 (4096 patterns, N = 256, object 4096^2): a complete FP64 oracle
iteration as well (about a minute and some 30 GB of host memory), every
output and the three metrics.
"""
import numpy as np
import pytest

from gpu_helpers import rel_l2, gpu_scan, amp32, covered_mask, to_dev, trajectory_bound, PERTURB
from oracle import pty_oracle as po
from ptysynth import make_scan

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _start_state(scan):
    """A realistic state: exit waves of the true object and probe (the data are noisy, so
    this is not a fixed point) with the start object and probe."""
    x = po.exit_waves(scan.obj_true.astype(np.complex64), scan.probe_true.astype(np.complex64),
                      scan.pos).astype(np.complex64)
    return x, scan.obj0.astype(np.complex64), scan.probe0.astype(np.complex64)


@pytest.mark.timeout(300)
def test_full_step_scan_n128():
    scan = make_scan("scan_n128", intensity_dtype=np.float32)
    abc = po.preset("RAAR", 0.75)
    print("case: full-size single step scan_n128 RAAR", flush=True)
    x, o, p = _start_state(scan)
    g = gpu_scan(scan)
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    g.set_algorithm_named("RAAR", 0.75)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    m = g.metrics()
    g.close()
    st = po.State(x.astype(np.complex128), o.astype(np.complex128), p.astype(np.complex128), 0)
    new, info = po.step(st, amp32(scan), scan.pos, *abc, blind=True)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x),
            "obj": rel_l2(o1, new.obj, covered_mask(scan)), "probe": rel_l2(p1, new.probe)}
    print("  errors", errs, flush=True)
    assert max(errs.values()) <= TOL, errs
    om = info["metrics"]
    for key in ("fourier_err", "consistency_err", "change"):
        assert abs(m[key] - om[key]) <= 1e-4 * abs(om[key]), (key, m[key], om[key])


@pytest.mark.timeout(900)
def test_full_step_large_n256():
    """A complete oracle iteration at the largest size (4096 patterns of 256^2
    on a 4096^2 object, the launch configuration bench.py times): every
    pattern's y and x_{k+1}, the whole object and probe, and the three metrics.
    The oracle step takes about a minute and some 30 GB of host memory."""
    scan = make_scan("large_n256", intensity_dtype=np.float32)
    name, prm = "RAAR", 0.75
    abc = po.preset(name, prm)
    print("case: full-size single step large_n256 RAAR", flush=True)
    x, o, p = _start_state(scan)
    g = gpu_scan(scan)
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    g.set_algorithm_named(name, prm)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    m = g.metrics()
    g.close()
    st = po.State(x.astype(np.complex128), o.astype(np.complex128), p.astype(np.complex128), 0)
    del x
    new, info = po.step(st, amp32(scan), scan.pos, *abc, blind=True)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x),
            "obj": rel_l2(o1, new.obj, covered_mask(scan)), "probe": rel_l2(p1, new.probe)}
    print("  errors", errs, flush=True)
    om = info["metrics"]
    print("  metrics gpu", m, "oracle", om, flush=True)
    assert max(errs.values()) <= TOL, errs
    for key in ("fourier_err", "consistency_err", "change"):
        assert abs(m[key] - om[key]) <= 1e-4 * abs(om[key]), (key, m[key], om[key])


@pytest.mark.timeout(300)
def test_full_two_steps_scan_n128_fourier_only():
    """Fourier-only metrics at full size (`bench.py --metrics fourier`: the x form with
    the split-exchange divide and no consistency or change partials), two iterations
    against two oracle iterations."""
    scan = make_scan("scan_n128", intensity_dtype=np.float32)
    abc = po.preset("RAAR", 0.75)
    print("case: full-size two steps scan_n128 RAAR, Fourier-only metrics", flush=True)
    x, o, p = _start_state(scan)
    g = gpu_scan(scan, full_metrics=False)
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    g.set_algorithm(*abc)
    g.iterate(2)
    x2, y1, o2, p2 = (t.cpu().numpy() for t in g.get_state())
    hist = g.metric_history()
    g.close()
    amp = amp32(scan)
    cov = covered_mask(scan)

    def two_steps(x_start):
        st = po.State(x_start.astype(np.complex128), o.astype(np.complex128), p.astype(np.complex128), 0)
        s1, i0 = po.step(st, amp, scan.pos, *abc, blind=True)
        s2, i1 = po.step(s1, amp, scan.pos, *abc, blind=True)
        return s2, i0, i1

    s2, i0, i1 = two_steps(x)
    errs = {"y": rel_l2(y1, i1["y"]), "x": rel_l2(x2, s2.x), "obj": rel_l2(o2, s2.obj, cov),
            "probe": rel_l2(p2, s2.probe)}
    # the second concur divides by overlap sums that, at the edge of the scanned
    # area, lie just above the guard (about 5e-11 against 1.6e-11 here), so the
    # object there amplifies any rounding: linearised two-iteration bound from
    # the gate and the oracle's own response to a 1e-7 perturbation of the start
    rng = np.random.default_rng(1)
    q2, _, qi = two_steps(x * (1 + PERTURB * rng.standard_normal(x.shape)))
    drift = {"y": rel_l2(qi["y"], i1["y"]), "x": rel_l2(q2.x, s2.x), "obj": rel_l2(q2.obj, s2.obj, cov),
             "probe": rel_l2(q2.probe, s2.probe)}
    tol = {k: float(trajectory_bound(v, 2)) for k, v in drift.items()}
    print("  errors", errs, "bounds", tol, flush=True)
    assert all(errs[k] <= tol[k] for k in errs), (errs, tol)
    for m, info in zip(hist, (i0, i1)):
        ef = info["metrics"]["fourier_err"]
        assert abs(m["fourier_err"] - ef) <= 1e-4 * ef, (m["fourier_err"], ef)


@pytest.mark.timeout(300)
def test_full_step_scan_n128_fp16():
    """FP16 exit-wave storage at full size (`bench.py --storage fp16`), from the
    float16-rounded start; bound 2e-3 (float16 unit roundoff 2^-11 per stored
    component, a few stores per iteration)."""
    scan = make_scan("scan_n128", intensity_dtype=np.float32)
    abc = po.preset("RAAR", 0.75)
    print("case: full-size single step scan_n128 RAAR, fp16 storage", flush=True)
    x, o, p = _start_state(scan)
    g = gpu_scan(scan, storage="fp16")
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    xs = g.get_state()[0].cpu().numpy()            # the stored (float16-rounded) start
    g.set_algorithm(*abc)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    st = po.State(xs.astype(np.complex128), o.astype(np.complex128), p.astype(np.complex128), 0)
    new, info = po.step(st, amp32(scan), scan.pos, *abc, blind=True)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x),
            "obj": rel_l2(o1, new.obj, covered_mask(scan)), "probe": rel_l2(p1, new.probe)}
    print("  errors", errs, flush=True)
    assert max(errs.values()) < 2e-3, errs
