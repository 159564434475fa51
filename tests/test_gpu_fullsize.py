"""GPU parity at full workload sizes, in the launch configuration bench.py times.

scan_n128 (1024 patterns, N = 128, object 1024^2): a complete FP64 oracle
iteration from the same float32 state (a few seconds on the host).

large_n256 (4096 patterns, N = 256, object 4096^2): too large for a complete
oracle step in a test, so the outputs are checked on samples the oracle can
compute one by one: y for sampled patterns (the divide from the known x), the
object at sampled pixels and every probe pixel from the GPU's own y (the
concur sums in float64), and x_{k+1} for sampled patterns from the GPU's new
object and probe.
"""
import numpy as np
import pytest

from gpu_helpers import rel_l2, gpu_scan, amp32, covered_mask, to_dev
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
    g.set_algorithm(*abc)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    st = po.State(x.astype(np.complex128), o.astype(np.complex128), p.astype(np.complex128), 0)
    new, info = po.step(st, amp32(scan), scan.pos, *abc, blind=True)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x),
            "obj": rel_l2(o1, new.obj, covered_mask(scan)), "probe": rel_l2(p1, new.probe)}
    print("  errors", errs, flush=True)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.timeout(600)
def test_sampled_step_large_n256():
    scan = make_scan("large_n256", intensity_dtype=np.float32)
    abc = po.preset("RAAR", 0.75)
    a, b, c = abc
    n = scan.n
    print("case: full-size sampled step large_n256 RAAR", flush=True)
    x, o, p = _start_state(scan)
    g = gpu_scan(scan)
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    g.set_algorithm(*abc)
    g.iterate(1)
    x1_d, y_d, o1_d, p1_d = g.get_state()
    g.close()
    y = y_d.cpu().numpy()
    del y_d
    o1 = o1_d.cpu().numpy()
    p1 = p1_d.cpu().numpy()
    rng = np.random.default_rng(9)
    J = scan.n_pos
    js = sorted(set([0, 1, J // 2, J - 1] + list(rng.integers(0, J, 6))))
    amp = np.sqrt(scan.intensity[js].astype(np.float64))
    # divide, on sampled patterns, from the known x
    y_ref = po.relax(lambda v: po.modulus_projection(v, amp), c)(x[js].astype(np.complex128))
    for i, j in enumerate(js):
        e = rel_l2(y[j], y_ref[i])
        assert e <= TOL, ("y", j, e)
    # object at sampled pixels, from the GPU's y and the start probe (float64 sums)
    cov = covered_mask(scan)
    rows, cols = np.nonzero(cov)
    pick = rng.choice(len(rows), 4000, replace=False)
    pr = p.astype(np.complex128)
    got, ref = [], []
    pos = scan.pos
    for r, q in zip(rows[pick], cols[pick]):
        sel = np.nonzero((pos[:, 0] <= r) & (r < pos[:, 0] + n) & (pos[:, 1] <= q) & (q < pos[:, 1] + n))[0]
        u0, u1 = r - pos[sel, 0], q - pos[sel, 1]
        pv = pr[u0, u1]
        num = np.sum(np.conj(pv) * y[sel, u0, u1].astype(np.complex128))
        den = np.sum(np.abs(pv) ** 2)
        thr = po.DEFAULT_TAU * np.max(np.abs(pr) ** 2)
        ref.append(num / den if den > thr else o[r, q])
        got.append(o1[r, q])
    e_obj = rel_l2(np.array(got), np.array(ref))
    print("  object sample error", e_obj, flush=True)
    assert e_obj <= TOL
    # probe at every pixel, from the GPU's y and new object (float64 sums over 4096 patterns)
    num = np.zeros((n, n), np.complex128)
    den = np.zeros((n, n), np.float64)
    for j0 in range(0, J, 256):
        sl = slice(j0, min(J, j0 + 256))
        op = po.patches(o1, pos[sl], n).astype(np.complex128)
        num += np.sum(np.conj(op) * y[sl].astype(np.complex128), axis=0)
        den += np.sum(np.abs(op) ** 2, axis=0)
    thr = po.DEFAULT_TAU * float(np.max(np.abs(o1.astype(np.complex128)) ** 2))
    p_ref = np.where(den > thr, num / np.where(den > 0, den, 1), p)
    e_prb = rel_l2(p1, p_ref)
    print("  probe error", e_prb, flush=True)
    assert e_prb <= TOL
    # the next iterate on sampled patterns, from the GPU's new object and probe
    x1 = x1_d.cpu().numpy()[js]
    z = po.exit_waves(o1.astype(np.complex128), p1.astype(np.complex128), pos[js])
    x_ref = a * (b * z + (1 - b) * y[js].astype(np.complex128)) + (1 - a) * x[js].astype(np.complex128)
    e_x = rel_l2(x1, x_ref)
    print("  next-iterate sample error", e_x, flush=True)
    assert e_x <= TOL


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
    # object there amplifies any rounding: bound 20 x the oracle's own change
    # under a 1e-7 perturbation of the start (at least 1e-5)
    rng = np.random.default_rng(1)
    q2, _, qi = two_steps(x * (1 + 1e-7 * rng.standard_normal(x.shape)))
    drift = {"y": rel_l2(qi["y"], i1["y"]), "x": rel_l2(q2.x, s2.x), "obj": rel_l2(q2.obj, s2.obj, cov),
             "probe": rel_l2(q2.probe, s2.probe)}
    tol = {k: max(TOL, 20 * v) for k, v in drift.items()}
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
