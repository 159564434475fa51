"""GPU parity of iteration-dependent relaxation, K concur sweeps and the shadow estimate.

Gates as for the plain iteration: one step from an identical float32 state
within 1e-5 of the oracle; free-running runs within the linearised
trajectory bound (the gate times the oracle's own amplification of a 1e-7
perturbation of the start, per iteration).
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
        if name == "tiny_n32":
            _SCANS[name] = make_scan("tiny_n32")
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


def lambda_schedule(n, lam0=0.9, lam1=0.3):
    """T_lambda with lambda falling linearly from lam0 to lam1 over n iterations."""
    return [po.preset("TLAMBDA", lam0 + (lam1 - lam0) * i / max(n - 1, 1)) for i in range(n)]


SCHEDULE = ([po.preset("RAAR", 0.75)] * 3 + [po.preset("DC")] * 2 + lambda_schedule(5)
            + [po.preset("RRR", 0.5)] * 2 + [(0.8, 1.3, 0.9)])


def oracle_drift_bound(scan, run, n_iter, n_seeds=3, eps=PERTURB):
    """Reference run and the linearised trajectory bound over n_iter
    iterations from its drift under a 1e-7 start perturbation."""
    amp = amp32(scan)
    cov = covered_mask(scan)
    base = po.init_state(scan.obj0.astype(np.complex64).astype(np.complex128),
                         scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos)
    ref = run(base.copy(), amp)
    worst = np.zeros(4)
    ef_r = np.array([m["fourier_err"] for m in ref.history])
    for sd in range(1, n_seeds + 1):
        rng = np.random.default_rng(sd)
        b = base.copy()
        b.x = b.x * (1 + eps * rng.standard_normal(b.x.shape))
        b = run(b, amp)
        ef_b = np.array([m["fourier_err"] for m in b.history])
        worst = np.maximum(worst, [rel_l2(b.x, ref.x), rel_l2(b.obj, ref.obj, cov), rel_l2(b.probe, ref.probe),
                                   float(np.max(np.abs(ef_b - ef_r) / ef_r))])
    return ref, trajectory_bound(worst, n_iter, eps=eps)


def compare_run(scan, g, ref, tol, what):
    x, y, o, p = (t.cpu().numpy() for t in g.get_state())
    ef_g = np.array([m["fourier_err"] for m in g.metric_history()])
    ef_o = np.array([m["fourier_err"] for m in ref.history])
    errs = np.array([rel_l2(x, ref.x), rel_l2(o, ref.obj, covered_mask(scan)), rel_l2(p, ref.probe),
                     float(np.max(np.abs(ef_g - ef_o) / ef_o))])
    say(f"  {what}: gpu-vs-oracle x/obj/probe/E_F", errs, "bound", tol)
    assert np.all(errs <= tol), (what, errs, tol)


def test_schedule_trajectory():
    scan = get_scan("tiny_n32")
    say("case: relaxation schedule", len(SCHEDULE), "iterations")
    g = gpu_scan(scan)
    g.iterate_schedule(SCHEDULE)
    assert g.iteration == len(SCHEDULE)
    ref, tol = oracle_drift_bound(scan, lambda st, amp: po.run_schedule(st, amp, scan.pos, SCHEDULE), len(SCHEDULE))
    compare_run(scan, g, ref, tol, "schedule")
    g.close()


def test_schedule_equals_piecewise_bitwise():
    scan = get_scan("tiny_n32")
    say("case: schedule vs piecewise set_algorithm + iterate")
    a = gpu_scan(scan)
    a.iterate_schedule(SCHEDULE)
    ra = [t.cpu().numpy() for t in a.get_state()]
    a.close()
    b = gpu_scan(scan)
    for abc in SCHEDULE:
        b.set_algorithm(*abc)
        b.iterate(1)
    rb = [t.cpu().numpy() for t in b.get_state()]
    b.close()
    for name, u, v in zip("xyop", ra, rb):
        assert np.array_equal(u.view(np.uint32), v.view(np.uint32)), name


def test_schedule_rejects_bad_entry_before_any_work():
    from paper_2311_11466_amd import PtyError
    scan = get_scan("tiny_n32")
    say("case: schedule validation")
    g = gpu_scan(scan)
    g.iterate(2)
    with pytest.raises(PtyError):
        g.iterate_schedule([po.preset("DC"), (0.0, 1.0, 1.0)])
    with pytest.raises(PtyError):
        g.iterate_schedule([po.preset("DC"), (1.0, float("nan"), 1.0)])
    assert g.iteration == 2
    with pytest.raises(PtyError):
        g.set_concur_sweeps(0)
    g.close()


@pytest.mark.parametrize("cfg", ["tiny_n32", "p128", "p256"])
def test_concur_sweeps_single_step(cfg):
    scan = get_scan(cfg)
    abc = po.preset("RAAR", 0.75)
    say("case: 3 concur sweeps, single step", cfg)
    st = round_state(oracle_state_after(scan, 2, abc))
    g = gpu_scan(scan)
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))
    g.set_algorithm(*abc)
    g.set_concur_sweeps(3)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    new, info = po.step(st, amp32(scan), scan.pos, *abc, sweeps=3)
    cov = covered_mask(scan)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x), "obj": rel_l2(o1, new.obj, cov),
            "probe": rel_l2(p1, new.probe)}
    # each sweep divides by the overlap sums again, so weakly lit object pixels
    # amplify float32 rounding; bound: the gate times the oracle's own
    # amplification of a 1e-7 perturbation of the state (one iteration)
    drift = {k: 0.0 for k in errs}
    for sd in (1, 2):
        rng = np.random.default_rng(sd)
        pst = po.State(st.x * (1 + PERTURB * rng.standard_normal(st.x.shape)), st.obj, st.probe, st.k)
        pn, pi = po.step(pst, amp32(scan), scan.pos, *abc, sweeps=3)
        d = {"y": rel_l2(pi["y"], info["y"]), "x": rel_l2(pn.x, new.x), "obj": rel_l2(pn.obj, new.obj, cov),
             "probe": rel_l2(pn.probe, new.probe)}
        drift = {k: max(drift[k], d[k]) for k in d}
    tol = {k: float(trajectory_bound(drift[k], 1)) for k in errs}
    say("  errors", {k: f"{v:.2e}" for k, v in errs.items()}, "bounds", {k: f"{v:.2e}" for k, v in tol.items()})
    assert all(errs[k] <= tol[k] for k in errs), (errs, tol)
    # three sweeps differ from one (the consensus moved further)
    one, _ = po.step(st, amp32(scan), scan.pos, *abc, sweeps=1)
    assert rel_l2(new.probe, one.probe) > 100 * TOL


def test_concur_sweeps_trajectory():
    scan = get_scan("tiny_n32")
    abc = po.preset("RAAR", 0.75)
    say("case: 2 concur sweeps, 10 iterations")
    g = gpu_scan(scan)
    g.set_algorithm(*abc)
    g.set_concur_sweeps(2)
    g.iterate(10)
    ref, tol = oracle_drift_bound(scan, lambda st, amp: po.run(st, amp, scan.pos, *abc, 10, sweeps=2), 10)
    compare_run(scan, g, ref, tol, "sweeps")
    g.close()


@pytest.mark.parametrize("cfg,sweeps", [("tiny_n32", 1), ("p128", 1), ("p256", 1), ("tiny_n32", 3)])
def test_shadow(cfg, sweeps):
    """Shadow P_C(P_D x) from the GPU's own state, against the oracle's shadow of
    that state; the scan's state is untouched and its continuation unchanged."""
    scan = get_scan(cfg)
    say("case: shadow", cfg, "sweeps", sweeps)
    g = gpu_scan(scan)
    g.set_algorithm_named("DR")
    g.set_concur_sweeps(sweeps)
    g.iterate(4)
    before = [t.cpu().numpy() for t in g.get_state()]
    o_s, p_s = (t.cpu().numpy() for t in g.shadow())
    after = [t.cpu().numpy() for t in g.get_state()]
    for name, u, v in zip("xop", [before[0], before[2], before[3]], [after[0], after[2], after[3]]):
        assert np.array_equal(u.view(np.uint32), v.view(np.uint32)), name
    st = po.State(before[0].astype(np.complex128), before[2].astype(np.complex128),
                  before[3].astype(np.complex128), 4)
    o_r, p_r = po.shadow(st, amp32(scan), scan.pos, blind=True, sweeps=sweeps)
    cov = covered_mask(scan)
    errs = (rel_l2(o_s, o_r, cov), rel_l2(p_s, p_r))
    say("  shadow obj/probe errors", errs)
    assert max(errs) <= TOL, errs
    # P_D x is what the y buffer holds now
    y_r = po.modulus_projection(st.x, amp32(scan))
    assert rel_l2(after[1], y_r) <= TOL
    # continuing after the shadow equals continuing without it
    g.iterate(2)
    cont = [t.cpu().numpy() for t in g.get_state()]
    g.close()
    h = gpu_scan(scan)
    h.set_algorithm_named("DR")
    h.set_concur_sweeps(sweeps)
    h.iterate(4)
    h.get_state()
    h.iterate(2)
    ref = [t.cpu().numpy() for t in h.get_state()]
    h.close()
    for name, u, v in zip("xyop", cont, ref):
        assert np.array_equal(u.view(np.uint32), v.view(np.uint32)), name
