"""GPU parity of the blend form against the FP64 oracle.

Without full metrics, for N <= 64 and a != 1, b != 1, the library keeps
w = (1-a) x + a(1-b) y in the x buffer between iterations and forms
x_{k+1} = ab P S_j O + w in the next divide prologue.  The iteration it
computes is the same (only the float32 rounding order differs), so the gates
are those of the x-form parity tests: two iterations from an identical state
within 1e-5 of the oracle (the second one runs the prologue that reads w),
trajectories within the oracle's own amplification bound, and bitwise
checkpoint/resume.
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
BLEND = [("RAAR", 0.75), ("DR", 0.0), ("RRR", 0.5), ("TLAMBDA", 0.5)]

_SCANS = {}


def get_scan(name):
    if name not in _SCANS:
        if name == "tiny_n32":
            _SCANS[name] = make_scan("tiny_n32")
        elif name == "p64":
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


def blend_scan(scan, storage="fp32"):
    return gpu_scan(scan, storage=storage, full_metrics=False)


def test_blend_form_rule():
    """The library keeps the blend w exactly when 1-a and a(1-b) are both
    nonzero, without full metrics and for N <= 64 (pty_state_form)."""
    for cfg in ("tiny_n32", "p64", "p128", "p256"):
        scan = get_scan(cfg)
        for full in (False, True):
            g = gpu_scan(scan, full_metrics=full)
            for name, prm in BLEND + [("DC", 0.0), ("AR", 0.0), ("SF", 0.0)]:
                g.set_algorithm_named(name, prm)
                a, b, _ = po.preset(name, prm)
                want = (not full and scan.n <= 64 and np.float32(1 - a) != 0 and np.float32(a * (1 - b)) != 0)
                assert g.state_form() == ("w" if want else "x"), (cfg, full, name)
            g.close()


def two_steps(scan, abc, storage="fp32", k_start=2):
    st = round_state(oracle_state_after(scan, k_start, po.preset("RAAR", 0.75)))
    g = blend_scan(scan, storage)
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))
    if storage == "fp16":
        st.x = g.get_state()[0].cpu().numpy().astype(np.complex128)
    g.set_algorithm(*abc)
    g.iterate(2)
    x2, y1, o2, p2 = (t.cpu().numpy() for t in g.get_state())
    hist = g.metric_history()
    g.close()
    amp = amp32(scan)
    s1, i0 = po.step(st, amp, scan.pos, *abc)
    s2, i1 = po.step(s1, amp, scan.pos, *abc)
    return (x2, y1, o2, p2, hist), (s2, i0, i1)


def check(scan, got, ref, tol, what):
    x2, y1, o2, p2, hist = got
    s2, i0, i1 = ref
    cov = covered_mask(scan)
    errs = {"y": rel_l2(y1, i1["y"]), "x": rel_l2(x2, s2.x), "obj": rel_l2(o2, s2.obj, cov),
            "probe": rel_l2(p2, s2.probe)}
    say(what, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (what, k, v)
    assert np.array_equal(o2[~cov], s2.obj[~cov].astype(np.complex64))
    assert len(hist) == 2
    for m, info in zip(hist, (i0, i1)):
        ef = info["metrics"]["fourier_err"]
        assert abs(m["fourier_err"] - ef) <= 1e-4 * ef, (what, m["fourier_err"], ef)
        # the blend form keeps no x_k: no consistency or change metric
        assert np.isnan(m["consistency_err"]) and np.isnan(m["change"]), (what, m)


@pytest.mark.parametrize("name,param", BLEND + [("custom", 0.0)])
def test_blend_two_steps_presets_n32(name, param):
    scan = get_scan("tiny_n32")
    abc = (0.3, 1.7, 0.6) if name == "custom" else po.preset(name, param)
    say("case: blend two steps tiny_n32", name, abc)
    got, ref = two_steps(scan, abc)
    check(scan, got, ref, TOL, f"blend {name}")


@pytest.mark.parametrize("cfg", ["p64"])
def test_blend_two_steps_sizes(cfg):
    scan = get_scan(cfg)
    abc = po.preset("RAAR", 0.75)
    say("case: blend two steps", cfg)
    got, ref = two_steps(scan, abc)
    check(scan, got, ref, TOL, f"blend {cfg}")


def test_blend_fp16_two_steps():
    """FP16 storage in the blend form: w and y rounded to float16 on store.

    Bound as for the x form (unit roundoff 2^-11 per stored component, about
    5e-4 relative per store, two iterations): 2e-3.
    """
    scan = make_scan("fp16_n32")
    abc = po.preset("RAAR", 0.75)
    say("case: blend fp16 two steps")
    got, ref = two_steps(scan, abc, storage="fp16")
    x2, y1, o2, p2, _ = got
    s2, _, i1 = ref
    cov = covered_mask(scan)
    errs = (rel_l2(y1, i1["y"]), rel_l2(x2, s2.x), rel_l2(o2, s2.obj, cov), rel_l2(p2, s2.probe))
    say("  blend fp16 errors y/x/obj/probe", errs)
    assert max(errs) < 2e-3


def schedule_run(scan, schedule, x_scale=None):
    """Oracle run of a list of (abc, iterations) from the start; x_scale perturbs x_0."""
    amp = amp32(scan)
    st = po.init_state(scan.obj0.astype(np.complex64).astype(np.complex128),
                       scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos)
    if x_scale is not None:
        st.x = st.x * x_scale
    efs = []
    for abc, n in schedule:
        for _ in range(n):
            st, info = po.step(st, amp, scan.pos, *abc)
            efs.append(info["metrics"]["fourier_err"])
    return st, np.array(efs)


@pytest.mark.parametrize("cfg,schedule", [
    ("tiny_n32", [(po.preset("RAAR", 0.75), 20)]),
    ("tiny_n32", [(po.preset("RAAR", 0.75), 3), (po.preset("DC"), 2), (po.preset("RRR", 0.5), 3),
                  (po.preset("SF"), 1), (po.preset("DR"), 3)]),
    ("p64", [(po.preset("TLAMBDA", 0.5), 8)]),
])
def test_blend_trajectory(cfg, schedule):
    """Free-running blend-form iterations, including switches of form between
    iterations (DC and SF run in the x form), against the oracle: bound 20 x
    the linearised trajectory bound (gate times the oracle's own amplification
    of a 1e-7 perturbation of the start, per iteration)."""
    scan = get_scan(cfg)
    say("case: blend trajectory", cfg, [(a, n) for a, n in schedule])
    g = blend_scan(scan)
    for abc, n in schedule:
        g.set_algorithm(*abc)
        g.iterate(n)
    x, y, o, p = (t.cpu().numpy() for t in g.get_state())
    ef_g = np.array([m["fourier_err"] for m in g.metric_history()])
    g.close()
    ref, ef_o = schedule_run(scan, schedule)
    cov = covered_mask(scan)
    worst = np.zeros(4)
    for sd in (1, 2, 3):
        rng = np.random.default_rng(sd)
        pert, ef_p = schedule_run(scan, schedule, 1 + PERTURB * rng.standard_normal(ref.x.shape))
        worst = np.maximum(worst, [rel_l2(pert.x, ref.x), rel_l2(pert.obj, ref.obj, cov),
                                   rel_l2(pert.probe, ref.probe), float(np.max(np.abs(ef_p - ef_o) / ef_o))])
    tol = trajectory_bound(worst, sum(n for _, n in schedule))
    errs = np.array([rel_l2(x, ref.x), rel_l2(o, ref.obj, cov), rel_l2(p, ref.probe),
                     float(np.max(np.abs(ef_g - ef_o) / ef_o))])
    say("  gpu-vs-oracle x/obj/probe/E_F", errs, "bound", tol)
    assert np.all(errs <= tol), (errs, tol)


@pytest.mark.parametrize("cfg", ["tiny_n32", "p64"])
def test_blend_checkpoint_resume_bitwise(cfg):
    """iterate(6) equals iterate(3), get_state, a new scan from that state, iterate(3)."""
    scan = get_scan(cfg)
    say("case: blend checkpoint", cfg)
    a = blend_scan(scan)
    a.set_algorithm_named("RAAR", 0.75)
    a.iterate(6)
    ref = [t.cpu().numpy() for t in a.get_state()]
    a.close()
    b = blend_scan(scan)
    b.set_algorithm_named("RAAR", 0.75)
    b.iterate(3)
    ck = b.get_state()
    b.iterate(3)             # the materialised state continues in the blend form
    cont = [t.cpu().numpy() for t in b.get_state()]
    b.close()
    c = blend_scan(scan)
    c.set_state(*ck)
    c.set_algorithm_named("RAAR", 0.75)
    c.iterate(3)
    got = [t.cpu().numpy() for t in c.get_state()]
    c.close()
    for name, r, q, u in zip("xyop", ref, got, cont):
        assert np.array_equal(r.view(np.uint32), q.view(np.uint32)), name
        assert np.array_equal(r.view(np.uint32), u.view(np.uint32)), name
