"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Gate: one iteration from an identical state (the oracle state rounded to
float32 and loaded with set_state) must give x_{k+1}, y_k = P^c_D x_k, O_{k+1}
and P_{k+1} within 1e-5 relative L2 of the oracle's iteration from the same
rounded state.  The gate is applied along the oracle's trajectory (k = 0, 1,
10, 50, 100, 199), for every named algorithm set through the library's own
table (pty_set_algorithm_named, compared with the oracle's presets), and to an
iteration that starts from the library's pending update (the second of two
uninterrupted iterations).  Free-running trajectories are compared with a
bound derived from the gate and the oracle's own amplification of a
difference.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import (rel_l2, gpu_scan, amp32, covered_mask, oracle_state_after, round_state,
                         to_dev, STEP_GATE, trajectory_bound, oracle_drift)
from oracle import pty_oracle as po
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu

TOL = STEP_GATE
PRESETS = [("DC", 0.0), ("AR", 0.0), ("DR", 0.0), ("SF", 0.0), ("RAAR", 0.75), ("RRR", 0.5),
           ("TLAMBDA", 0.5)]
CUSTOM = [(0.3, 1.7, 0.6), (1.25, 0.5, 1.5)]
SIZES = ["tiny_n32", "p64", "p128", "p256"]

_SCANS = {}
_TRAJ = {}


def get_scan(name):
    if name not in _SCANS:
        if name == "tiny_n32":
            _SCANS[name] = make_scan("tiny_n32")
        elif name == "p64":      # 5 x 5 raster on a 172 x 172 object: ragged 64 x 16 tiles
            _SCANS[name] = make_scan(small_config("p64", 64, 5, 24, jitter=2, photons=1e6, seed=31))
        elif name == "p128":     # 4 x 4 raster on a 260 x 260 object
            _SCANS[name] = make_scan(small_config("p128", 128, 4, 40, jitter=2, photons=1e6, seed=41))
        elif name == "p256":     # 3 x 3 raster on a 430 x 430 object
            _SCANS[name] = make_scan(small_config("p256", 256, 3, 80, jitter=3, photons=1e5, seed=51))
        else:
            raise KeyError(name)
    return _SCANS[name]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_state(scan_name, k, blind=True):
    """The oracle's blind RAAR(0.75) state after k iterations from the scan's
    start (cached per scan), rounded to float32."""
    key = (scan_name, blind)
    scan = get_scan(scan_name)
    if key not in _TRAJ:
        _TRAJ[key] = {0: po.init_state(scan.obj0, scan.probe0, scan.pos)}
    traj = _TRAJ[key]
    k0 = max(i for i in traj if i <= k)
    st = traj[k0]
    for i in range(k0, k):
        st, _ = po.step(st, amp32(scan), scan.pos, *po.preset("RAAR", 0.75), blind=blind)
        traj[i + 1] = st
    return round_state(traj[k])


def set_algo(g, algo):
    """Select algo on the GPU scan: a named algorithm (name, param) through the
    library's table, or an (a, b, c) triple.  Returns the oracle's (a, b, c)."""
    if isinstance(algo[0], str):
        g.set_algorithm_named(*algo)
        return po.preset(*algo)
    g.set_algorithm(*algo)
    return tuple(algo)


def load(g, st):
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))


def single_step(scan_name, algo, blind=True, k_start=2, storage="fp32", full_metrics=True):
    """One GPU iteration and one oracle iteration from the same float32 state."""
    scan = get_scan(scan_name)
    st = oracle_state(scan_name, k_start, blind)
    g = gpu_scan(scan, storage=storage, blind=blind, full_metrics=full_metrics)
    load(g, st)
    abc = set_algo(g, algo)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    m = g.metrics(allow_diverged=True)
    new, info = po.step(st, amp32(scan), scan.pos, *abc, blind=blind)
    g.close()
    return (x1, y0, o1, p1, m), (new, info)


def check_step(scan, got, ref, tol=TOL, what="", metrics=("fourier_err", "consistency_err", "change")):
    x1, y0, o1, p1, m = got
    new, info = ref
    cov = covered_mask(scan)
    errs = {"y": rel_l2(y0, info["y"]), "x": rel_l2(x1, new.x), "obj": rel_l2(o1, new.obj, cov),
            "probe": rel_l2(p1, new.probe)}
    say(what, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (what, k, v)
    # pixels no window covers keep their value exactly
    assert np.array_equal(o1[~cov], new.obj[~cov].astype(np.complex64))
    om = info["metrics"]
    for key in metrics:
        assert abs(m[key] - om[key]) <= 1e-4 * abs(om[key]) + 1e-12, (what, key, m[key], om[key])


@pytest.mark.parametrize("cfg", SIZES)
@pytest.mark.parametrize("name,param", PRESETS)
def test_single_step_named(cfg, name, param):
    """Every named algorithm, selected through the library's table, against the
    oracle's preset: an (a, b, c) table slip fails here."""
    say("case: single step", cfg, name, param)
    got, ref = single_step(cfg, (name, param))
    check_step(get_scan(cfg), got, ref, what=f"{cfg} {name}")


@pytest.mark.parametrize("abc", CUSTOM)
def test_single_step_custom_abc(abc):
    say("case: single step tiny_n32 abc", abc)
    got, ref = single_step("tiny_n32", abc)
    check_step(get_scan("tiny_n32"), got, ref, what=f"n32 {abc}")


@pytest.mark.parametrize("cfg,k", [("tiny_n32", k) for k in (0, 1, 10, 50, 100, 199)]
                         + [("p128", k) for k in (0, 10, 50)] + [("p256", k) for k in (0, 10)])
def test_single_step_along_trajectory(cfg, k):
    """The gate at iterations along the oracle's blind RAAR(0.75) trajectory."""
    say("case: single step along the trajectory", cfg, "k =", k)
    got, ref = single_step(cfg, ("RAAR", 0.75), k_start=k)
    check_step(get_scan(cfg), got, ref, what=f"{cfg} k={k}")


@pytest.mark.parametrize("cfg", ["tiny_n32", "p128", "p256"])
def test_single_step_known_probe(cfg):
    say("case: known probe", cfg)
    got, ref = single_step(cfg, ("DR", 0.0), blind=False)
    check_step(get_scan(cfg), got, ref, what=f"{cfg} known")
    assert np.array_equal(got[3], ref[0].probe.astype(np.complex64))


@pytest.mark.parametrize("full_metrics", [True, False])
@pytest.mark.parametrize("cfg", SIZES)
@pytest.mark.parametrize("name,param", PRESETS)
def test_pending_step(cfg, name, param, full_metrics):
    """The gate on an iteration that starts from the library's pending update.

    The second of two uninterrupted iterations forms x_{k+1} in its prologue
    from the first iteration's (a b, a(1-b), 1-a) (or from the stored blend w);
    a twin scan runs the first iteration alone and reads its state back (the
    library materialises x with the prologue's arithmetic and is bitwise
    deterministic), and the oracle's iteration from that state is compared
    with the second iteration at 1e-5."""
    scan = get_scan(cfg)
    say("case: pending step", cfg, name, param, "full metrics" if full_metrics else "fourier only")
    st = oracle_state(cfg, 2)
    a = gpu_scan(scan, full_metrics=full_metrics)
    load(a, st)
    abc = set_algo(a, (name, param))
    form = a.state_form()
    a.iterate(1)
    x1, _, o1, p1 = (t.cpu().numpy() for t in a.get_state())
    a.close()
    b = gpu_scan(scan, full_metrics=full_metrics)
    load(b, st)
    set_algo(b, (name, param))
    b.iterate(2)
    x2, y1, o2, p2 = (t.cpu().numpy() for t in b.get_state())
    hist = b.metric_history()
    b.close()
    s1 = po.State(x1.astype(np.complex128), o1.astype(np.complex128), p1.astype(np.complex128), 1)
    new, info = po.step(s1, amp32(scan), scan.pos, *abc, blind=True)
    metrics = ("fourier_err", "consistency_err", "change") if full_metrics else ("fourier_err",)
    check_step(scan, (x2, y1, o2, p2, hist[-1]), (new, info), what=f"{cfg} {name} pending ({form} form)",
               metrics=metrics)
    assert hist[-1]["iteration"] == 1


@pytest.mark.parametrize("cfg,algo,n_iter", [
    ("tiny_n32", ("RAAR", 0.75), 20),
    ("tiny_n32", ("DC", 0.0), 20),
    ("p64", ("RRR", 0.5), 10),
    ("p256", ("DR", 0.0), 5),
])
def test_trajectory(cfg, algo, n_iter):
    """Free-running iterations from the start: state and Fourier-error history,
    within the linearised bound n_iter * gate * (oracle amplification)."""
    scan = get_scan(cfg)
    say("case: trajectory", cfg, algo, n_iter)
    g = gpu_scan(scan)
    abc = set_algo(g, algo)
    g.iterate(n_iter)
    x, y, o, p = (t.cpu().numpy() for t in g.get_state())
    hist = g.metric_history()
    g.close()
    amp = amp32(scan)
    cov = covered_mask(scan)
    base = po.init_state(scan.obj0.astype(np.complex64).astype(np.complex128),
                         scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos)

    def run(x0):
        b = base.copy()
        b.x = x0
        return po.run(b, amp, scan.pos, *abc, n_iter, blind=True)

    def diff(b, r):
        ef_a = np.array([m["fourier_err"] for m in r.history])
        ef_b = np.array([m["fourier_err"] for m in b.history])
        return [rel_l2(b.x, r.x), rel_l2(b.obj, r.obj, cov), rel_l2(b.probe, r.probe),
                float(np.max(np.abs(ef_a - ef_b) / ef_a))]
    ref, drift = oracle_drift(run, base.x, diff)
    tol = trajectory_bound(drift, n_iter)
    ef_g = np.array([m["fourier_err"] for m in hist])
    ef_o = np.array([m["fourier_err"] for m in ref.history])
    errs = np.array([rel_l2(x, ref.x), rel_l2(o, ref.obj, cov), rel_l2(p, ref.probe),
                     float(np.max(np.abs(ef_g - ef_o) / ef_o))])
    say("  gpu-vs-oracle x/obj/probe/E_F", errs, "oracle drift", drift, "bound", tol)
    assert np.all(errs <= tol), (errs, tol)
    assert [m["iteration"] for m in hist] == list(range(n_iter))


def test_fixed_point_noise_free():
    """The true object, probe and exit waves of noise-free data are a fixed point."""
    scan = get_scan("tiny_n32")
    say("case: fixed point")
    g = gpu_scan(scan, obj0=scan.obj_true, probe0=scan.probe_true)
    x_true = po.exit_waves(scan.obj_true, scan.probe_true, scan.pos)
    for name, prm in PRESETS:
        g.set_state(to_dev(x_true.astype(np.complex64)), None, to_dev(scan.obj_true.astype(np.complex64)),
                    to_dev(scan.probe_true.astype(np.complex64)))
        g.set_algorithm_named(name, prm)
        g.iterate(1)
        x, y, o, p = (t.cpu().numpy() for t in g.get_state())
        assert rel_l2(x, x_true) < 1e-5, name
        assert rel_l2(p, scan.probe_true) < 1e-5, name
        m = g.metrics()
        assert m["fourier_err"] < 1e-10 and m["consistency_err"] < 1e-10, (name, m)
    g.close()


def test_deterministic_bitwise():
    scan = get_scan("p128")
    say("case: determinism")
    out = []
    for _ in range(2):
        g = gpu_scan(scan)
        g.set_algorithm_named("RAAR", 0.75)
        g.iterate(4)
        out.append([t.cpu().numpy() for t in g.get_state()])
        g.close()
    for a, b in zip(*out):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("cfg", ["tiny_n32", "p256"])
def test_checkpoint_resume_bitwise(cfg):
    scan = get_scan(cfg)
    say("case: checkpoint", cfg)
    a = gpu_scan(scan)
    a.set_algorithm_named("DR")
    a.iterate(6)
    ref = [t.cpu().numpy() for t in a.get_state()]
    a.close()
    b = gpu_scan(scan)
    b.set_algorithm_named("DR")
    b.iterate(3)
    ck = b.get_state()
    b.close()
    c = gpu_scan(scan)
    c.set_state(*ck)
    c.set_algorithm_named("DR")
    c.iterate(3)
    got = [t.cpu().numpy() for t in c.get_state()]
    c.close()
    for name, r, q in zip("xyop", ref, got):
        assert np.array_equal(r.view(np.uint32), q.view(np.uint32)), name


def test_probe_update_start():
    scan = get_scan("tiny_n32")
    say("case: probe_update_start")
    g = gpu_scan(scan, probe_update_start=3)
    g.set_algorithm_named("DC")
    g.iterate(3)
    assert np.array_equal(g.probe().cpu().numpy(), scan.probe0.astype(np.complex64))
    g.iterate(1)
    assert not np.array_equal(g.probe().cpu().numpy(), scan.probe0.astype(np.complex64))
    g.close()


def test_edge_single_position_exact_object():
    """J = 1, object exactly N x N: every pixel covered once; ragged everywhere."""
    rng = np.random.default_rng(5)
    n = 32
    obj = (rng.uniform(0.5, 1, (n, n)) * np.exp(1j * rng.uniform(-1, 1, (n, n))))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    pos = np.zeros((1, 2), np.int32)
    inten = np.abs(np.fft.fft2(obj * probe))[None] ** 2 * rng.uniform(0.5, 1.5, (1, n, n))

    class S:  # minimal scan record for the helpers
        pass
    s = S()
    s.pos, s.intensity, s.obj0, s.probe0 = pos, inten, np.ones((n, n), complex), probe
    say("case: single position")
    g = gpu_scan(s)
    g.set_algorithm_named("RAAR", 0.75)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    st = po.init_state(np.ones((n, n)), probe.astype(np.complex64).astype(np.complex128), pos)
    new, info = po.step(st, np.sqrt(inten.astype(np.float32).astype(np.float64)), pos,
                        *po.preset("RAAR", 0.75))
    assert rel_l2(y0, info["y"]) < TOL and rel_l2(x1, new.x) < TOL
    assert rel_l2(o1, new.obj) < TOL and rel_l2(p1, new.probe) < TOL


@pytest.mark.parametrize("cfg", ["tiny_n32", "p128", "p256"])
def test_edge_zero_wave_and_zero_data(cfg):
    """x_j = 0 (phase taken as 0: P_D x_j = F^-1 A_j) and I_j = 0 (P_D x_j = 0).
    At N = 128 every frequency of the zero wave takes the phase-0 value on both
    halves of the split-exchange work-group (one of which holds the spectrum
    with odd frequencies negated)."""
    scan = get_scan(cfg)
    say("case: zero wave / zero data", cfg)
    inten = scan.intensity.copy()
    inten[5] = 0.0

    class S:
        pass
    s = S()
    s.pos, s.intensity, s.obj0, s.probe0 = scan.pos, inten, scan.obj0, scan.probe0
    st = oracle_state(cfg, 1)
    st.x[3] = 0.0
    g = gpu_scan(s)
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))
    g.set_algorithm_named("DC")
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    amp = np.sqrt(inten.astype(np.float32).astype(np.float64))
    new, info = po.step(st, amp, scan.pos, 1, 1, 1)
    assert rel_l2(y0[3], np.fft.ifft2(amp[3])) < TOL
    assert np.abs(y0[5]).max() == 0.0
    assert rel_l2(y0, info["y"]) < TOL and rel_l2(o1, new.obj, covered_mask(scan)) < TOL


@pytest.mark.parametrize("cfg", ["fp16_n32", "p64", "p128", "p256"])
def test_fp16_storage_single_step(cfg):
    """FP16 exit-wave storage: one step from the same (FP16-representable) state,
    at every pattern size (N = 128: the split-exchange divide; N = 256: the
    three passes through a separate float32 intermediate).

    Bound: x and y are rounded to float16 on store (unit roundoff 2^-11 ~ 4.9e-4
    per component), so their relative L2 error is at most about 5e-4; the
    object and probe inherit it from y.  Gate: 1e-3 at every size (measured
    about 2e-4 for y, x and the object).
    """
    scan = make_scan("fp16_n32") if cfg == "fp16_n32" else get_scan(cfg)
    say("case: fp16 single step", cfg)
    g = gpu_scan(scan, storage="fp16")
    st = round_state(oracle_state_after(scan, 2, po.preset("RAAR", 0.75)))
    g.set_state(to_dev(st.x.astype(np.complex64)), None, to_dev(st.obj.astype(np.complex64)),
                to_dev(st.probe.astype(np.complex64)))
    # the state the library now holds is x rounded to float16 (times its scale)
    xs = g.get_state()[0].cpu().numpy()
    assert rel_l2(xs, st.x) < 5e-4
    st.x = xs.astype(np.complex128)
    g.set_algorithm_named("RAAR", 0.75)
    g.iterate(1)
    x1, y0, o1, p1 = (t.cpu().numpy() for t in g.get_state())
    g.close()
    new, info = po.step(st, amp32(scan), scan.pos, *po.preset("RAAR", 0.75))
    cov = covered_mask(scan)
    errs = (rel_l2(y0, info["y"]), rel_l2(x1, new.x), rel_l2(o1, new.obj, cov), rel_l2(p1, new.probe))
    say("  fp16 errors y/x/obj/probe", errs)
    assert max(errs) < 1e-3, errs


def test_c1_known_probe_then_blind_dc():
    """The 32-pixel scan's reference run: DC with the probe held for 50
    iterations, then blind, 200 iterations in all (probe_update_start = 50),
    against the oracle's same run, within the linearised trajectory bound.
    (The scan description both holds the probe for 50 iterations and starts
    it from a disc of radius 8; the reading taken here holds that start probe
    for 50 iterations.)"""
    scan = get_scan("tiny_n32")
    abc = po.preset("DC")
    n_iter, start = 200, 50
    say("case: C1 DC, probe held for 50 iterations then updated, 200 iterations")
    g = gpu_scan(scan, probe_update_start=start)
    g.set_algorithm(*abc)
    g.iterate(n_iter)
    x, y, o, p = (t.cpu().numpy() for t in g.get_state())
    ef_g = np.array([m["fourier_err"] for m in g.metric_history()])
    g.close()
    amp = amp32(scan)
    cov = covered_mask(scan)

    def run(seed):
        st = po.init_state(scan.obj0.astype(np.complex64).astype(np.complex128),
                           scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos)
        if seed is not None:
            rng = np.random.default_rng(seed)
            st.x = st.x * (1 + 1e-7 * rng.standard_normal(st.x.shape))
        return po.run(st, amp, scan.pos, *abc, n_iter, probe_update_start=start)
    ref = run(None)
    ef_r = np.array([m["fourier_err"] for m in ref.history])
    worst = np.zeros(4)
    for sd in (1, 2):
        b = run(sd)
        ef_b = np.array([m["fourier_err"] for m in b.history])
        worst = np.maximum(worst, [rel_l2(b.x, ref.x), rel_l2(b.obj, ref.obj, cov), rel_l2(b.probe, ref.probe),
                                   float(np.max(np.abs(ef_b - ef_r) / ef_r))])
    tol = trajectory_bound(worst, n_iter)
    errs = np.array([rel_l2(x, ref.x), rel_l2(o, ref.obj, cov), rel_l2(p, ref.probe),
                     float(np.max(np.abs(ef_g - ef_r) / ef_r))])
    say("  gpu-vs-oracle x/obj/probe/E_F", errs, "bound", tol)
    assert np.all(errs <= tol), (errs, tol)
    # the probe is untouched while held
    assert ef_g[-1] < ef_g[0]
