"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with
an independent fact: a brute-force definition, a closed form, an invariant, a
textbook library routine or a hand-derived worked example.  They are plain
functions (not tests) so that the mutation tests can run them against a
deliberately broken oracle and check that each planted mistake is caught.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np

from oracle import pty_oracle as po
from oracle.toy import ThreeCircles

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def naive_dft2(x):
    """Brute-force 2-D DFT, X[k,l] = sum_{m,n} x[m,n] exp(-2 pi i (k m / N0 + l n / N1))."""
    n0, n1 = x.shape
    out = np.zeros((n0, n1), dtype=np.complex128)
    for k in range(n0):
        for l in range(n1):
            s = 0j
            for m in range(n0):
                for n in range(n1):
                    ang = -2.0 * np.pi * (k * m / n0 + l * n / n1)
                    s += x[m, n] * complex(np.cos(ang), np.sin(ang))
            out[k, l] = s
    return out


# --------------------------------------------------------------------------
# Fourier transform
# --------------------------------------------------------------------------
def pin_dft_brute_force():
    rng = _rng(1)
    for n in (1, 2, 3, 4, 8, 16):
        x = _crandn(rng, n, n)
        ref = naive_dft2(x)
        got = po.dft2(x)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * n * n), n
        back = po.idft2(ref)
        assert np.allclose(back, x, rtol=1e-12, atol=1e-12), n


def pin_dft_parseval_delta():
    rng = _rng(2)
    for n in (8, 32):
        x = _crandn(rng, 3, n, n)
        f = po.dft2(x)
        assert np.allclose(np.sum(np.abs(f) ** 2, axis=(1, 2)),
                           n * n * np.sum(np.abs(x) ** 2, axis=(1, 2)), rtol=1e-12)
        d = np.zeros((n, n), complex)
        d[0, 0] = 1.0
        assert np.allclose(po.dft2(d), 1.0)
        d = np.zeros((n, n), complex)
        d[0, 1] = 1.0   # a shift by one column is a linear phase along the column index
        ramp = np.exp(-2j * np.pi * np.arange(n) / n)
        assert np.allclose(po.dft2(d), np.broadcast_to(ramp[None, :], (n, n)))


# --------------------------------------------------------------------------
# Relaxed projections and reflections (Introduction)
# --------------------------------------------------------------------------
def pin_relaxation_algebra():
    rng = _rng(3)
    amp = np.abs(_crandn(rng, 2, 8, 8))
    x = _crandn(rng, 2, 8, 8)

    def proj(v):
        return po.modulus_projection(v, amp)
    px = proj(x)
    assert np.allclose(po.relax(proj, 0.0)(x), x)
    assert np.allclose(po.relax(proj, 1.0)(x), px)
    assert np.allclose(po.reflect(proj)(x), 2 * px - x)
    # a = 0.5 lands half way, a = 1.5 beyond the projection along the same line
    assert np.allclose(po.relax(proj, 0.5)(x) - x, 0.5 * (px - x))
    assert np.allclose(po.relax(proj, 1.5)(x) - x, 1.5 * (px - x))


# --------------------------------------------------------------------------
# Divide: the modulus projection
# --------------------------------------------------------------------------
def pin_modulus_projection():
    rng = _rng(4)
    j, n = 3, 16
    amp = np.abs(_crandn(rng, j, n, n))
    x = _crandn(rng, j, n, n)
    px = po.modulus_projection(x, amp)
    # the image lies in the set: |F P_D x| = A
    assert np.allclose(np.abs(po.dft2(px)), amp, rtol=1e-12, atol=1e-12)
    # idempotent, and points of the set are fixed
    assert np.allclose(po.modulus_projection(px, amp), px, rtol=1e-12, atol=1e-12)
    # it keeps the Fourier phase of x
    fx, fp = po.dft2(x), po.dft2(px)
    assert np.allclose(fp * np.abs(fx), fx * amp, rtol=1e-10, atol=1e-10)
    # nearest point: no random member of the set is closer to x
    d0 = np.sum(np.abs(px - x) ** 2)
    for _ in range(64):
        w = po.idft2(amp * np.exp(2j * np.pi * rng.random((j, n, n))))
        assert d0 <= np.sum(np.abs(w - x) ** 2) + 1e-9
    # where F x = 0 the phase is taken as zero
    z = np.zeros((1, n, n), complex)
    pz = po.modulus_projection(z, amp[:1])
    assert np.allclose(po.dft2(pz), amp[:1])


# --------------------------------------------------------------------------
# Concur: least-squares overlap consensus
# --------------------------------------------------------------------------
def _tiny_problem(seed=5):
    rng = _rng(seed)
    h = w = 6
    n = 4
    pos = np.array([[0, 0], [1, 2], [2, 1], [2, 2]], dtype=np.int32)
    probe = _crandn(rng, n, n)
    obj = _crandn(rng, h, w)
    y = _crandn(rng, len(pos), n, n)
    return h, w, n, pos, probe, obj, y


def _dense_object_operator(h, w, n, pos, probe):
    """Matrix M with (M o)[j, u] = P(u) O(pos_j + u), built entry by entry."""
    m = np.zeros((len(pos) * n * n, h * w), dtype=np.complex128)
    for j, (p, q) in enumerate(pos):
        for u0 in range(n):
            for u1 in range(n):
                m[j * n * n + u0 * n + u1, (p + u0) * w + (q + u1)] = probe[u0, u1]
    return m


def pin_object_step_is_least_squares():
    h, w, n, pos, probe, obj, y = _tiny_problem()
    m = _dense_object_operator(h, w, n, pos, probe)
    sol, *_ = np.linalg.lstsq(m, y.reshape(-1), rcond=None)
    covered = np.abs(m).sum(axis=0) > 0
    got = po.concur_object(y, obj, probe, pos)
    assert np.allclose(got.reshape(-1)[covered], sol[covered], rtol=1e-10, atol=1e-10)
    # pixels no patch covers keep their previous value
    assert np.array_equal(got.reshape(-1)[~covered], obj.reshape(-1)[~covered])


def pin_probe_step_is_least_squares():
    h, w, n, pos, probe, obj, y = _tiny_problem(6)
    # (M p)[j, u] = O(pos_j + u) P(u): one column per probe pixel
    m = np.zeros((len(pos) * n * n, n * n), dtype=np.complex128)
    for j, (p, q) in enumerate(pos):
        for u0 in range(n):
            for u1 in range(n):
                m[j * n * n + u0 * n + u1, u0 * n + u1] = obj[p + u0, q + u1]
    sol, *_ = np.linalg.lstsq(m, y.reshape(-1), rcond=None)
    got = po.concur_probe(y, obj, probe, pos)
    assert np.allclose(got.reshape(-1), sol, rtol=1e-10, atol=1e-10)


def pin_concur_is_average_in_the_plain_case():
    """With a unit probe and all copies on the same window, P_C is the mean."""
    rng = _rng(7)
    n, j = 8, 5
    pos = np.zeros((j, 2), dtype=np.int32)
    y = _crandn(rng, j, n, n)
    obj0 = _crandn(rng, n, n)
    z, o, p = po.concur(y, obj0, np.ones((n, n), complex), pos, update_probe=False)
    assert np.allclose(o, y.mean(axis=0))
    assert np.allclose(z, np.broadcast_to(y.mean(axis=0), y.shape))


def pin_concur_projection_properties():
    h, w, n, pos, probe, obj, y = _tiny_problem(8)
    # known probe: linear, idempotent and self-adjoint on the product space
    def pc(v):
        return po.concur(v, obj, probe, pos, update_probe=False)[0]
    z = pc(y)
    assert np.allclose(pc(z), z, rtol=1e-10, atol=1e-10)
    rng = _rng(9)
    v = _crandn(rng, *y.shape)
    assert np.isclose(np.vdot(pc(v), y), np.vdot(v, pc(y)), rtol=1e-10)
    # blind, warm started from its own output: a second sweep changes nothing
    zb, ob, pb = po.concur(y, obj, probe, pos, update_probe=True)
    zb2, ob2, pb2 = po.concur(zb, ob, pb, pos, update_probe=True)
    assert np.allclose(zb2, zb, rtol=1e-9, atol=1e-9)
    # each half-step of the blind sweep does not increase sum_j |P S_j O - y_j|^2
    def f(o, p):
        return np.sum(np.abs(po.exit_waves(o, p, pos) - y) ** 2)
    o1 = po.concur_object(y, obj, probe, pos)
    p1 = po.concur_probe(y, o1, probe, pos)
    assert f(o1, probe) <= f(obj, probe) + 1e-12
    assert f(o1, p1) <= f(o1, probe) + 1e-12


def pin_concur_sweeps_alternating_least_squares():
    """K sweeps: sum_j |P S_j O - y_j|^2 never increases from sweep to sweep;
    for exit waves that some (O*, P*) explains exactly, the sweeps from a
    perturbed start drive it to zero (each sweep must use the previous
    sweep's probe and object)."""
    h, w, n, pos, probe, obj, y = _tiny_problem(11)

    def f(o, p, target):
        return np.sum(np.abs(po.exit_waves(o, p, pos) - target) ** 2)
    vals = []
    for k in range(1, 7):
        _, o, p = po.concur(y, obj, probe, pos, update_probe=True, sweeps=k)
        vals.append(f(o, p, y))
    assert all(b <= a + 1e-12 for a, b in zip(vals, vals[1:])), vals
    assert vals[-1] < vals[0]
    rng = _rng(14)
    y_exact = po.exit_waves(obj, probe, pos)
    o0 = obj + 0.3 * _crandn(rng, *obj.shape)
    p0 = probe + 0.3 * _crandn(rng, *probe.shape)
    _, o, p = po.concur(y_exact, o0, p0, pos, update_probe=True, sweeps=200)
    assert f(o, p, y_exact) <= 1e-10 * f(o0, p0, y_exact)
    # the known-probe consensus is a projection: more sweeps change nothing
    _, o1, _ = po.concur(y, obj, probe, pos, update_probe=False, sweeps=1)
    _, o3, _ = po.concur(y, obj, probe, pos, update_probe=False, sweeps=3)
    assert np.allclose(o1, o3, rtol=1e-12, atol=1e-12)


def pin_shadow_recovers_the_true_state():
    """Noise-free data and the true exit waves: P_D leaves x unchanged and the
    consensus of the true exit waves is the true (O, P), so the shadow is the
    truth; from a perturbed start it is an unrelaxed divide plus consensus,
    i.e. one DC step's (O, P)."""
    h, w, n, pos, probe, obj, _ = _tiny_problem(12)
    amp = np.abs(po.dft2(po.exit_waves(obj, probe, pos)))
    st = po.init_state(obj, probe, pos)
    o, p = po.shadow(st, amp, pos)
    assert np.allclose(o, obj, rtol=1e-10, atol=1e-10)
    assert np.allclose(p, probe, rtol=1e-10, atol=1e-10)
    rng = _rng(13)
    st2 = po.State(st.x + 0.1 * _crandn(rng, *st.x.shape), obj * 0.9, probe, 0)
    o2, p2 = po.shadow(st2, amp, pos)
    new, _ = po.step(st2, amp, pos, 1.0, 1.0, 1.0)
    assert np.allclose(o2, new.obj, rtol=1e-12, atol=1e-12)
    assert np.allclose(p2, new.probe, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# The generalised iteration
# --------------------------------------------------------------------------
def _frac(s):
    return float(Fraction(s))


def pin_three_circle_worked_example():
    with open(os.path.join(GOLDEN, "three_circles.json")) as fh:
        g = json.load(fh)
    toy = ThreeCircles([complex(*c["center"]) for c in g["circles"]],
                       [c["radius"] for c in g["circles"]])
    x0 = np.array([complex(*p) for p in g["x0"]])
    for case in g["cases"]:
        a, b, c = po.preset(case["algorithm"], case["param"])
        x = x0
        for _ in range(case["steps"]):
            x = toy.step(x, a, b, c)
        exp = np.array([complex(_frac(re), _frac(im)) for re, im in case["expected"]])
        assert np.allclose(x, exp, rtol=0, atol=1e-14), (case["algorithm"], x, exp)
    # the common point, copied into every slot, is a fixed point of any (a, b, c)
    p = np.full(3, complex(*g["common_point"]))
    for abc in [(1, 1, 1), (0.5, 2, 2), (0.3, 1.7, 0.6), (1.2, 0.5, 1.5)]:
        assert np.allclose(toy.step(p, *abc), p)
    # Douglas-Rachford from the worked start: its shadow P_D x reaches the
    # common point; divide and concur settles on a fixed point of its own
    # (the sets are not convex, so that point need not be the intersection)
    x = x0
    for _ in range(400):
        x = toy.step(x, *po.preset("DR"))
    assert np.allclose(toy.divide(x), 0, atol=1e-10)
    x = x0
    for _ in range(400):
        x = toy.step(x, 1, 1, 1)
    assert np.allclose(toy.step(x, 1, 1, 1), x, atol=1e-12)


def _ptycho_ops(seed=10):
    h, w, n, pos, probe, obj, y = _tiny_problem(seed)
    rng = _rng(seed + 1)
    amp = np.abs(_crandn(rng, len(pos), n, n))

    def pd(v):
        return po.modulus_projection(v, amp)

    def pc(v):
        return po.concur(v, obj, probe, pos, update_probe=False)[0]
    return pd, pc, y


def pin_presets_match_textbook_updates():
    """abc with each preset equals the algorithm's own update rule."""
    pd, pc, x = _ptycho_ops()
    beta, lam = 0.75, 0.4
    pdx = pd(x)
    rdx = 2 * pdx - x

    def step(name, param=0.0):
        return po.abc_iteration(x, pd, pc, *po.preset(name, param))[0]
    assert np.allclose(step("DC"), pc(pdx))
    assert np.allclose(step("AR"), pc(rdx))
    assert np.allclose(step("DR"), x + pc(rdx) - pdx)
    assert np.allclose(step("SF"), 2 * pc(pdx) - pdx)
    rc_rd = 2 * pc(rdx) - rdx
    assert np.allclose(step("RAAR", beta), beta / 2 * (rc_rd + x) + (1 - beta) * pdx)
    assert np.allclose(step("RRR", beta), x + beta * (pc(rdx) - pdx))
    assert np.allclose(step("TLAMBDA", lam), pc((1 + lam) * pdx - lam * x) - lam * (pdx - x))
    # RAAR with beta = 1 is Douglas-Rachford
    assert np.allclose(po.preset("RAAR", 1.0), po.preset("DR"))


def pin_true_state_is_fixed_point(scan):
    """Noise-free data: the true (x, O, P) is left unchanged by every preset."""
    amp = scan.amplitude
    st = po.init_state(scan.obj_true, scan.probe_true, scan.pos)
    for name, prm in [("DC", 0), ("AR", 0), ("DR", 0), ("SF", 0), ("RAAR", 0.75),
                      ("RRR", 0.5), ("TLAMBDA", 0.5)]:
        new, info = po.step(st, amp, scan.pos, *po.preset(name, prm), blind=True)
        rx = np.linalg.norm(new.x - st.x) / np.linalg.norm(st.x)
        assert rx < 1e-12, (name, rx)
        assert np.allclose(new.probe, st.probe, rtol=1e-10, atol=1e-10)
        covered = np.zeros(scan.obj_true.shape, bool)
        n = scan.n
        for p, q in scan.pos:
            covered[p:p + n, q:q + n] = True
        assert np.allclose(new.obj[covered], st.obj[covered], rtol=1e-10, atol=1e-10)
        m = info["metrics"]
        assert m["fourier_err"] < 1e-20 and m["consistency_err"] < 1e-20 and m["change"] < 1e-12


# --------------------------------------------------------------------------
# Metrics and division guards (error lines of Figs. 7-8, read as E_F, E_C and
# the change; relative guards), against a hand-derived worked example
# --------------------------------------------------------------------------
def _golden_metrics():
    with open(os.path.join(GOLDEN, "metrics_tiny.json")) as fh:
        return json.load(fh)


def _farr(rows):
    return np.array([[_frac(v) for v in r] for r in rows], dtype=np.float64)


def pin_metrics_worked_example():
    """One step of DC and RAAR(3/4), known and updated probe, on the 2 x 2
    worked example: E_F, E_C, the change and the new (O, P) equal the values
    derived by hand."""
    g = _golden_metrics()
    s = g["start"]
    obj0 = _farr(s["object"]).astype(np.complex128)
    probe0 = _farr(s["probe"]).astype(np.complex128)
    amp = np.stack([_farr(a) for a in s["amplitude"]])
    pos = np.array(s["positions"], dtype=np.int32)
    for case in g["cases"]:
        a, b, c = (_frac(v) for v in case["abc"])
        st = po.init_state(obj0, probe0, pos)
        new, info = po.step(st, amp, pos, a, b, c, blind=case["blind"])
        m = info["metrics"]
        name = case["name"]
        assert m["iteration"] == 0, name
        assert np.isclose(m["fourier_err"], _frac(case["fourier_err"]), rtol=1e-13, atol=0), (name, m)
        assert np.isclose(m["consistency_err"], _frac(case["consistency_err"]), rtol=1e-13, atol=0), (name, m)
        assert np.isclose(m["change"], np.sqrt(_frac(case["change_squared"])), rtol=1e-13, atol=0), (name, m)
        assert np.allclose(new.obj, _farr(case["object"]), rtol=1e-13, atol=1e-15), name
        assert np.allclose(new.probe, _farr(case["probe"]), rtol=1e-13, atol=1e-15), name


def pin_guards_are_relative():
    """The guards compare a denominator with tau times max|P|^2 (object) or
    max|O|^2 (probe): the hand-derived kept/updated pixels, and invariance of
    both steps under a common rescaling of the exit waves and the probe (or
    object), which an absolute threshold would break."""
    g = _golden_metrics()["guard"]
    pos = np.array(_golden_metrics()["start"]["positions"], dtype=np.int32)
    oc = g["object_case"]
    y = np.stack([_farr(v) for v in oc["y"]]).astype(np.complex128)
    got = po.concur_object(y, np.ones((2, 3), complex), _farr(oc["probe"]).astype(complex), pos)
    assert np.allclose(got, _farr(oc["expected"]), rtol=1e-13, atol=0), got
    pc = g["probe_case"]
    y = np.stack([_farr(v) for v in pc["y"]]).astype(np.complex128)
    got = po.concur_probe(y, _farr(pc["object"]).astype(complex), np.ones((2, 2), complex), pos)
    assert np.allclose(got, _farr(pc["expected"]), rtol=1e-13, atol=0), got
    # scale invariance on a random problem whose smallest denominators straddle
    # tau at the extreme scales
    h, w, n, pos, probe, obj, y = _tiny_problem(15)
    o_ref = po.concur_object(y, obj, probe, pos)
    p_ref = po.concur_probe(y, obj, probe, pos)
    for s in (1e-7, 1e7):
        o_s = po.concur_object(s * y, obj, s * probe, pos)
        assert np.allclose(o_s, o_ref, rtol=1e-10, atol=1e-12), s
        p_s = po.concur_probe(s * y, s * obj, probe, pos)
        assert np.allclose(p_s, p_ref, rtol=1e-10, atol=1e-12), s


ALL_PINS = [
    pin_dft_brute_force,
    pin_dft_parseval_delta,
    pin_relaxation_algebra,
    pin_modulus_projection,
    pin_object_step_is_least_squares,
    pin_probe_step_is_least_squares,
    pin_concur_is_average_in_the_plain_case,
    pin_concur_projection_properties,
    pin_concur_sweeps_alternating_least_squares,
    pin_shadow_recovers_the_true_state,
    pin_three_circle_worked_example,
    pin_presets_match_textbook_updates,
    pin_metrics_worked_example,
    pin_guards_are_relative,
]
