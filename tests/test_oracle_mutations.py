"""Plant plausible mistakes in the oracle (on the CPU) and check a pin catches each.

Every mutation is a copy of an oracle function with one slip in it: a dropped
conjugate, a swapped relaxation, a wrong sign, a missing normalisation.  The
oracle's pins must fail on every one of them; a mutation that survives all
pins would show a blind spot.
"""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import pty_oracle as po
from oracle import toy
from ptysynth import make_scan


def _obj_no_conj(y, obj, probe, pos, tau=po.DEFAULT_TAU):
    n = probe.shape[0]
    num = np.zeros(obj.shape, complex)
    den = np.zeros(obj.shape)
    for j, (p, q) in enumerate(np.asarray(pos)):
        num[p:p + n, q:q + n] += probe * y[j]          # slip: conj dropped
        den[p:p + n, q:q + n] += np.abs(probe) ** 2
    out = obj.copy()
    ok = den > tau * np.max(np.abs(probe) ** 2)
    out[ok] = num[ok] / den[ok]
    return out


def _probe_no_conj(y, obj, probe, pos, tau=po.DEFAULT_TAU):
    n = probe.shape[0]
    num = np.zeros((n, n), complex)
    den = np.zeros((n, n))
    for j, (p, q) in enumerate(np.asarray(pos)):
        o = obj[p:p + n, q:q + n]
        num += o * y[j]                                 # slip: conj dropped
        den += np.abs(o) ** 2
    out = probe.copy()
    ok = den > tau * np.max(np.abs(obj) ** 2)
    out[ok] = num[ok] / den[ok]
    return out


def _probe_den_not_squared(y, obj, probe, pos, tau=po.DEFAULT_TAU):
    n = probe.shape[0]
    num = np.zeros((n, n), complex)
    den = np.zeros((n, n))
    for j, (p, q) in enumerate(np.asarray(pos)):
        o = obj[p:p + n, q:q + n]
        num += np.conj(o) * y[j]
        den += np.abs(o)                                # slip: |O| instead of |O|^2
    out = probe.copy()
    ok = den > tau
    out[ok] = num[ok] / den[ok]
    return out


def _abc_swapped(x, divide, concur, a, b, c):
    y = po.relax(divide, b)(x)                          # slip: b and c swapped
    w = po.relax(concur, c)(y)
    return a * w + (1.0 - a) * x, y


def _abc_blend_sign(x, divide, concur, a, b, c):
    y = po.relax(divide, c)(x)
    w = po.relax(concur, b)(y)
    return a * w - (1.0 - a) * x, y                     # slip: sign of the blend


def _abc_concur_first(x, divide, concur, a, b, c):
    y = po.relax(concur, b)(x)                          # slip: concur before divide
    w = po.relax(divide, c)(y)
    return a * w + (1.0 - a) * x, y


def _relax_wrong(proj, a):
    return lambda x: a * proj(x) + (1.0 + a) * x        # slip: sign


def _modulus_unit(x, amp):
    f = po.dft2(x)
    m = np.abs(f)
    return po.idft2(np.where(m > 0, f / np.where(m > 0, m, 1), 1.0))  # slip: amplitude dropped


def _modulus_unnormalised_inverse(x, amp):
    f = po.dft2(x)
    m = np.abs(f)
    g = np.where(m > 0, amp * f / np.where(m > 0, m, 1), amp)
    n = x.shape[-1]
    return po.idft2(g) * n * n                          # slip: 1/N^2 missing


def _dft_inverse_kernel(x):
    n0, n1 = np.asarray(x).shape[-2:]
    return np.fft.ifft2(x, axes=(-2, -1)) * n0 * n1     # slip: exp(+i...) kernel


def _exit_conj_probe(obj, probe, pos):
    return np.conj(probe)[None] * po.patches(obj, pos, probe.shape[0])  # slip


def _preset_ar_wrong(name, param=0.0):
    if name.upper() == "AR":
        return (1.0, 2.0, 1.0)                          # slip: AR read as SF
    return _orig_preset(name, param)


def _preset_raar_wrong(name, param=0.0):
    if name.upper() == "RAAR":
        return (0.5, param, 2.0)                        # slip: b = beta, not 2 beta
    return _orig_preset(name, param)


_orig_preset = po.preset


def _concur_stale_probe(y, obj, probe, pos, tau=po.DEFAULT_TAU, update_probe=True, sweeps=1):
    obj_new, probe_new = obj, np.array(probe)
    for _ in range(int(sweeps)):
        obj_new = po.concur_object(y, obj_new, probe, pos, tau)    # slip: first probe every sweep
        if update_probe:
            probe_new = po.concur_probe(y, obj_new, probe_new, pos, tau)
    return po.exit_waves(obj_new, probe_new, pos), obj_new, probe_new


def _shadow_no_divide(state, amp, pos, blind=True, tau=po.DEFAULT_TAU, sweeps=1):
    _, o, p = po.concur(state.x, state.obj, state.probe, pos, tau, bool(blind), sweeps)  # slip: P_D skipped
    return o, p


def _step_with(ef_scale=1.0, ef_den_spectrum=False, ec_normalised=True, change_sqrt=True):
    """A copy of the oracle's step with one slip in its metric block."""
    def step(state, amp, pos, a, b, c, blind=True, tau=po.DEFAULT_TAU, probe_update_start=0, sweeps=1):
        amp = np.asarray(amp, dtype=np.float64)
        update_probe = bool(blind) and state.k >= probe_update_start
        out = {}

        def concur_op(y):
            z, o, p = po.concur(y, state.obj, state.probe, pos, tau, update_probe, sweeps)
            out["obj"], out["probe"], out["z"] = o, p, z
            return z
        x = state.x
        mag = np.abs(po.dft2(x))
        ef_num = ef_scale * float(np.sum((mag - amp) ** 2))
        ef_den = float(np.sum(mag * mag)) if ef_den_spectrum else float(np.sum(amp * amp))
        x_next, y = po.abc_iteration(x, lambda v: po.modulus_projection(v, amp), concur_op, a, b, c)
        z = out["z"]
        ec_num = float(np.sum(np.abs(z - y) ** 2))
        ec_den = float(np.sum(np.abs(y) ** 2)) if ec_normalised else 1.0
        dx = float(np.sum(np.abs(x_next - x) ** 2)) / float(np.sum(np.abs(x) ** 2))
        metrics = {"iteration": state.k, "fourier_err": ef_num / ef_den, "consistency_err": ec_num / ec_den,
                   "change": float(np.sqrt(dx)) if change_sqrt else dx}
        new = po.State(x_next, out["obj"], out["probe"], state.k + 1, state.history + [metrics])
        return new, {"y": y, "z": z, "metrics": metrics}
    return step


def _obj_absolute_tau(y, obj, probe, pos, tau=po.DEFAULT_TAU):
    n = probe.shape[0]
    num = np.zeros(obj.shape, complex)
    den = np.zeros(obj.shape)
    for j, (p, q) in enumerate(np.asarray(pos)):
        num[p:p + n, q:q + n] += np.conj(probe) * y[j]
        den[p:p + n, q:q + n] += np.abs(probe) ** 2
    out = np.array(obj, dtype=complex, copy=True)
    ok = den > tau                                      # slip: threshold not relative to max|P|^2
    out[ok] = num[ok] / den[ok]
    return out


def _probe_absolute_tau(y, obj, probe, pos, tau=po.DEFAULT_TAU):
    n = probe.shape[0]
    num = np.zeros((n, n), complex)
    den = np.zeros((n, n))
    for j, (p, q) in enumerate(np.asarray(pos)):
        o = obj[p:p + n, q:q + n]
        num += np.conj(o) * y[j]
        den += np.abs(o) ** 2
    out = np.array(probe, dtype=complex, copy=True)
    ok = den > tau                                      # slip: threshold not relative to max|O|^2
    out[ok] = num[ok] / den[ok]
    return out


MUTATIONS = {
    "object_no_conj": [("concur_object", _obj_no_conj)],
    "probe_no_conj": [("concur_probe", _probe_no_conj)],
    "probe_den_not_squared": [("concur_probe", _probe_den_not_squared)],
    "abc_b_c_swapped": [("abc_iteration", _abc_swapped)],
    "abc_blend_sign": [("abc_iteration", _abc_blend_sign)],
    "abc_concur_first": [("abc_iteration", _abc_concur_first)],
    "relax_sign": [("relax", _relax_wrong)],
    "modulus_amplitude_dropped": [("modulus_projection", _modulus_unit)],
    "modulus_inverse_unnormalised": [("modulus_projection", _modulus_unnormalised_inverse)],
    "dft_sign": [("dft2", _dft_inverse_kernel)],
    "exit_wave_conj_probe": [("exit_waves", _exit_conj_probe)],
    "preset_ar": [("preset", _preset_ar_wrong)],
    "preset_raar": [("preset", _preset_raar_wrong)],
    "concur_sweeps_stale_probe": [("concur", _concur_stale_probe)],
    "shadow_without_divide": [("shadow", _shadow_no_divide)],
    "change_without_sqrt": [("step", _step_with(change_sqrt=False))],
    "fourier_err_doubled": [("step", _step_with(ef_scale=2.0))],
    "fourier_err_over_spectrum_energy": [("step", _step_with(ef_den_spectrum=True))],
    "consistency_err_unnormalised": [("step", _step_with(ec_normalised=False))],
    "object_guard_absolute": [("concur_object", _obj_absolute_tau)],
    "probe_guard_absolute": [("concur_probe", _probe_absolute_tau)],
}


@pytest.fixture(scope="module")
def tiny_scan():
    return make_scan("tiny_n32")


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch, tiny_scan):
    for attr, fn in MUTATIONS[name]:
        monkeypatch.setattr(po, attr, fn)
        if hasattr(toy, attr):
            monkeypatch.setattr(toy, attr, fn)
    checks = list(pins.ALL_PINS) + [lambda: pins.pin_true_state_is_fixed_point(tiny_scan)]
    caught = 0
    for pin in checks:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, f"mutation {name} survived every pin"
