"""CPU tests: the FP64 oracle against its pins."""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import pty_oracle as po
from ptysynth import make_scan


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


@pytest.fixture(scope="module")
def tiny_scan():
    return make_scan("tiny_n32")


def test_true_state_is_fixed_point(tiny_scan):
    pins.pin_true_state_is_fixed_point(tiny_scan)


def test_known_probe_dc_converges(tiny_scan):
    """Divide and concur with the true probe reduces the object error from the start."""
    s = tiny_scan
    amp = s.amplitude
    st = po.init_state(s.obj0, s.probe_true, s.pos)
    r0, r1, c0, c1 = s.metric_box()
    e0 = po.aligned_error(st.obj[r0:r1, c0:c1], s.obj_true[r0:r1, c0:c1])
    st = po.run(st, amp, s.pos, 1, 1, 1, 50, blind=False)
    e1 = po.aligned_error(st.obj[r0:r1, c0:c1], s.obj_true[r0:r1, c0:c1])
    assert e1 < 0.1 * e0
    ef = [m["fourier_err"] for m in st.history]
    assert ef[-1] < ef[0]


def test_blind_raar_reduces_fourier_error(tiny_scan):
    s = tiny_scan
    st = po.init_state(s.obj0, s.probe0, s.pos)
    st = po.run(st, s.amplitude, s.pos, *po.preset("RAAR", 0.75), 30, blind=True)
    ef = [m["fourier_err"] for m in st.history]
    assert ef[-1] < 0.2 * ef[0]


def test_probe_update_start(tiny_scan):
    """The probe stays at its start value before probe_update_start."""
    s = tiny_scan
    st = po.init_state(s.obj0, s.probe0, s.pos)
    st2 = po.run(st, s.amplitude, s.pos, 1, 1, 1, 3, blind=True, probe_update_start=3)
    assert np.array_equal(st2.probe, s.probe0)
    st3, _ = po.step(st2, s.amplitude, s.pos, 1, 1, 1, blind=True, probe_update_start=3)
    assert not np.allclose(st3.probe, s.probe0)


def test_aligned_error_removes_global_scale():
    rng = np.random.default_rng(0)
    t = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    assert po.aligned_error((0.3 - 2j) * t, t) < 1e-28
    assert po.aligned_error(t + 1, t) > 1e-3


def test_aligned_error_is_the_minimum_over_complex_scale():
    """The closed-form scale agrees with a numerical minimisation over g."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(21)
    t = rng.standard_normal((12, 9)) + 1j * rng.standard_normal((12, 9))
    e = t * (0.7 + 0.2j) + 0.3 * (rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape))

    def f(v):
        g = v[0] + 1j * v[1]
        return float(np.sum(np.abs(t - g * e) ** 2) / np.sum(np.abs(t) ** 2))
    best = minimize(f, [0.0, 0.0], method="Nelder-Mead", options={"xatol": 1e-12, "fatol": 1e-15}).fun
    assert abs(po.aligned_error(e, t) - best) <= 1e-9
    assert po.aligned_error(e, t) <= f([1.0, 0.0])
