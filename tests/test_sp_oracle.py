"""The SP oracle against its pins, and planted mistakes that the pins must catch."""
import numpy as np
import pytest

import sp_pins
from oracle import pty_oracle as po
from oracle import sp_oracle as sp


@pytest.mark.parametrize("pin", sp_pins.SP_PINS, ids=lambda f: f.__name__)
def test_sp_pin(pin):
    pin()


def _iter_factory(slip):
    orig = sp.sp_iteration

    def mutated(obj, probe, pos, amp, batches, alpha=1.0, beta=1.0, blind=True):
        obj = np.array(obj, dtype=np.complex128)
        probe = np.array(probe, dtype=np.complex128)
        amp = np.asarray(amp, dtype=np.float64)
        n = probe.shape[0]
        num = den = 0.0
        for members in batches:
            pmax = float(np.max(np.abs(probe) ** 2))
            dprobe = np.zeros_like(probe)
            new_obj = obj.copy()
            for j in members:
                p, q = int(pos[j][0]), int(pos[j][1])
                o_win = obj[p:p + n, q:q + n]
                psi = probe * o_win
                a, b = po.fourier_error_terms(psi[None], amp[j][None])
                num, den = num + a, den + b
                d = po.modulus_projection(psi[None], amp[j][None])[0] - psi
                cp = probe if slip == "no_conj" else np.conj(probe)
                scale = float(np.max(np.abs(probe))) if slip == "max_not_squared" else pmax
                new_obj[p:p + n, q:q + n] = o_win + alpha * cp * d / scale
                if blind:
                    src = new_obj[p:p + n, q:q + n] if slip == "new_object_in_probe" else o_win
                    omax = float(np.max(np.abs(src) ** 2))
                    dprobe += beta * np.conj(src) * d / omax
            obj = new_obj
            probe = probe + (dprobe if slip != "probe_sign" else -dprobe)
        return obj, probe, num / den
    return mutated


@pytest.mark.parametrize("slip", ["no_conj", "max_not_squared", "new_object_in_probe", "probe_sign"])
def test_sp_mutation_caught(slip, monkeypatch):
    monkeypatch.setattr(sp, "sp_iteration", _iter_factory(slip))
    caught = 0
    for pin in sp_pins.SP_PINS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, slip
