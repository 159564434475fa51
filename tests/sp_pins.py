"""Pins of the SP oracle against facts that do not depend on its code: exact
projections in the constant-modulus cases, the noise-free fixed point, the
equivalence of disjoint batches with the sequential order, linearity in the
relaxation, and the batching invariants."""
from __future__ import annotations

import numpy as np

from oracle import pty_oracle as po
from oracle import sp_oracle as sp


def _rng(seed):
    return np.random.default_rng(seed)


def _cr(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _problem(seed=1, n=8):
    rng = _rng(seed)
    pos = np.array([[0, 0], [0, 5], [5, 0], [5, 5], [3, 3], [9, 9], [0, 10]], dtype=np.int32)
    h = w = 20
    obj = _cr(rng, h, w)
    probe = _cr(rng, n, n)
    amp = np.abs(po.dft2(_cr(rng, len(pos), n, n)))
    return pos, obj, probe, amp, n


def pin_sp_object_step_is_exact_for_constant_modulus_probe():
    pos, obj, _, amp, n = _problem(2)
    rng = _rng(3)
    probe = 2.0 * np.exp(1j * rng.uniform(-np.pi, np.pi, (n, n)))      # |P| = 2 everywhere
    o1, p1, _ = sp.sp_iteration(obj, probe, pos, amp, [[0]], alpha=1.0, blind=False)
    psi = p1 * o1[0:n, 0:n]
    assert np.allclose(np.abs(po.dft2(psi)), amp[0], rtol=1e-10, atol=1e-10)
    mask = np.ones(obj.shape, bool)
    mask[0:n, 0:n] = False
    assert np.array_equal(o1[mask], obj[mask])
    assert np.array_equal(p1, probe)


def pin_sp_probe_step_is_exact_for_constant_modulus_object():
    pos, _, probe, amp, n = _problem(4)
    rng = _rng(5)
    obj = 0.5 * np.exp(1j * rng.uniform(-np.pi, np.pi, (20, 20)))       # |O| = 0.5 everywhere
    o1, p1, _ = sp.sp_iteration(obj, probe, pos, amp, [[3]], alpha=0.0, beta=1.0, blind=True)
    assert np.array_equal(o1, obj)
    psi = p1 * obj[5:5 + n, 5:5 + n]
    assert np.allclose(np.abs(po.dft2(psi)), amp[3], rtol=1e-10, atol=1e-10)


def pin_sp_true_state_is_fixed_point():
    pos, obj, probe, _, n = _problem(6)
    amp = np.abs(po.dft2(po.exit_waves(obj, probe, pos)))
    o1, p1, ef = sp.sp_run(obj, probe, pos, amp, 2, max_batch=1)
    assert np.allclose(o1, obj, rtol=1e-12, atol=1e-12)
    assert np.allclose(p1, probe, rtol=1e-12, atol=1e-12)
    assert max(ef) < 1e-24


def pin_sp_disjoint_batches_equal_sequential_order():
    pos, obj, probe, amp, n = _problem(7)
    rng = _rng(8)
    for _ in range(3):
        order = rng.permutation(len(pos))
        seq = sp.sp_iteration(obj, probe, pos, amp, [[int(j)] for j in order], blind=False)
        bat = sp.sp_iteration(obj, probe, pos, amp, sp.batches_by_level(pos, order, n), blind=False)
        assert np.allclose(seq[0], bat[0], rtol=1e-12, atol=1e-12)
        assert np.isclose(seq[2], bat[2], rtol=1e-12)


def pin_sp_relaxation_is_linear():
    pos, obj, probe, amp, n = _problem(9)
    o1, _, _ = sp.sp_iteration(obj, probe, pos, amp, [[4]], alpha=1.0, blind=False)
    o3, _, _ = sp.sp_iteration(obj, probe, pos, amp, [[4]], alpha=0.3, blind=False)
    o0, _, _ = sp.sp_iteration(obj, probe, pos, amp, [[4]], alpha=0.0, blind=False)
    assert np.array_equal(o0, obj)
    assert np.allclose(o3 - obj, 0.3 * (o1 - obj), rtol=1e-12, atol=1e-12)


def pin_sp_batching_invariants():
    rng = _rng(10)
    n = 16
    pos = np.stack([rng.integers(0, 80, 60), rng.integers(0, 80, 60)], axis=1)
    for max_batch in (0, 1, 3):
        order = rng.permutation(len(pos))
        bats = sp.batches_by_level(pos, order, n, max_batch)
        flat = [j for b in bats for j in b]
        assert sorted(flat) == list(range(len(pos)))
        where = {j: k for k, b in enumerate(bats) for j in b}
        for b in bats:
            assert max_batch == 0 or len(b) <= max_batch
            for i in range(len(b)):
                for k in range(i + 1, len(b)):
                    assert not sp.windows_overlap(pos[b[i]], pos[b[k]], n)
        rank = {int(j): r for r, j in enumerate(order)}
        for a in range(len(pos)):
            for b in range(len(pos)):
                if a != b and rank[a] < rank[b] and sp.windows_overlap(pos[a], pos[b], n):
                    assert where[a] < where[b]


def pin_sp_fourier_error_definition():
    pos, obj, probe, amp, n = _problem(11)
    _, _, ef = sp.sp_iteration(obj, probe, pos, amp, [[0, 3, 5]], blind=True)
    psi = po.exit_waves(obj, probe, pos[[0, 3, 5]])
    mag = np.abs(np.fft.fft2(psi))
    ref = np.sum((mag - amp[[0, 3, 5]]) ** 2) / np.sum(amp[[0, 3, 5]] ** 2)
    assert np.isclose(ef, ref, rtol=1e-12)


def pin_sp_blind_step_is_a_gradient_step_at_the_old_point():
    """Blind step for one position: both moves are steepest-descent steps of
    f = sum |psi' - P S_j O|^2 (psi' held fixed) taken at the old (O, P), with
    steps alpha / max|P|^2 and beta / max|S_j O|^2.  The descent direction is
    taken from central differences of f, not from the oracle's expression."""
    pos, obj, probe, amp, n = _problem(12)
    j = 4
    p0, q0 = pos[j]
    o_win = obj[p0:p0 + n, q0:q0 + n]
    target = po.modulus_projection((probe * o_win)[None], amp[j][None])[0]

    def grad(fun, z):
        g = np.zeros_like(z)
        h = 1e-6
        for idx in np.ndindex(z.shape):
            for unit in (1.0, 1j):
                zp, zm = z.copy(), z.copy()
                zp[idx] += h * unit
                zm[idx] -= h * unit
                g[idx] += unit * (fun(zp) - fun(zm)) / (2 * h)
        return g                      # = d f / d Re z + i d f / d Im z = -2 conj(other) (psi' - P O)
    g_p = grad(lambda pp: np.sum(np.abs(target - pp * o_win) ** 2), probe)
    g_o = grad(lambda oo: np.sum(np.abs(target - probe * oo) ** 2), o_win)
    alpha, beta = 0.7, 0.4
    o1, p1, _ = sp.sp_iteration(obj, probe, pos, amp, [[j]], alpha=alpha, beta=beta, blind=True)
    pmax = np.max(np.abs(probe) ** 2)
    omax = np.max(np.abs(o_win) ** 2)
    assert np.allclose(p1 - probe, -0.5 * beta * g_p / omax, rtol=1e-6, atol=1e-7)
    assert np.allclose(o1[p0:p0 + n, q0:q0 + n] - o_win, -0.5 * alpha * g_o / pmax, rtol=1e-6, atol=1e-7)


SP_PINS = [
    pin_sp_blind_step_is_a_gradient_step_at_the_old_point,
    pin_sp_object_step_is_exact_for_constant_modulus_probe,
    pin_sp_probe_step_is_exact_for_constant_modulus_object,
    pin_sp_true_state_is_fixed_point,
    pin_sp_disjoint_batches_equal_sequential_order,
    pin_sp_relaxation_is_linear,
    pin_sp_batching_invariants,
    pin_sp_fourier_error_definition,
]
