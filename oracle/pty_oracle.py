"""FP64 CPU oracle of the generalised 'abc' set-projection iteration for blind
ptychography (Mei & Maiden, "Set projection algorithms for blind ptychographic
phase retrieval").

TEST INFRASTRUCTURE ONLY.  This module is the parity authority for the HIP
library; it is imported by the test-suite, by the package smoke check and by
the benchmark's CPU-baseline leg, and by nothing on the product path.  It
shares no code with the GPU implementation.

Every array is complex128 / float64.  Library primitives used as single steps:
``numpy.fft.fft2`` / ``ifft2`` (the unnormalised DFT and its inverse), nothing
else.  No blocking, fusion or reordering beyond what the definitions state.

Where the paper is silent the following readings are taken (they are listed
with their reasons in the design notes):

* Relaxed projection (Introduction): P^a_S x = a P_S x + (1 - a) x, reflection
  R_S = P^2_S.
* Generalised iteration (Introduction, the 'abc' formula):
  x_{k+1} = a P^b_C P^c_D x_k + (1 - a) x_k -- divide first, then concur, then
  the outer a-blend.
* Product space (Introduction, divide and concur): one copy per constraint;
  in ptychography one exit wave per scan position, x = [x_0 .. x_{J-1}].
* Divide (P_D): per exit wave the Fourier-modulus projection
  F^-1[ sqrt(I_j) * F x_j / |F x_j| ], with the phase taken as 0 where
  F x_j = 0 (any phase is a nearest point there).
* Concur (P_C): the paper's plain average generalises to the least-squares
  consensus of the exit waves with a common object O and probe P (the flow of
  the 'abc' method updates probe and object).  Blind: one Gauss-Seidel sweep,
  object from the current probe, then probe from the new object, warm started
  from the stored (O, P).  Divisions are guarded: where the denominator is not
  above tau times the maximum of |P|^2 (object step) or |O|^2 (probe step) the
  old value is kept.  P_C y is then z_j = P S_j O.
* Relaxed concur: P^b_C y = b z + (1 - b) y with z built from the fresh (O, P).
* Metrics: E_F = sum (|F x| - A)^2 / sum A^2 of the current iterate,
  E_C = sum |z - y|^2 / sum |y|^2, change = ||x_{k+1} - x_k|| / ||x_k||.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

DEFAULT_TAU = 1e-10


# --------------------------------------------------------------------------
# Operator algebra (Introduction: relaxed projection and reflection)
# --------------------------------------------------------------------------
def relax(proj: Callable, a: float) -> Callable:
    """P^a_S = a P_S + (1 - a) I."""
    def op(x):
        return a * proj(x) + (1.0 - a) * x
    return op


def reflect(proj: Callable) -> Callable:
    """R_S = P^2_S = 2 P_S - I."""
    return relax(proj, 2.0)


def abc_iteration(x, divide: Callable, concur: Callable, a: float, b: float, c: float):
    """x_{k+1} = a P^b_C P^c_D x_k + (1 - a) x_k (the generalised formula).

    Returns (x_{k+1}, y) with y = P^c_D x_k, so callers can report metrics.
    """
    y = relax(divide, c)(x)
    w = relax(concur, b)(y)
    return a * w + (1.0 - a) * x, y


# Named algorithms as (a, b, c) for the generalised formula.  The paper names
# them and gives (1, 1, 1) for divide and concur; the others are the readings
# that reproduce each algorithm's textbook update (checked in the tests).
def preset(name: str, param: float = 0.0):
    name = name.upper()
    if name == "DC":
        return (1.0, 1.0, 1.0)
    if name == "AR":
        return (1.0, 1.0, 2.0)
    if name == "DR":
        return (0.5, 2.0, 2.0)
    if name == "SF":
        return (1.0, 2.0, 1.0)
    if name == "RAAR":
        return (0.5, 2.0 * param, 2.0)
    if name == "RRR":
        return (param / 2.0, 2.0, 2.0)
    if name in ("TLAMBDA", "T_LAMBDA", "TL"):
        return (1.0 / (1.0 + param), 1.0 + param, 1.0 + param)
    raise ValueError(f"unknown algorithm {name!r}")


# --------------------------------------------------------------------------
# Fourier transforms (library primitives; unnormalised forward, 1/N^2 inverse)
# --------------------------------------------------------------------------
def dft2(x):
    return np.fft.fft2(np.asarray(x, dtype=np.complex128), axes=(-2, -1))


def idft2(f):
    return np.fft.ifft2(np.asarray(f, dtype=np.complex128), axes=(-2, -1))


# --------------------------------------------------------------------------
# Divide: the Fourier-modulus projection of every exit wave
# --------------------------------------------------------------------------
def modulus_projection(x, amp):
    """P_D x: keep the phase of F x_j, impose |F x_j| = A_j (phase 0 where F x_j = 0)."""
    psi = dft2(x)
    mag = np.abs(psi)
    safe = np.where(mag > 0, mag, 1.0)
    psi_new = np.where(mag > 0, amp * psi / safe, amp + 0j)
    return idft2(psi_new)


def fourier_error_terms(x, amp):
    """(sum (|F x| - A)^2, sum A^2) of the current iterate."""
    mag = np.abs(dft2(x))
    return float(np.sum((mag - amp) ** 2)), float(np.sum(amp * amp))


# --------------------------------------------------------------------------
# Concur: overlap consensus with a common object and probe
# --------------------------------------------------------------------------
def patches(obj, pos, n):
    """S_j O for all j: the N x N windows of the object at the scan positions."""
    return np.stack([obj[p:p + n, q:q + n] for p, q in np.asarray(pos)])


def exit_waves(obj, probe, pos):
    """x_j = P * S_j O (the flow's first step: exit waves for all positions)."""
    return probe[None] * patches(obj, pos, probe.shape[0])


def concur_object(y, obj, probe, pos, tau=DEFAULT_TAU):
    """Least-squares object for fixed probe: N_O / D_O, summed over j ascending.

    N_O = sum_j S_j^T (conj(P) y_j),  D_O = sum_j S_j^T |P|^2;
    where D_O <= tau * max|P|^2 the previous object value is kept.
    """
    n = probe.shape[0]
    num = np.zeros(obj.shape, dtype=np.complex128)
    den = np.zeros(obj.shape, dtype=np.float64)
    pc = np.conj(probe)
    p2 = np.abs(probe) ** 2
    for j, (p, q) in enumerate(np.asarray(pos)):
        num[p:p + n, q:q + n] += pc * y[j]
        den[p:p + n, q:q + n] += p2
    thr = tau * float(np.max(p2))
    out = np.array(obj, dtype=np.complex128, copy=True)
    ok = den > thr
    out[ok] = num[ok] / den[ok]
    return out


def concur_probe(y, obj, probe, pos, tau=DEFAULT_TAU):
    """Least-squares probe for fixed object: N_P / D_P, summed over j ascending.

    N_P = sum_j conj(S_j O) y_j,  D_P = sum_j |S_j O|^2;
    where D_P <= tau * max|O|^2 the previous probe value is kept.
    """
    n = probe.shape[0]
    num = np.zeros((n, n), dtype=np.complex128)
    den = np.zeros((n, n), dtype=np.float64)
    for j, (p, q) in enumerate(np.asarray(pos)):
        o = obj[p:p + n, q:q + n]
        num += np.conj(o) * y[j]
        den += np.abs(o) ** 2
    thr = tau * float(np.max(np.abs(obj) ** 2))
    out = np.array(probe, dtype=np.complex128, copy=True)
    ok = den > thr
    out[ok] = num[ok] / den[ok]
    return out


def concur(y, obj, probe, pos, tau=DEFAULT_TAU, update_probe=True, sweeps=1):
    """P_C y: object step, then (blind) probe step, then re-extract the exit waves.

    ``sweeps`` repeats the (object, probe) pair with the same y, each object
    step from the previous sweep's probe (alternating least squares on the
    bilinear consensus; the reading with one sweep is the default).
    Returns (z, O_new, P_new) with z_j = P_new * S_j O_new.
    """
    obj_new, probe_new = obj, np.array(probe)
    for _ in range(int(sweeps)):
        obj_new = concur_object(y, obj_new, probe_new, pos, tau)
        if update_probe:
            probe_new = concur_probe(y, obj_new, probe_new, pos, tau)
    return exit_waves(obj_new, probe_new, pos), obj_new, probe_new


# --------------------------------------------------------------------------
# One iteration of the 'abc' ptychographic method
# --------------------------------------------------------------------------
@dataclass
class State:
    x: np.ndarray           # complex128 [J, N, N]: the product-space iterate x_k
    obj: np.ndarray         # complex128 [H, W]
    probe: np.ndarray       # complex128 [N, N]
    k: int = 0
    history: list = field(default_factory=list)

    def copy(self):
        return State(self.x.copy(), self.obj.copy(), self.probe.copy(), self.k, list(self.history))


def init_state(obj0, probe0, pos) -> State:
    obj0 = np.asarray(obj0, dtype=np.complex128)
    probe0 = np.asarray(probe0, dtype=np.complex128)
    return State(exit_waves(obj0, probe0, pos), obj0.copy(), probe0.copy(), 0)


def step(state: State, amp, pos, a, b, c, blind=True, tau=DEFAULT_TAU,
         probe_update_start=0, sweeps=1):
    """One generalised iteration from (x_k, O_k, P_k).

    Returns (new_state, info) where info holds y = P^c_D x_k, z = P_C y and the
    metrics of this iteration.  The reported object and probe are those of the
    concur step of this iteration.
    """
    amp = np.asarray(amp, dtype=np.float64)
    update_probe = bool(blind) and state.k >= probe_update_start
    out = {}

    def divide(x):
        return modulus_projection(x, amp)

    def concur_op(y):
        z, o, p = concur(y, state.obj, state.probe, pos, tau, update_probe, sweeps)
        out["obj"], out["probe"], out["z"] = o, p, z
        return z

    x = state.x
    ef_num, ef_den = fourier_error_terms(x, amp)
    x_next, y = abc_iteration(x, divide, concur_op, a, b, c)
    z = out["z"]
    ec_num = float(np.sum(np.abs(z - y) ** 2))
    ec_den = float(np.sum(np.abs(y) ** 2))
    dx_num = float(np.sum(np.abs(x_next - x) ** 2))
    dx_den = float(np.sum(np.abs(x) ** 2))
    metrics = {
        "iteration": state.k,
        "fourier_err": ef_num / ef_den if ef_den > 0 else float("nan"),
        "consistency_err": ec_num / ec_den if ec_den > 0 else float("nan"),
        "change": float(np.sqrt(dx_num / dx_den)) if dx_den > 0 else float("nan"),
    }
    new = State(x_next, out["obj"], out["probe"], state.k + 1, state.history + [metrics])
    return new, {"y": y, "z": z, "metrics": metrics}


def run(state: State, amp, pos, a, b, c, n_iter, **kw) -> State:
    for _ in range(n_iter):
        state, _ = step(state, amp, pos, a, b, c, **kw)
    return state


def run_schedule(state: State, amp, pos, abcs, **kw) -> State:
    """Iteration-dependent relaxation: iteration i uses abcs[i] = (a_i, b_i, c_i)."""
    for a, b, c in abcs:
        state, _ = step(state, amp, pos, a, b, c, **kw)
    return state


def shadow(state: State, amp, pos, blind=True, tau=DEFAULT_TAU, sweeps=1):
    """The shadow estimate P_C(P_D x_k): the consensus (O, P) of the unrelaxed
    divide of the current iterate, warm started from the state's (O, P).  At a
    fixed point of the DR family the solution is P_D x*, so this is the
    estimate to report there; the state is not changed."""
    y = modulus_projection(state.x, np.asarray(amp, dtype=np.float64))
    _, o, p = concur(y, state.obj, state.probe, pos, tau, bool(blind), sweeps)
    return o, p


# --------------------------------------------------------------------------
# Evaluation against ground truth (global complex scale removed)
# --------------------------------------------------------------------------
def aligned_error(est, truth):
    """min over complex g of sum |truth - g est|^2 / sum |truth|^2."""
    est = np.asarray(est, dtype=np.complex128).ravel()
    truth = np.asarray(truth, dtype=np.complex128).ravel()
    ee = np.vdot(est, est).real
    if ee == 0:
        return 1.0
    g = np.vdot(est, truth) / ee
    return float(np.sum(np.abs(truth - g * est) ** 2) / np.sum(np.abs(truth) ** 2))
