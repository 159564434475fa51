"""Helpers for the GPU parity tests: build a scan on the device and the
matching FP64 oracle reference from the same seeded inputs."""
from __future__ import annotations

import numpy as np

from oracle import pty_oracle as po


def rel_l2(got, ref, mask=None):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    if mask is not None:
        got, ref = got[mask], ref[mask]
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_scan(scan, storage="fp32", blind=True, probe_update_start=0, full_metrics=True,
             obj0=None, probe0=None, tau=0.0):
    import torch
    from paper_2311_11466_amd import Scan
    obj0 = scan.obj0 if obj0 is None else obj0
    probe0 = scan.probe0 if probe0 is None else probe0
    return Scan(to_dev(scan.pos.astype(np.int32)), to_dev(scan.intensity.astype(np.float32)),
                to_dev(obj0.astype(np.complex64)), to_dev(probe0.astype(np.complex64)),
                storage=storage, blind=blind, probe_update_start=probe_update_start,
                full_metrics=full_metrics, tau=tau)


def amp32(scan):
    """Amplitudes the GPU sees: sqrt of the float32 intensities (evaluated in float64)."""
    return np.sqrt(scan.intensity.astype(np.float32).astype(np.float64))


def covered_mask(scan):
    m = np.zeros((scan.config.obj_h, scan.config.obj_w), bool)
    n = scan.n
    for p, q in scan.pos:
        m[p:p + n, q:q + n] = True
    return m


def oracle_state_after(scan, k, abc, blind=True, probe0=None):
    """FP64 oracle state after k iterations from the scan's start."""
    st = po.init_state(scan.obj0, scan.probe0 if probe0 is None else probe0, scan.pos)
    return po.run(st, amp32(scan), scan.pos, *abc, k, blind=blind) if k else st


def round_state(st, dtype=np.complex64):
    return po.State(st.x.astype(dtype).astype(np.complex128), st.obj.astype(dtype).astype(np.complex128),
                    st.probe.astype(dtype).astype(np.complex128), st.k)


def fp16_round(a, scale):
    """Round complex values the way FP16 storage does: x * scale to float16 (RNE), back, / scale."""
    a = np.asarray(a, dtype=np.complex128)
    re = (a.real.astype(np.float32) * np.float32(scale)).astype(np.float16).astype(np.float64) / scale
    im = (a.imag.astype(np.float32) * np.float32(scale)).astype(np.float16).astype(np.float64) / scale
    return re + 1j * im


# Single-step parity gate (relative L2), the per-iteration tolerance of the
# float32 path against the FP64 oracle from an identical state.
STEP_GATE = 1e-5
# relative size of the start perturbation used to measure the oracle's own
# amplification of a difference
PERTURB = 1e-7


def trajectory_bound(drift, n_iter, gate=STEP_GATE, eps=PERTURB):
    """Bound of a free-running GPU trajectory against the oracle's, per quantity.

    Linearised error propagation: every GPU iteration differs from the
    oracle's iteration from the same state by at most `gate` (relative; the
    single-step gate), and the oracle itself turns a start difference of
    relative size eps into `drift` after n_iter iterations, i.e. amplifies by
    at most drift / eps (taken as at least 1).  Summing n_iter per-step
    differences, each amplified at most that much, bounds the trajectory
    difference by n_iter * gate * max(drift / eps, 1).  The bound says nothing
    once it reaches order one (strongly amplifying iterations); the tests print
    the measured difference next to it.
    """
    d = np.maximum(np.asarray(drift, dtype=np.float64), eps)
    return n_iter * gate * d / eps


def oracle_drift(run, base_x, compare, seeds=(1, 2), eps=PERTURB):
    """Largest difference `compare(perturbed, reference)` between the oracle run
    from base_x and from base_x perturbed by a relative eps (per seed)."""
    ref = run(base_x)
    worst = None
    for sd in seeds:
        rng = np.random.default_rng(sd)
        b = run(base_x * (1 + eps * rng.standard_normal(base_x.shape)))
        d = np.asarray(compare(b, ref), dtype=np.float64)
        worst = d if worst is None else np.maximum(worst, d)
    return ref, worst
