"""GPU parity of the algorithm-comparison harness (error lines of Figs. 7-8).

The object error kernel against the oracle's aligned error on the same
float32 arrays, and the harness's per-iteration Fourier and object error
lines against the oracle's runs of the same presets (the linearised
trajectory bound: single-step gate times the oracle's own amplification of a
1e-7 start perturbation, per iteration).
"""
import sys

import numpy as np
import pytest

from gpu_helpers import amp32, gpu_scan, rel_l2, to_dev, trajectory_bound
from oracle import pty_oracle as po
from ptysynth import comparison_config, make_scan

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small_scan():
    return make_scan(comparison_config("small"))


def test_object_error_matches_oracle(small_scan):
    scan = small_scan
    say("case: object error kernel")
    r0, r1, c0, c1 = scan.metric_box()
    rng = np.random.default_rng(3)
    truth = scan.obj_true[r0:r1, c0:c1].astype(np.complex64)
    g = gpu_scan(scan)
    for est in (scan.obj_true * (0.4 - 1.1j), scan.obj_true + 0.05 * rng.standard_normal(scan.obj_true.shape),
                scan.obj0, np.zeros_like(scan.obj0)):
        est32 = est.astype(np.complex64)
        g.set_state(to_dev(po.exit_waves(est32, scan.probe0, scan.pos).astype(np.complex64)), None,
                    to_dev(est32), to_dev(scan.probe0.astype(np.complex64)))
        got = g.object_error(to_dev(truth), r0, c0)
        ref = po.aligned_error(est32[r0:r1, c0:c1], truth)
        say("  gpu", got, "oracle", ref)
        assert abs(got - ref) <= 1e-9 * max(ref, 1e-6), (got, ref)
    g.close()


def test_error_lines_match_oracle(small_scan):
    from paper_2311_11466_amd.compare import error_lines
    scan = small_scan
    algs = (("DC", 0.0), ("RAAR", 0.75), ("TLAMBDA", 0.5))
    n_iter = 12
    box = scan.metric_box()
    r0, r1, c0, c1 = box
    say("case: error lines", [a for a, _ in algs], n_iter)
    lines = error_lines(scan.pos, scan.intensity.astype(np.float32), scan.obj0, scan.probe0, scan.obj_true, box,
                        algorithms=algs, n_iter=n_iter, timed=False)
    amp = amp32(scan)
    truth = scan.obj_true[r0:r1, c0:c1]
    for (name, prm), (lab, got) in zip(algs, lines.items()):
        abc = po.preset(name, prm)

        def run(x_scale):
            st = po.init_state(scan.obj0.astype(np.complex64).astype(np.complex128),
                               scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos)
            if x_scale is not None:
                st.x = st.x * x_scale
            ef, eo = [], []
            for _ in range(n_iter):
                st, info = po.step(st, amp, scan.pos, *abc)
                ef.append(info["metrics"]["fourier_err"])
                eo.append(po.aligned_error(st.obj[r0:r1, c0:c1], truth))
            return np.array(ef), np.array(eo)
        ef_r, eo_r = run(None)
        drift = np.zeros(2)
        for sd in (1, 2, 3):
            rng = np.random.default_rng(sd)
            ef_p, eo_p = run(1 + 1e-7 * rng.standard_normal((scan.n_pos, scan.n, scan.n)))
            drift = np.maximum(drift, [np.max(np.abs(ef_p - ef_r) / ef_r), np.max(np.abs(eo_p - eo_r) / eo_r)])
        tol = trajectory_bound(drift, n_iter)
        errs = np.array([np.max(np.abs(np.array(got["fourier_err"]) - ef_r) / ef_r),
                         np.max(np.abs(np.array(got["object_err"]) - eo_r) / eo_r)])
        say(f"  {lab}: E_F/E_O line errors", errs, "bound", tol)
        assert len(got["fourier_err"]) == n_iter and len(got["object_err"]) == n_iter
        assert np.all(errs <= tol), (lab, errs, tol)
