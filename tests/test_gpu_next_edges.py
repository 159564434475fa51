"""Edge cases of the schedule, shadow, object-error and sequential-projection
entry points (GPU, through the C ABI)."""
import sys

import numpy as np
import pytest

from gpu_helpers import amp32, covered_mask, gpu_scan, rel_l2, to_dev
from oracle import pty_oracle as po
from oracle import sp_oracle as sp
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    return make_scan("tiny_n32")


def test_empty_schedule_is_a_no_op(tiny):
    say("case: empty schedule")
    g = gpu_scan(tiny)
    g.iterate(2)
    before = [t.cpu().numpy() for t in g.get_state()]
    g.iterate_schedule([])
    assert g.iteration == 2
    after = [t.cpu().numpy() for t in g.get_state()]
    for u, v in zip(before, after):
        assert np.array_equal(u.view(np.uint32), v.view(np.uint32))
    g.close()


def test_object_error_box_checks(tiny):
    from paper_2311_11466_amd import PtyError
    say("case: object error boxes")
    g = gpu_scan(tiny)
    h, w = tiny.obj_true.shape
    whole = g.object_error(to_dev(tiny.obj_true.astype(np.complex64)), 0, 0)
    ref = po.aligned_error(tiny.obj0.astype(np.complex64), tiny.obj_true.astype(np.complex64))
    assert abs(whole - ref) <= 1e-9 * ref
    corner = g.object_error(to_dev(tiny.obj_true[h - 5:, w - 7:].astype(np.complex64)), h - 5, w - 7)
    ref = po.aligned_error(tiny.obj0[h - 5:, w - 7:].astype(np.complex64),
                           tiny.obj_true[h - 5:, w - 7:].astype(np.complex64))
    assert abs(corner - ref) <= 1e-9 * max(ref, 1e-6)
    with pytest.raises(PtyError):
        g.object_error(to_dev(tiny.obj_true[:4, :4].astype(np.complex64)), h - 3, 0)
    with pytest.raises(PtyError):
        g.object_error(to_dev(tiny.obj_true[:4, :4].astype(np.complex64)), -1, 0)
    g.close()


def test_shadow_of_a_fresh_scan(tiny):
    say("case: shadow before any iteration")
    g = gpu_scan(tiny)
    o, p = (t.cpu().numpy() for t in g.shadow())
    st = po.init_state(tiny.obj0.astype(np.complex64).astype(np.complex128),
                       tiny.probe0.astype(np.complex64).astype(np.complex128), tiny.pos)
    ro, rp = po.shadow(st, amp32(tiny), tiny.pos)
    errs = (rel_l2(o, ro, covered_mask(tiny)), rel_l2(p, rp))
    say("  errors", errs)
    assert max(errs) <= 1e-5
    assert g.iteration == 0
    g.close()


def test_sp_with_float16_storage(tiny):
    """SP keeps its probe steps in the exit-wave buffers; with float16 storage
    they span x and y.  The object and probe are float32 either way."""
    say("case: SP on a float16-storage scan")
    a = gpu_scan(tiny, storage="fp16")
    b = gpu_scan(tiny, storage="fp32")
    for _ in range(2):
        a.sp_iterate()
        b.sp_iterate()
    oa, pa = a.object().cpu().numpy(), a.probe().cpu().numpy()
    ob, pb = b.object().cpu().numpy(), b.probe().cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(oa.view(np.uint32), ob.view(np.uint32))
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))


def test_sp_single_position():
    scan = make_scan(small_config("one", 64, 1, 10, jitter=0, photons=None, seed=61))
    say("case: SP with one position")
    assert scan.n_pos == 1
    g = gpu_scan(scan)
    nb = g.sp_iterate()
    assert nb == 1
    o, p = g.object().cpu().numpy(), g.probe().cpu().numpy()
    g.close()
    ro, rp, _ = sp.sp_run(scan.obj0.astype(np.complex64).astype(np.complex128),
                          scan.probe0.astype(np.complex64).astype(np.complex128), scan.pos, amp32(scan), 1)
    errs = (rel_l2(o, ro, covered_mask(scan)), rel_l2(p, rp))
    say("  errors", errs)
    assert max(errs) <= 1e-5


def test_sampled_profile(tiny):
    """pty_profile(m): the launches of every m-th iteration are timed."""
    say("case: sampled event timing")
    g = gpu_scan(tiny)
    g.profile(True, every=4)
    g.iterate(9)                    # iterations 0..8: 0, 4 and 8 are timed
    prof = g.profile_read()
    g.profile(False)
    assert prof["divide"][1] == 3 and prof["object"][1] == 3 and prof["final"][1] == 3, prof
    assert all(ms > 0 for ms, n in prof.values() if n)
    g.profile(True)
    g.iterate(2)
    assert g.profile_read()["divide"][1] == 2
    g.close()


def test_metrics_after_sequential_projections(tiny):
    """After an SP iteration the consistency and change slots are NaN (not
    formed); pty_get_metrics still reports success."""
    say("case: metrics after SP")
    g = gpu_scan(tiny, full_metrics=True)
    g.iterate(2)
    g.sp_iterate()
    m = g.metrics()                         # raises on PTY_ERR_DIVERGED
    assert np.isfinite(m["fourier_err"]) and np.isnan(m["consistency_err"]) and np.isnan(m["change"])
    assert m["iteration"] == 2
    g.iterate(1)
    m = g.metrics()
    assert np.isfinite(m["fourier_err"])
    g.close()
