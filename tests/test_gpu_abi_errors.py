"""Error paths of the C ABI on a live scan (GPU): each rejected call returns
its status and leaves the scan as it was, so a scan that saw the bad call
iterates to the same bits as one that did not; a non-finite state is reported
as divergence, not hidden."""
import ctypes
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_scan, to_dev
from ptysynth import make_scan

pytestmark = pytest.mark.gpu

INVALID_ARG, BAD_STATE, DIVERGED = 1, 4, 5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    return make_scan("tiny_n32")


def _bits(g):
    return [t.cpu().numpy().view(np.uint32) for t in g.get_state()]


def _status(exc_info):
    return exc_info.value.status


def test_rejected_calls_leave_the_scan_unchanged(tiny):
    from paper_2311_11466_amd import PtyError
    say("case: rejected set_algorithm / iterate calls on a live scan")
    ref = gpu_scan(tiny)
    ref.set_algorithm_named("RAAR", 0.75)
    ref.iterate(3)
    g = gpu_scan(tiny)
    g.set_algorithm_named("RAAR", 0.75)
    g.iterate(1)
    for abc in [(float("nan"), 1.0, 1.0), (0.0, 1.0, 1.0), (1.0, float("inf"), 1.0), (1.0, 1.0, float("nan"))]:
        with pytest.raises(PtyError) as e:
            g.set_algorithm(*abc)
        assert _status(e) == INVALID_ARG, abc
    with pytest.raises(PtyError) as e:
        g.iterate(-1)
    assert _status(e) == INVALID_ARG
    import paper_2311_11466_amd as pk
    L = pk.load_library()
    assert L.pty_set_algorithm_named(g._h, 99, 0.0) == INVALID_ARG          # no such algorithm
    assert L.pty_set_algorithm_named(g._h, 4, float("nan")) == INVALID_ARG  # RAAR with beta NaN
    assert g.iteration == 1
    g.iterate(2)
    assert g.iteration == 3
    for a, b in zip(_bits(g), _bits(ref)):
        assert np.array_equal(a, b)
    g.close()
    ref.close()


def test_metrics_before_the_first_iteration(tiny):
    from paper_2311_11466_amd import PtyError
    say("case: metrics before any iteration")
    g = gpu_scan(tiny)
    with pytest.raises(PtyError) as e:
        g.metrics()
    assert _status(e) == BAD_STATE
    g.iterate(1)
    m = g.metrics()
    assert m["iteration"] == 0 and np.isfinite(m["fourier_err"])
    g.close()


def test_getters_check_the_destination_size(tiny):
    import paper_2311_11466_amd as pk
    say("case: getters with a too small destination")
    g = gpu_scan(tiny)
    L = pk.load_library()
    h, w = tiny.obj0.shape
    small = (ctypes.c_float * 8)()
    assert L.pty_get_object(g._h, small, 8, 0) == INVALID_ARG
    assert L.pty_get_probe(g._h, small, 8, 0) == INVALID_ARG
    whole = (ctypes.c_float * (2 * h * w))()
    assert L.pty_get_object(g._h, whole, 2 * h * w, 0) == 0
    got = np.frombuffer(whole, dtype=np.complex64).reshape(h, w)
    assert np.array_equal(got.view(np.uint32), tiny.obj0.astype(np.complex64).view(np.uint32))
    g.close()


def test_non_finite_state_is_reported_as_divergence(tiny):
    """An exit wave set to infinity makes the Fourier error of the next
    iteration non-finite: pty_get_metrics returns PTY_ERR_DIVERGED (with the
    metrics filled in) instead of a number, and the scan stays usable."""
    from paper_2311_11466_amd import PtyError
    say("case: divergence is reported")
    g = gpu_scan(tiny)
    x, y, o, p = (t.cpu().numpy() for t in g.get_state())
    x = x.copy()
    x[0, 3, 5] = np.inf
    g.set_state(to_dev(x), None, to_dev(o), to_dev(p))
    g.set_algorithm_named("DC")
    g.iterate(1)
    with pytest.raises(PtyError) as e:
        g.metrics()
    assert _status(e) == DIVERGED
    m = g.metrics(allow_diverged=True)
    assert not np.isfinite(m["fourier_err"])
    g.iterate(1)                                          # still accepts work
    assert g.iteration == 2
    g.close()
