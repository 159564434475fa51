"""The allocation-free object error (pty_object_error_noalloc) through the C
ABI: on two calls in a row, the second with a smaller box, it equals the
scan-based pty_object_error (same kernels and summation order: bitwise) and
the oracle's aligned error; oversized boxes are rejected before device work."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import gpu_scan, to_dev
from oracle import pty_oracle as po
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu


def test_object_error_noalloc_matches_scan_entry_point():
    import torch
    import paper_2311_11466_amd as pk
    L = pk.load_library()
    scan = make_scan(small_config("na", 64, 4, 24, jitter=1, photons=1e6, seed=91))
    print("case: object error without allocation, N = 64, two calls", flush=True)
    g = gpu_scan(scan)
    g.set_algorithm_named("RAAR", 0.75)
    g.iterate(3)
    obj = g.object()                                   # complex64 device tensor [H, W]
    H, W = obj.shape
    stream = torch.cuda.current_stream()
    err_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    boxes = [(3, 5, H - 9, W - 7), (10, 12, 17, 23)]   # the second smaller
    for r0, c0, h, w in boxes:
        truth = to_dev(np.ascontiguousarray(scan.obj_true[r0:r0 + h, c0:c0 + w]).astype(np.complex64))
        ref = g.object_error(truth, r0, c0)            # the scan-based entry point
        st = L.pty_object_error_noalloc(ctypes.c_void_p(obj.data_ptr()), H, W, ctypes.c_void_p(truth.data_ptr()),
                                        r0, c0, h, w, ctypes.c_void_p(err_dev.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream))
        assert st == 0, L.pty_last_error()
        torch.cuda.synchronize()
        got = float(err_dev.item())
        oracle = po.aligned_error(obj.cpu().numpy()[r0:r0 + h, c0:c0 + w], truth.cpu().numpy())
        print(f"  box {h}x{w}: noalloc {got!r} scan {ref!r} oracle {oracle!r}", flush=True)
        assert np.float64(got).view(np.uint64) == np.float64(ref).view(np.uint64)
        assert abs(got - oracle) <= 1e-9 * max(abs(oracle), 1e-30) + 1e-15
    g.close()


def test_object_error_noalloc_rejects_oversized_box():
    import torch
    import paper_2311_11466_amd as pk
    L = pk.load_library()
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    # 4100 x 4100 > 4096^2 pixels: rejected from the sizes alone, before any launch
    st = L.pty_object_error_noalloc(p, 4100, 4100, p, 0, 0, 4100, 4100, p, None)
    assert st == 1 and b"static scratch" in L.pty_last_error()
    st = L.pty_object_error_noalloc(p, 8, 8, p, 4, 4, 8, 8, p, None)    # box outside the object
    assert st == 1
