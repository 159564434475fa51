"""The C ABI: every symbol include/ptyabc.h declares is exported, and the
host-side argument checks work without a GPU (no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_11466_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptyabc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pty_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("library not built")
    return pk.load_library()


def test_header_matches_binding_list():
    assert declared_functions() == sorted(pk.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(**kw):
    d = pk.ScanDesc(n=32, n_pos=4, obj_h=64, obj_w=64, storage=0, blind=1, full_metrics=1)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_bytes_host_only(lib):
    d = _desc()
    b = lib.pty_workspace_bytes(ctypes.byref(d))
    assert b > 0 and b % 256 == 0
    # x, y (8 B), sqrt(I) (4 B) per pattern pixel at least
    assert b >= 4 * 32 * 32 * (8 + 8 + 4)
    d16 = _desc(storage=1)
    assert lib.pty_workspace_bytes(ctypes.byref(d16)) < b
    # bigger problems need more
    assert lib.pty_workspace_bytes(ctypes.byref(_desc(n_pos=400))) > b


@pytest.mark.parametrize("field,value", [("n", 48), ("n", 512), ("n_pos", 0), ("obj_h", 16),
                                         ("storage", 2), ("blind", 3), ("tau", -1.0),
                                         ("tau", float("nan")), ("metric_capacity", -1),
                                         ("n_pos", 2 ** 30)])   # (position, tile) pairs beyond int
def test_invalid_desc_rejected(lib, field, value):
    d = _desc(**{field: value})
    assert lib.pty_workspace_bytes(ctypes.byref(d)) == 0
    out = ctypes.c_void_p()
    st = lib.pty_create_scan(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(out))
    assert st == 1 and not out.value
    assert len(lib.pty_last_error()) > 0


def test_null_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.pty_create_scan(None, None, 0, None, ctypes.byref(out)) == 1
    assert lib.pty_iterate(None, 1) == 1
    assert lib.pty_set_algorithm(None, 1.0, 1.0, 1.0) == 1
    assert lib.pty_get_iteration(None) == -1
    assert lib.pty_iterate_schedule(None, None, 1) == 1
    assert lib.pty_set_concur_sweeps(None, 2) == 1
    assert lib.pty_shadow(None, None, None) == 1
    assert lib.pty_sp_iterate(None, None, 0, 1.0, 1.0) == 1
    assert lib.pty_sp_last_batches(None) == -1
    lib.pty_destroy_scan(None)  # no-op


def test_status_strings(lib):
    for code, text in pk.STATUS.items():
        assert lib.pty_status_string(code).decode() == text
    assert lib.pty_status_string(99).decode() == "unknown status"


def test_positions_checked_before_device_work(lib):
    """A window outside the object is rejected from host data, touching no GPU."""
    n, j = 32, 2
    pos = np.array([[0, 0], [40, 0]], np.int32)   # 40 + 32 > 64
    inten = np.ones((j, n, n), np.float32)
    obj = np.ones((64, 64), np.complex64)
    prb = np.ones((n, n), np.complex64)
    d = _desc(n_pos=j, pos=pos.ctypes.data, intensity=inten.ctypes.data, init_object=obj.ctypes.data,
              init_probe=prb.ctypes.data)
    out = ctypes.c_void_p()
    st = lib.pty_create_scan(ctypes.byref(d), ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(out))
    assert st == 1 and b"outside" in lib.pty_last_error()


def test_named_algorithms_match_oracle_presets(lib):
    """The library's (a, b, c) table (pty_algorithm_abc, a host-only call)
    equals the oracle's presets, which the pins tie to each algorithm's
    textbook update."""
    from oracle import pty_oracle as po
    for name, code in pk.ALGORITHMS.items():
        for prm in (0.0, 0.3, 0.5, 0.75, 1.0):
            out = (ctypes.c_double * 3)()
            assert lib.pty_algorithm_abc(code, prm, out) == 0
            assert tuple(out) == pytest.approx(po.preset(name, prm), rel=0, abs=1e-15), (name, prm)
    out = (ctypes.c_double * 3)()
    assert lib.pty_algorithm_abc(99, 0.5, out) == 1
    assert lib.pty_algorithm_abc(0, float("nan"), out) == 1
    assert lib.pty_algorithm_abc(0, 0.5, None) == 1
    assert lib.pty_state_form(None) == -1


def test_algorithmic_bytes_model():
    import bench
    ab = bench.algorithmic_bytes

    def per_px(n, abc, storage="fp32", full=True, form="x", blind=True):
        return sum(ab(k, n, 1, abc, blind, storage, full, form) for k in ("divide", "object", "probe")) // (n * n)
    raar, dc, sf = (0.5, 1.5, 2.0), (1, 1, 1), (1, 2, 1)
    # blind, general (a, b, c), float32: 52 bytes per pattern pixel; the divide alone 36
    assert per_px(128, raar) == 52 and ab("divide", 256, 1, raar, True, "fp32", True, "x") == 36 * 256 * 256
    assert per_px(128, raar, "fp16") == 28
    # a = b = 1 without full metrics: x is not kept, y and sqrt(I) only
    assert per_px(64, dc, full=False) == 28
    assert per_px(64, dc, full=False, blind=False) == 20
    # blend form: w and sqrt(I) in, w and y out, then y twice: 44 (float32), 24 (float16)
    assert per_px(64, raar, full=False, form="w") == 44
    assert per_px(64, raar, "fp16", full=False, form="w") == 24
    # SF (a = 1) in the x form reads y only: 36 + 16 bytes
    assert per_px(128, sf, full=False) == 36


def test_object_error_noalloc_checks_sizes_on_the_host(lib):
    """Oversized or misplaced boxes are rejected from the sizes alone, before
    any device call (the pointers here are never dereferenced)."""
    fake = ctypes.c_void_p(256)
    assert lib.pty_object_error_noalloc(fake, 4100, 4100, fake, 0, 0, 4100, 4100, fake, None) == 1
    assert b"static scratch" in lib.pty_last_error()
    assert lib.pty_object_error_noalloc(fake, 8, 8, fake, 4, 4, 8, 8, fake, None) == 1
    assert lib.pty_object_error_noalloc(None, 8, 8, fake, 0, 0, 8, 8, fake, None) == 1
