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


def test_algorithmic_bytes_model():
    # blind, general (a, b, c), float32: 52 bytes per pattern pixel
    assert pk.algorithmic_bytes_per_projection(128, 0.5, 1.5) == 52 * 128 * 128
    assert pk.algorithmic_bytes_per_projection(128, 0.5, 1.5, storage="fp16") == 28 * 128 * 128 + 4 * 0
    assert pk.algorithmic_bytes_per_projection(64, 1, 1, full_metrics=False) == 28 * 64 * 64
    assert pk.algorithmic_bytes_per_projection(64, 1, 1, blind=False, full_metrics=False) == 20 * 64 * 64
    # blend form (no full metrics, N <= 64, a != 1, b != 1): w and sqrt(I) in,
    # w and y out, then y twice: 44 bytes (float32), 24 (float16)
    assert pk.algorithmic_bytes_per_projection(64, 0.5, 1.5, full_metrics=False) == 44 * 64 * 64
    assert pk.algorithmic_bytes_per_projection(64, 0.5, 1.5, storage="fp16", full_metrics=False) == 24 * 64 * 64
    # N = 128 and N = 256 keep x (split exchanges; three passes)
    assert pk.algorithmic_bytes_per_projection(128, 0.5, 1.5, full_metrics=False) == 52 * 128 * 128
    assert pk.algorithmic_bytes_per_projection(256, 0.5, 1.5, full_metrics=False) == 52 * 256 * 256
    # SF (a = 1): the x form reads y only, 36 + 16 bytes
    assert pk.algorithmic_bytes_per_projection(128, 1, 2, full_metrics=False) == 36 * 128 * 128
