"""MI355X (gfx950) library for the generalised 'abc' set-projection iteration of
blind ptychography (Mei & Maiden, "Set projection algorithms for blind
ptychographic phase retrieval").

This module is the Python binding of ``libptyabc.so``: argument marshalling
only.  Every step of the iteration runs in the library's HIP kernels; PyTorch
provides device memory (the scan workspace, input and output tensors) and the
stream.  There is no CPU fallback: without the built library, or without a
GPU, constructing a Scan raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptyabc.so")

PTY_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "device error",
          4: "bad state", 5: "diverged", 6: "unsupported"}
ALGORITHMS = {"DC": 0, "AR": 1, "DR": 2, "SF": 3, "RAAR": 4, "RRR": 5, "TLAMBDA": 6}
STORAGE = {"fp32": 0, "fp16": 1}

# the symbols include/ptyabc.h declares
EXPORTS = [
    "pty_workspace_bytes", "pty_create_scan", "pty_set_algorithm", "pty_set_algorithm_named",
    "pty_iterate", "pty_iterate_many", "pty_synchronize", "pty_get_object", "pty_get_probe",
    "pty_get_metrics", "pty_get_metric_history", "pty_get_iteration", "pty_get_state",
    "pty_set_state", "pty_destroy_scan", "pty_status_string", "pty_last_error",
    "pty_profile", "pty_profile_read", "pty_iterate_schedule", "pty_set_concur_sweeps", "pty_shadow",
    "pty_object_error", "pty_sp_iterate", "pty_sp_last_batches", "pty_algorithm_abc", "pty_state_form",
    "pty_object_error_noalloc",
]
KERNEL_CLASSES = ["divide", "divide_cols", "divide_rows_inv", "object", "probe", "final"]


class PtyError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class ScanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_pos", ctypes.c_int32),
        ("obj_h", ctypes.c_int32), ("obj_w", ctypes.c_int32),
        ("pos", ctypes.c_void_p), ("intensity", ctypes.c_void_p),
        ("init_object", ctypes.c_void_p), ("init_probe", ctypes.c_void_p),
        ("inputs_on_device", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("blind", ctypes.c_int32), ("probe_update_start", ctypes.c_int32),
        ("full_metrics", ctypes.c_int32), ("metric_capacity", ctypes.c_int32),
        ("tau", ctypes.c_double),
    ]


class Metrics(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int64), ("fourier_err", ctypes.c_double),
                ("consistency_err", ctypes.c_double), ("change", ctypes.c_double)]

    def as_dict(self):
        return {"iteration": int(self.iteration), "fourier_err": self.fourier_err,
                "consistency_err": self.consistency_err, "change": self.change}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libptyabc.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2311_11466_amd.build.build() first")
    # torch ships its own HIP runtime under the same sonames as ROCm's.  The
    # library must bind to the runtime torch uses, so torch is imported and
    # its GPU state initialised first; loaded before torch, the library's
    # code objects register with ROCm's runtime and its HIP calls then find no
    # device in a process where torch runs the GPU.
    torch = _torch()
    torch.cuda.is_available()
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.pty_workspace_bytes.argtypes = [ctypes.POINTER(ScanDesc)]
    L.pty_workspace_bytes.restype = ctypes.c_size_t
    L.pty_create_scan.argtypes = [ctypes.POINTER(ScanDesc), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.pty_set_algorithm.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.pty_set_algorithm_named.argtypes = [P, ctypes.c_int32, ctypes.c_double]
    L.pty_iterate.argtypes = [P, ctypes.c_int32]
    L.pty_iterate_many.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.c_int32]
    L.pty_synchronize.argtypes = [P]
    L.pty_get_object.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int32]
    L.pty_get_probe.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int32]
    L.pty_get_metrics.argtypes = [P, ctypes.POINTER(Metrics)]
    L.pty_get_metric_history.argtypes = [P, ctypes.POINTER(Metrics), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]
    L.pty_get_iteration.argtypes = [P]
    L.pty_get_iteration.restype = ctypes.c_int64
    L.pty_get_state.argtypes = [P, P, P, P, P, ctypes.c_int32]
    L.pty_set_state.argtypes = [P, P, P, P, P, ctypes.c_int32]
    L.pty_destroy_scan.argtypes = [P]
    L.pty_destroy_scan.restype = None
    L.pty_status_string.argtypes = [ctypes.c_int32]
    L.pty_status_string.restype = ctypes.c_char_p
    L.pty_last_error.argtypes = []
    L.pty_last_error.restype = ctypes.c_char_p
    L.pty_profile.argtypes = [P, ctypes.c_int32]
    L.pty_iterate_schedule.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    L.pty_set_concur_sweeps.argtypes = [P, ctypes.c_int32]
    L.pty_shadow.argtypes = [P, P, P]
    L.pty_object_error.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_double)]
    L.pty_sp_iterate.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double]
    L.pty_algorithm_abc.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.pty_object_error_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, P, P]
    L.pty_state_form.argtypes = [P]
    L.pty_state_form.restype = ctypes.c_int32
    L.pty_sp_last_batches.argtypes = [P]
    L.pty_sp_last_batches.restype = ctypes.c_int32
    L.pty_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_int32]
    for name in ("pty_profile", "pty_profile_read", "pty_create_scan", "pty_set_algorithm", "pty_set_algorithm_named", "pty_iterate",
                 "pty_iterate_many", "pty_synchronize", "pty_get_object", "pty_get_probe",
                 "pty_get_metrics", "pty_get_metric_history", "pty_get_state", "pty_set_state",
                 "pty_iterate_schedule", "pty_set_concur_sweeps", "pty_shadow", "pty_object_error", "pty_sp_iterate",
                 "pty_algorithm_abc", "pty_object_error_noalloc"):
        getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def _check(status: int, where: str):
    if status != PTY_OK:
        raise PtyError(status, where, load_library().pty_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def algorithm_abc(name: str, param: float = 0.0):
    """(a, b, c) the library uses for a named algorithm (pty_algorithm_abc)."""
    L = load_library()
    out = (ctypes.c_double * 3)()
    _check(L.pty_algorithm_abc(ALGORITHMS[name.upper()], float(param), out), "pty_algorithm_abc")
    return (out[0], out[1], out[2])


class Scan:
    """One ptychographic scan resident on the GPU.

    pos [J, 2] int32, intensity [J, N, N] float32, init_object [H, W] complex64,
    init_probe [N, N] complex64: torch tensors on the GPU (copied) or host
    arrays (numpy or CPU tensors; copied through host memory).
    """

    def __init__(self, pos, intensity, init_object, init_probe, *, storage: str = "fp32",
                 blind: bool = True, probe_update_start: int = 0, full_metrics: bool = True,
                 metric_capacity: int = 0, tau: float = 0.0, device=None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the ptychography library runs only on the device")
        L = load_library()
        self._L = L
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        on_dev = isinstance(intensity, torch.Tensor) and intensity.is_cuda
        if on_dev:
            pos_t = pos.to(self.device, torch.int32).contiguous()
            inten_t = intensity.to(self.device, torch.float32).contiguous()
            obj_t = init_object.to(self.device, torch.complex64).contiguous()
            prb_t = init_probe.to(self.device, torch.complex64).contiguous()
        else:
            pos_t = np.ascontiguousarray(np.asarray(pos), dtype=np.int32)
            inten_t = np.ascontiguousarray(np.asarray(intensity), dtype=np.float32)
            obj_t = np.ascontiguousarray(np.asarray(init_object), dtype=np.complex64)
            prb_t = np.ascontiguousarray(np.asarray(init_probe), dtype=np.complex64)
        j, n, n2 = inten_t.shape
        h, w = obj_t.shape
        if n != n2 or tuple(prb_t.shape) != (n, n) or tuple(pos_t.shape) != (j, 2):
            raise ValueError("shape mismatch among pos, intensity, init_object, init_probe")

        def ptr(a):
            return a.data_ptr() if on_dev else a.ctypes.data

        self._keep = (pos_t, inten_t, obj_t, prb_t)
        d = ScanDesc(n=n, n_pos=j, obj_h=h, obj_w=w, pos=ptr(pos_t), intensity=ptr(inten_t),
                     init_object=ptr(obj_t), init_probe=ptr(prb_t), inputs_on_device=int(on_dev),
                     storage=STORAGE[storage], blind=int(bool(blind)),
                     probe_update_start=int(probe_update_start), full_metrics=int(bool(full_metrics)),
                     metric_capacity=int(metric_capacity), tau=float(tau))
        nbytes = L.pty_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise PtyError(1, "pty_workspace_bytes", L.pty_last_error().decode())
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(L.pty_create_scan(ctypes.byref(d), ctypes.c_void_p(self.workspace.data_ptr()),
                                     ctypes.c_size_t(self.workspace_bytes),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                   "pty_create_scan")
        self._h = handle
        self._keep = None
        self.n, self.n_pos, self.obj_h, self.obj_w = n, j, h, w
        self.storage = storage

    # -- control -----------------------------------------------------------
    def set_algorithm(self, a: float, b: float, c: float):
        _check(self._L.pty_set_algorithm(self._h, float(a), float(b), float(c)), "pty_set_algorithm")

    def set_algorithm_named(self, name: str, param: float = 0.0):
        _check(self._L.pty_set_algorithm_named(self._h, ALGORITHMS[name.upper()], float(param)),
               "pty_set_algorithm_named")

    def iterate(self, n: int = 1):
        _check(self._L.pty_iterate(self._h, int(n)), "pty_iterate")

    def iterate_schedule(self, abcs):
        """One iteration per (a, b, c) triple of abcs, in order."""
        flat = [float(v) for t in abcs for v in t]
        if len(flat) % 3:
            raise ValueError("abcs must hold (a, b, c) triples")
        buf = (ctypes.c_double * max(1, len(flat)))(*flat)
        _check(self._L.pty_iterate_schedule(self._h, buf, len(flat) // 3), "pty_iterate_schedule")

    def set_concur_sweeps(self, sweeps: int):
        _check(self._L.pty_set_concur_sweeps(self._h, int(sweeps)), "pty_set_concur_sweeps")

    def shadow(self):
        """The shadow estimate P_C(P_D x): (object, probe) as complex64 device tensors."""
        o = self._empty(self.obj_h, self.obj_w)
        p = self._empty(self.n, self.n)
        _check(self._L.pty_shadow(self._h, ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(p.data_ptr())),
               "pty_shadow")
        self.synchronize()
        return o, p

    def sp_iterate(self, order=None, max_batch: int = 0, alpha: float = 1.0, beta: float = 1.0) -> int:
        """One iteration of sequential projections (pty_sp_iterate); returns the
        number of batches.  A batch sums the probe steps of its windows, so with
        batched orders beta should be about 1 / (mean batch size), e.g.
        beta = number of batches / n_pos; beta = 1 suits max_batch = 1."""
        if order is None:
            buf = None
        else:
            order = [int(v) for v in order]
            if len(order) != self.n_pos:
                raise ValueError(f"order must hold {self.n_pos} positions")
            buf = (ctypes.c_int32 * len(order))(*order)
        _check(self._L.pty_sp_iterate(self._h, buf, int(max_batch), float(alpha), float(beta)), "pty_sp_iterate")
        return int(self._L.pty_sp_last_batches(self._h))

    def object_error(self, truth_box, r0: int, c0: int) -> float:
        """Aligned error of the current object against truth_box (a complex64
        device tensor [h, w]) placed at (r0, c0)."""
        torch = _torch()
        t = truth_box.contiguous()
        h, w = t.shape
        torch.cuda.current_stream(self.device).synchronize()   # t may come from another stream
        out = ctypes.c_double()
        _check(self._L.pty_object_error(self._h, ctypes.c_void_p(t.data_ptr()), int(r0), int(c0), int(h), int(w),
                                        ctypes.byref(out)), "pty_object_error")
        return float(out.value)

    def synchronize(self):
        _check(self._L.pty_synchronize(self._h), "pty_synchronize")

    def state_form(self) -> str:
        """Exit-wave state the next iteration keeps: "x" or "w" (the blend
        (1-a) x + a(1-b) y), as the library decides it (pty_state_form)."""
        return "w" if self._L.pty_state_form(self._h) == 1 else "x"

    @property
    def iteration(self) -> int:
        return int(self._L.pty_get_iteration(self._h))

    # -- results -----------------------------------------------------------
    def _empty(self, *shape):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.complex64, device=self.device)

    def object(self):
        out = self._empty(self.obj_h, self.obj_w)
        _check(self._L.pty_get_object(self._h, ctypes.c_void_p(out.data_ptr()), out.numel() * 2, 1),
               "pty_get_object")
        return out

    def probe(self):
        out = self._empty(self.n, self.n)
        _check(self._L.pty_get_probe(self._h, ctypes.c_void_p(out.data_ptr()), out.numel() * 2, 1),
               "pty_get_probe")
        return out

    def metrics(self, allow_diverged: bool = False):
        m = Metrics()
        st = self._L.pty_get_metrics(self._h, ctypes.byref(m))
        if st == 5 and allow_diverged:
            return m.as_dict()
        _check(st, "pty_get_metrics")
        return m.as_dict()

    def metric_history(self, cap: int = 1 << 20):
        cap = int(min(cap, max(self.iteration, 1)))
        buf = (Metrics * cap)()
        n = ctypes.c_int32()
        _check(self._L.pty_get_metric_history(self._h, buf, cap, ctypes.byref(n)), "pty_get_metric_history")
        return [buf[i].as_dict() for i in range(n.value)]

    def get_state(self):
        """(x, y, object, probe) as complex64 device tensors."""
        x = self._empty(self.n_pos, self.n, self.n)
        y = self._empty(self.n_pos, self.n, self.n)
        o = self._empty(self.obj_h, self.obj_w)
        p = self._empty(self.n, self.n)
        _check(self._L.pty_get_state(self._h, *(ctypes.c_void_p(t.data_ptr()) for t in (x, y, o, p)), 1),
               "pty_get_state")
        return x, y, o, p

    def set_state(self, x, y=None, obj=None, probe=None):
        torch = _torch()

        def dev(t, shape):
            if t is None:
                return None
            t = torch.as_tensor(t).to(self.device, torch.complex64).contiguous()
            if tuple(t.shape) != shape:
                raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
            return t
        wave = (self.n_pos, self.n, self.n)
        ts = [dev(x, wave), dev(y, wave), dev(obj, (self.obj_h, self.obj_w)), dev(probe, (self.n, self.n))]
        torch.cuda.synchronize(self.device)
        ptrs = [ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p() for t in ts]
        _check(self._L.pty_set_state(self._h, *ptrs, 1), "pty_set_state")

    def profile(self, enable: bool = True, every: int = 1):
        """Start (clearing totals) or stop per-kernel HIP-event timing; with
        every = m the launches of every m-th iteration are timed."""
        _check(self._L.pty_profile(self._h, int(every) if enable else 0), "pty_profile")

    def profile_read(self):
        """{kernel class: (total ms, launches)} since profile(True)."""
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self._L.pty_profile_read(self._h, ms, cnt, n), "pty_profile_read")
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "_h", None):
            self._L.pty_destroy_scan(self._h)
            self._h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def iterate_many(scans: Sequence[Scan], n: int):
    """n iterations of each scan, launched interleaved so scans on distinct streams overlap."""
    L = load_library()
    arr = (ctypes.c_void_p * len(scans))(*[s._h for s in scans])
    _check(L.pty_iterate_many(arr, len(scans), int(n)), "pty_iterate_many")


def workspace_bytes(n: int, n_pos: int, obj_h: int, obj_w: int, storage: str = "fp32",
                    metric_capacity: int = 0) -> int:
    """Exact device workspace of a scan of this shape (positions do not matter)."""
    L = load_library()
    d = ScanDesc(n=n, n_pos=n_pos, obj_h=obj_h, obj_w=obj_w, storage=STORAGE[storage], blind=1,
                 full_metrics=1, metric_capacity=metric_capacity)
    return int(L.pty_workspace_bytes(ctypes.byref(d)))


__all__ = ["Scan", "iterate_many", "load_library", "algorithm_abc", "workspace_bytes", "PtyError",
           "EXPORTS", "LIB_PATH"]
