"""Synthetic scans: the five workloads of the hot path plus small test scans.

Recipe (the paper's experiment section describes a simulated specimen, two
probe sizes and a raster scan but gives no sizes, so every number below is a
stated reading):

* Object: amplitude drawn i.i.d. uniform on [0.5, 1] and phase uniform on
  [-pi/2, pi/2]; each map is smoothed with a separable Gaussian (sigma 3 px,
  taps truncated at +-12 px, circular boundary) and then min-max rescaled
  back onto its interval.
* Probe: a disc of radius r about pixel (N/2, N/2) times the quadratic phase
  exp(i * phi_edge * (rho / r)**2).
* Scan: a row-major raster of top-left corners centred in the object, with
  independent integer jitter uniform on {-k..k} per axis.
* Data: far-field intensities |F(P * O_j)|**2 with F the unnormalised 2-D DFT
  (zero frequency at index [0, 0], no shift).  With photon noise, one global
  factor scales the mean pattern total to the requested photon count and the
  counts are drawn from a Poisson law; the true probe is scaled by the
  square root of that factor so that it stays consistent with the data.
* Start: object of ones; probe a flat disc (radius 8 for the tiny scan,
  0.8 r otherwise) scaled so its energy matches the data by Parseval,
  sum |P0|**2 = mean_j sum_u I_j(u) / N**2.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import scipy.fft
import scipy.ndimage


def _workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return 1


@dataclass(frozen=True)
class ScanConfig:
    name: str
    obj_h: int
    obj_w: int
    n: int
    raster: tuple          # (rows, cols) of the scan raster
    step: int              # raster pitch in pixels
    jitter: int            # integer jitter, uniform on {-jitter..jitter}
    probe_radius: float
    probe_edge_phase: float
    photons: Optional[float]          # None: noise-free data
    seed_obj: int
    seed_pos: int
    seed_noise: Optional[int]
    init_probe_radius: float
    n_pos: Optional[int] = None       # truncate the raster to this many positions


# The five workloads.  tiny_n32 and fp16_n32 share one scan.
CONFIGS = {
    "tiny_n32": ScanConfig("tiny_n32", 128, 128, 32, (8, 8), 12, 1, 10.0, 0.5,
                           None, 101, 102, None, 8.0),
    "scan_n128": ScanConfig("scan_n128", 1024, 1024, 128, (32, 32), 28, 2, 56.0,
                            3 * math.pi, 1e6, 201, 202, 203, 0.8 * 56.0),
    "large_n256": ScanConfig("large_n256", 4096, 4096, 256, (64, 64), 56, 3, 112.0,
                             3 * math.pi, 1e4, 301, 302, 303, 0.8 * 112.0),
    "fp16_n32": ScanConfig("fp16_n32", 128, 128, 32, (8, 8), 12, 1, 10.0, 0.5,
                           None, 101, 102, None, 8.0),
}


@dataclass
class Scan:
    config: ScanConfig
    obj_true: np.ndarray        # complex128 [H, W]
    probe_true: np.ndarray      # complex128 [N, N]
    pos: np.ndarray             # int32 [J, 2], (row, col) of each patch's top-left
    intensity: np.ndarray       # float64 or float32 [J, N, N], unshifted
    obj0: np.ndarray            # complex128 [H, W], starting object
    probe0: np.ndarray          # complex128 [N, N], starting probe
    scale: float = 1.0          # photon scale applied to the data (1 if noise-free)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.config.n

    @property
    def n_pos(self) -> int:
        return int(self.pos.shape[0])

    @property
    def amplitude(self) -> np.ndarray:
        """sqrt of the intensities in float64 (a measurement transform only)."""
        return np.sqrt(np.asarray(self.intensity, dtype=np.float64))

    def metric_box(self):
        """Object rows/cols spanned by the probe centres: (r0, r1, c0, c1), half-open."""
        h = self.n // 2
        r0 = int(self.pos[:, 0].min()) + h
        r1 = int(self.pos[:, 0].max()) + h + 1
        c0 = int(self.pos[:, 1].min()) + h
        c1 = int(self.pos[:, 1].max()) + h + 1
        return r0, r1, c0, c1


def _gauss_taps(sigma: float = 3.0, half: int = 12) -> np.ndarray:
    t = np.arange(-half, half + 1, dtype=np.float64)
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    return g / g.sum()


def _rescale(v: np.ndarray, lo: float, hi: float) -> np.ndarray:
    vmin, vmax = float(v.min()), float(v.max())
    if vmax - vmin <= 0:
        return np.full_like(v, 0.5 * (lo + hi))
    return lo + (hi - lo) * (v - vmin) / (vmax - vmin)


def smooth_object(h: int, w: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.0, size=(h, w))
    pha = rng.uniform(-math.pi / 2, math.pi / 2, size=(h, w))
    taps = _gauss_taps()
    out = []
    for m in (amp, pha):
        m = scipy.ndimage.convolve1d(m, taps, axis=0, mode="wrap")
        m = scipy.ndimage.convolve1d(m, taps, axis=1, mode="wrap")
        out.append(m)
    amp = _rescale(out[0], 0.5, 1.0)
    pha = _rescale(out[1], -math.pi / 2, math.pi / 2)
    return amp * np.exp(1j * pha)


def disc_probe(n: int, radius: float, edge_phase: float = 0.0) -> np.ndarray:
    u = np.arange(n, dtype=np.float64) - n / 2
    rho2 = u[:, None] ** 2 + u[None, :] ** 2
    inside = rho2 <= radius * radius
    phase = edge_phase * rho2 / (radius * radius)
    return np.where(inside, np.exp(1j * phase), 0.0).astype(np.complex128)


def raster_positions(h: int, w: int, n: int, rows: int, cols: int, step: int,
                     jitter: int, seed: int, n_pos: Optional[int] = None) -> np.ndarray:
    """Row-major jittered raster of patch top-left corners, centred in the object."""
    rng = np.random.default_rng(seed)
    span_r = (rows - 1) * step + n
    span_c = (cols - 1) * step + n
    off_r = (h - span_r) // 2
    off_c = (w - span_c) // 2
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    base = np.stack([off_r + ii.ravel() * step, off_c + jj.ravel() * step], axis=1)
    jit = rng.integers(-jitter, jitter + 1, size=base.shape) if jitter > 0 else 0
    pos = (base + jit).astype(np.int64)
    if n_pos is not None:
        pos = pos[:n_pos]
    pos = np.clip(pos, 0, [h - n, w - n])
    return pos.astype(np.int32)


def far_field_intensity(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray,
                        dtype=np.float64, chunk: int = 256) -> np.ndarray:
    """|F(P * O[p:p+N, q:q+N])|**2 for every position (the forward model of the data)."""
    n = probe.shape[0]
    out = np.empty((pos.shape[0], n, n), dtype=dtype)
    rr = np.arange(n)
    for s in range(0, pos.shape[0], chunk):
        p = pos[s:s + chunk]
        patches = obj[p[:, 0, None, None] + rr[None, :, None],
                      p[:, 1, None, None] + rr[None, None, :]]
        f = scipy.fft.fft2(patches * probe[None], axes=(-2, -1), workers=_workers())
        out[s:s + chunk] = (f.real ** 2 + f.imag ** 2).astype(dtype)
    return out


def initial_guess(intensity: np.ndarray, n: int, radius: float, h: int, w: int):
    """Object of ones and a flat disc probe whose energy matches the data."""
    p0 = disc_probe(n, radius, 0.0)
    mean_total = float(np.mean(np.sum(intensity, axis=(1, 2), dtype=np.float64)))
    energy = np.sum(np.abs(p0) ** 2)
    p0 = p0 * math.sqrt(mean_total / (n * n) / energy)
    return np.ones((h, w), dtype=np.complex128), p0


def make_scan(cfg, intensity_dtype=np.float64) -> Scan:
    """Build a scan from a ScanConfig or the name of one in CONFIGS."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    obj = smooth_object(cfg.obj_h, cfg.obj_w, cfg.seed_obj)
    probe = disc_probe(cfg.n, cfg.probe_radius, cfg.probe_edge_phase)
    pos = raster_positions(cfg.obj_h, cfg.obj_w, cfg.n, cfg.raster[0], cfg.raster[1],
                           cfg.step, cfg.jitter, cfg.seed_pos, cfg.n_pos)
    scale = 1.0
    if cfg.photons is None:
        inten = far_field_intensity(obj, probe, pos, dtype=intensity_dtype)
    else:
        inten = far_field_intensity(obj, probe, pos, dtype=np.float64)
        mean_total = float(np.mean(np.sum(inten, axis=(1, 2))))
        scale = cfg.photons / mean_total
        rng = np.random.default_rng(cfg.seed_noise)
        inten = rng.poisson(inten * scale).astype(intensity_dtype)
        probe = probe * math.sqrt(scale)
    obj0, probe0 = initial_guess(inten, cfg.n, cfg.init_probe_radius, cfg.obj_h, cfg.obj_w)
    return Scan(cfg, obj, probe, pos, inten, obj0, probe0, scale)


def small_config(name: str, n: int, raster: int, step: int, jitter: int = 1,
                 photons: Optional[float] = None, seed: int = 7, n_pos: Optional[int] = None,
                 margin: int = 4) -> ScanConfig:
    """A compact scan of the same recipe (used for parity cases that span several tiles)."""
    span = (raster - 1) * step + n + 2 * jitter + 2 * margin
    r = 0.4375 * n
    return ScanConfig(name, span, span, n, (raster, raster), step, jitter, r, 0.5 * math.pi,
                      photons, seed, seed + 1, seed + 2 if photons else None, 0.8 * r, n_pos)


def comparison_config(probe: str, photons: Optional[float] = 1e6) -> ScanConfig:
    """The algorithm comparison of the paper's Figs. 7-8: one synthetic object
    and raster, measured with a big or a small probe (the two probes of
    Fig. 6).  N = 64, a 16 x 16 raster of pitch 12; probe radius 24 (linear
    overlap 75 %) or 12 (50 %); Poisson data at `photons` per pattern."""
    if probe not in ("big", "small"):
        raise ValueError("probe must be 'big' or 'small'")
    n, raster, step, jitter, margin = 64, 16, 12, 1, 4
    span = (raster - 1) * step + n + 2 * jitter + 2 * margin
    r = 24.0 if probe == "big" else 12.0
    return ScanConfig(f"compare_{probe}", span, span, n, (raster, raster), step, jitter, r, 0.5 * math.pi,
                      photons, 601, 602, 603 if photons else None, 0.8 * r)


def make_request(i: int, base_seed: int = 501000):
    """One request of the served mixed load: (ScanConfig, algorithm name, parameter).

    N uniform over {64, 128, 256}; J uniform over 100..2000 on a jittered raster
    of about 70 % linear overlap; photons log-uniform over 1e4..1e7; algorithm
    drawn from the six named ones with a random valid parameter.
    """
    rng = np.random.default_rng(base_seed + i)
    n = int(rng.choice([64, 128, 256]))
    j = int(rng.integers(100, 2001))
    photons = float(10 ** rng.uniform(4, 7))
    r = 0.4375 * n
    step = int(round(0.3 * 2 * r))
    jitter = {64: 1, 128: 2, 256: 3}[n]
    cols = int(math.ceil(math.sqrt(j)))
    rows = int(math.ceil(j / cols))
    span = (max(rows, cols) - 1) * step + n
    hw = span + 2 * jitter + 8
    algo = str(rng.choice(["DC", "AR", "DR", "SF", "RAAR", "RRR"]))
    param = 0.0
    if algo == "RAAR":
        param = float(rng.uniform(0.5, 0.95))
    elif algo == "RRR":
        param = float(rng.uniform(0.3, 1.0))
    cfg = ScanConfig(f"req{i}", hw, hw, n, (rows, cols), step, jitter, r, 3 * math.pi,
                     photons, base_seed + i, base_seed + i + 7, base_seed + i + 13,
                     0.8 * r, j)
    return cfg, algo, param


def with_positions(cfg: ScanConfig, n_pos: int) -> ScanConfig:
    return replace(cfg, n_pos=n_pos)
