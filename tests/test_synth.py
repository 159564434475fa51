"""CPU tests of the seeded synthetic-scan generator."""
import numpy as np

from ptysynth import make_scan, make_request, CONFIGS
from ptysynth.scans import small_config, raster_positions


def test_tiny_scan_recipe():
    s = make_scan("tiny_n32")
    c = s.config
    assert s.pos.shape == (64, 2) and s.pos.dtype == np.int32
    assert s.intensity.shape == (64, 32, 32)
    assert (s.pos >= 0).all() and (s.pos[:, 0] <= c.obj_h - c.n).all() and (s.pos[:, 1] <= c.obj_w - c.n).all()
    amp = np.abs(s.obj_true)
    assert np.isclose(amp.min(), 0.5) and np.isclose(amp.max(), 1.0)
    ph = np.angle(s.obj_true)
    assert np.isclose(ph.min(), -np.pi / 2) and np.isclose(ph.max(), np.pi / 2)
    # probe support is the r = 10 disc, unit modulus inside
    assert np.sum(np.abs(s.probe_true) > 0) == np.sum(
        (np.arange(32)[:, None] - 16) ** 2 + (np.arange(32)[None, :] - 16) ** 2 <= 100)
    # start probe energy matches the data (Parseval)
    assert np.isclose(np.sum(np.abs(s.probe0) ** 2) * 32 * 32, np.mean(s.intensity.sum(axis=(1, 2))))
    assert np.all(s.obj0 == 1)


def test_reproducible_and_seeded():
    a = make_scan("tiny_n32")
    b = make_scan("tiny_n32")
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.intensity, b.intensity)


def test_raster_jitter_range():
    pos = raster_positions(1024, 1024, 128, 32, 32, 28, 2, 202)
    base_r = (1024 - (31 * 28 + 128)) // 2 + np.repeat(np.arange(32), 32) * 28
    base_c = (1024 - (31 * 28 + 128)) // 2 + np.tile(np.arange(32), 32) * 28
    jr, jc = pos[:, 0] - base_r, pos[:, 1] - base_c
    assert jr.min() == -2 and jr.max() == 2 and jc.min() == -2 and jc.max() == 2


def test_poisson_photon_scale():
    cfg = small_config("t", 64, 4, 24, photons=1e6, seed=11)
    s = make_scan(cfg)
    tot = s.intensity.sum(axis=(1, 2))
    assert abs(tot.mean() / 1e6 - 1) < 0.01
    assert np.all(s.intensity == np.round(s.intensity))


def test_requests_are_valid():
    for i in range(12):
        cfg, algo, prm = make_request(i)
        assert cfg.n in (64, 128, 256) and 100 <= cfg.n_pos <= 2000
        assert algo in ("DC", "AR", "DR", "SF", "RAAR", "RRR")
        rows, cols = cfg.raster
        assert rows * cols >= cfg.n_pos
        pos = raster_positions(cfg.obj_h, cfg.obj_w, cfg.n, rows, cols, cfg.step, cfg.jitter,
                               cfg.seed_pos, cfg.n_pos)
        assert pos.shape[0] == cfg.n_pos
        assert (pos >= 0).all() and (pos[:, 0] <= cfg.obj_h - cfg.n).all()


def test_config_table():
    assert CONFIGS["scan_n128"].raster == (32, 32) and CONFIGS["large_n256"].n == 256
