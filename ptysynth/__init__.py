"""Seeded synthetic ptychographic scans.

This package is the only code shared by the FP64 oracle, the tests and the
GPU benchmark.  It simulates the *measurement* (object, probe, scan raster,
far-field intensities, photon noise) and the starting guesses.  It contains
none of the reconstruction arithmetic: no projection, no overlap consensus,
no relaxation.

The scans stand in for the blood-cell simulation of the paper's experiment
section, whose image is not available.
"""
from .scans import (  # noqa: F401
    Scan,
    ScanConfig,
    CONFIGS,
    make_scan,
    make_request,
    comparison_config,
    smooth_object,
    disc_probe,
    raster_positions,
    far_field_intensity,
    initial_guess,
)
