import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture
def rng():
    return np.random.default_rng(12345)


def small_raster(ncomp=3, ny=8, nx=8, ndet=4, sweeps=None, fsample=100.0,
                 fknee=(1.0, 2.0), drift_deg=10.0, white=False, seed=(99, 0),
                 layout="hex", diameter=3.0, sigma_scatter=0.1):
    from synth import raster_scan
    sweeps = ny if sweeps is None else sweeps
    return raster_scan(ncomp=ncomp, ny=ny, nx=nx, ndet=ndet, nsamp=4 * nx * sweeps,
                       fsample=fsample, layout=layout, hex_diameter_px=diameter,
                       sigma=1.0, sigma_scatter=sigma_scatter, fknee=fknee,
                       alpha=-3.0, drift_deg=drift_deg, seed=seed, white=white)
