"""Pins of the oracle's convergence diagnostics: Parseval for the binned
spectra, pure E and pure B patterns, the bin a plane wave lands in, the mask,
cosmic-variance units, and the block-averaged crossing step on series with a
known crossing.  (The A-norm estimate is pinned in test_oracle_precon.py.)"""

import numpy as np
import pytest

from oracle import diagnostics as D


def _wide(ny, nx, pix):
    # enough bins of width 10 to hold every mode
    lmax = 2 * np.pi * np.sqrt(0.5) / (pix * D.ARCMIN)
    return 10.0, int(lmax / 10.0) + 2


@pytest.mark.parametrize("ny,nx", [(16, 16), (8, 32)])
def test_parseval_for_all_bins(rng, ny, nx):
    pix = 0.5
    dell, nb = _wide(ny, nx, pix)
    m = rng.standard_normal((3, ny * nx))
    mask = np.ones(ny * nx)
    C, n = D.map_spectra(m, mask, ny, nx, pix, dell, nb)
    assert n.sum() == ny * nx
    norm = (pix * D.ARCMIN) ** 2 / (ny * nx)
    tot = (C * n).sum(axis=1) / norm          # sum of |X(k)|^2 per component
    np.testing.assert_allclose(tot[0], ny * nx * np.sum(m[0] ** 2), rtol=1e-12)
    # the E/B rotation keeps |Q|^2 + |U|^2 mode by mode
    np.testing.assert_allclose(tot[1] + tot[2], ny * nx * np.sum(m[1:] ** 2), rtol=1e-12)


def test_pure_e_and_pure_b_patterns():
    ny, nx, pix = 32, 32, 1.0
    y, x = np.mgrid[0:ny, 0:nx]
    ky, kx = 3, 5                          # integer cycles across the map
    phase = 2 * np.pi * (ky * y / ny + kx * x / nx)
    phi = np.arctan2(ky / ny, kx / nx)
    T = np.zeros((ny, nx))
    e_map = np.stack([T, np.cos(phase) * np.cos(2 * phi), np.cos(phase) * np.sin(2 * phi)])
    b_map = np.stack([T, -np.cos(phase) * np.sin(2 * phi), np.cos(phase) * np.cos(2 * phi)])
    dell, nb = _wide(ny, nx, pix)
    mask = np.ones(ny * nx)
    Ce, _ = D.map_spectra(e_map.reshape(3, -1), mask, ny, nx, pix, dell, nb)
    Cb, _ = D.map_spectra(b_map.reshape(3, -1), mask, ny, nx, pix, dell, nb)
    assert Ce[1].max() > 0 and Ce[2].max() <= 1e-20 * Ce[1].max()
    assert Cb[2].max() > 0 and Cb[1].max() <= 1e-20 * Cb[2].max()
    # all the power sits in the bin of ell = 2 pi |k| / pixel
    ell = 2 * np.pi * np.hypot(ky / ny, kx / nx) / (pix * D.ARCMIN)
    assert np.argmax(Ce[1]) == int(ell // dell)


def test_mask_zeroes_inactive_pixels(rng):
    ny = nx = 16
    m = rng.standard_normal((1, ny * nx))
    mask = (rng.random(ny * nx) > 0.3).astype(float)
    dell, nb = _wide(ny, nx, 0.5)
    a, _ = D.map_spectra(m, mask, ny, nx, 0.5, dell, nb)
    b, _ = D.map_spectra(m * mask, np.ones(ny * nx), ny, nx, 0.5, dell, nb)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=0)


def test_spectrum_error_in_cosmic_variance_units():
    c_in = np.array([2.0, 4.0, 0.0])
    counts = np.array([8.0, 200.0, 10.0])
    e = D.spectrum_error(np.array([3.0, 4.2, 1.0]), c_in, counts)
    np.testing.assert_allclose(e[:2], [1.0 / (2.0 * np.sqrt(2 / 4.0)), 0.2 / (4.0 * np.sqrt(2 / 100.0))])
    assert np.isnan(e[2])


def test_convergence_step_on_known_crossings():
    steps = np.arange(0, 400)
    lin = 1.0 - steps / 200.0                   # crosses 0.1 at step 180
    assert D.convergence_step(steps, lin, 0.1, block=50) == pytest.approx(180.0, abs=1e-9)
    assert D.convergence_step(steps, lin, 0.1, block=1) == pytest.approx(180.0, abs=1e-9)
    assert D.convergence_step(steps, np.full(400, 0.05), 0.1, block=50) == pytest.approx(24.5)
    assert D.convergence_step(steps, np.full(400, 0.5), 0.1) is None
