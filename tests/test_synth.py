"""Checks of the seeded input generator (not part of either compute path)."""

import numpy as np

from synth import (make_workload, noise_spectrum, draw_noise, hex_focal_plane,
                   raster_scan, crosslinked_torus_scan)


def test_noise_periodogram_matches_spectrum():
    n, fs = 4096, 100.0
    S = noise_spectrum(n, fs, np.array([1.3]), np.array([2.0]))[0]
    rng = np.random.default_rng(7)
    nreal = 400
    acc = np.zeros(n // 2 + 1)
    for _ in range(nreal):
        x = draw_noise(S, rng)
        acc += np.abs(np.fft.rfft(x)) ** 2 / n
    ratio = acc / nreal / S
    # each interior bin: mean of nreal chi^2_2/2 variables, sd 1/sqrt(nreal)
    inner = ratio[1:-1]
    assert abs(inner.mean() - 1) < 0.01
    assert np.all(np.abs(inner - 1) < 6 / np.sqrt(nreal))


def test_spectrum_dc_bin_and_shape():
    S = noise_spectrum(1024, 100.0, np.array([2.0]), np.array([1.0]))[0]
    assert S[0] == S[1]
    f = np.arange(513) * 100.0 / 1024
    np.testing.assert_allclose(S[5], 4.0 * (1 + (f[5] / 1.0) ** -3))


def test_raster_line_four_samples_per_pixel_per_sweep():
    s = make_workload("intensity_small")
    assert s.pix.shape == (8, 2**14)
    # detector 0, row 0 sweep: each of 64 pixels hit exactly 4 times
    row0 = s.pix[0, :256]
    assert np.all(np.bincount(row0, minlength=64)[:64] == 4)
    # detector d sits d rows above: first sweep hits row d
    for d in range(8):
        assert np.all(s.pix[d, :256] // 64 == d)
    # the last 7 detectors leave the map on the top rows
    assert (s.pix[7] < 0).sum() == 7 * 256


def test_hex_focal_plane_diameter():
    dy, dx = hex_focal_plane(256, 60.0, rotation=0.3)
    r = np.hypot(dy, dx)
    assert np.isclose(r.max(), 30.0)
    assert abs(dy.mean()) < 1e-9 and abs(dx.mean()) < 1e-9
    assert len(set(zip(np.round(dy, 6), np.round(dx, 6)))) == 256


def test_seeded_reproducible_and_distinct():
    a = raster_scan(ncomp=3, ny=16, nx=16, ndet=4, nsamp=4 * 16 * 16, fsample=100.0,
                    hex_diameter_px=4.0, drift_deg=10.0, seed=(2, 0))
    b = raster_scan(ncomp=3, ny=16, nx=16, ndet=4, nsamp=4 * 16 * 16, fsample=100.0,
                    hex_diameter_px=4.0, drift_deg=10.0, seed=(2, 0))
    c = raster_scan(ncomp=3, ny=16, nx=16, ndet=4, nsamp=4 * 16 * 16, fsample=100.0,
                    hex_diameter_px=4.0, drift_deg=10.0, seed=(2, 1))
    assert np.array_equal(a.pix, b.pix) and np.array_equal(a.inv_noise, b.inv_noise)
    assert not np.array_equal(a.pix, c.pix)
    np.testing.assert_allclose(a.cos2psi**2 + a.sin2psi**2, 1.0, atol=1e-6)


def test_crosslinked_torus_geometry():
    s = crosslinked_torus_scan(3, L=8, periods=2)
    assert s.ndet == 24
    h = np.bincount(s.pix.ravel(), minlength=64)
    assert np.all(h == h[0])


def test_batch_recipe_is_seeded_and_in_range():
    from synth import batch_scan_spec
    specs = [batch_scan_spec(i) for i in range(64)]
    assert specs == [batch_scan_spec(i) for i in range(64)]
    for sp in specs:
        assert 32 <= sp["ndet"] <= 512
        assert 2**16 <= sp["nsamp"] <= 2**21 and sp["nsamp"] & (sp["nsamp"] - 1) == 0
        assert sp["ny"] == sp["nx"] and 128 <= sp["ny"] <= 1024
        assert sp["hex_diameter_px"] == max(60.0, 8.0 * sp["ny"] ** 2 / sp["nsamp"])
    # uneven: several lengths, detector counts and map sizes
    assert len({sp["nsamp"] for sp in specs}) >= 4 and len({sp["ny"] for sp in specs}) >= 3
