"""Pins of the oracle's boresight pointing expansion: hand-computed pixels for
an unturned and a quarter-turned focal plane, the pixel-edge rule, the
angle-sum weights against direct trigonometry, and agreement with the
generator's own per-sample pointing (an independent expansion that uses the
angles directly)."""

import math

import numpy as np
import pytest

import oracle
from oracle.boresight import expand_pointing
from conftest import small_raster
from synth import boresight_only


def _bore(yb, xb, phi):
    yb, xb = np.asarray(yb, float), np.asarray(xb, float)
    phi = np.broadcast_to(np.asarray(phi, float), yb.shape)
    return np.stack([yb, xb, np.cos(phi), np.sin(phi), np.cos(2 * phi), np.sin(2 * phi)])


def _dets(dy, dx, psi):
    psi = np.asarray(psi, float)
    return np.stack([np.asarray(dy, float), np.asarray(dx, float), np.cos(2 * psi),
                     np.sin(2 * psi)])


def test_unturned_focal_plane():
    # 8 x 8 map; the boresight walks along x on row 3.2; detectors 1 px up / 2 px right
    bore = _bore([3.2, 3.2, 3.2, 3.2], [0.0, 1.4, 1.6, 7.4], 0.0)
    det = _dets([0.0, 1.0], [0.0, 2.0], [0.0, 0.3])
    pix, c2, s2 = expand_pointing(bore, det, 8, 8)
    # detector 0: rows round(3.2) = 3, columns 0, 1, 2, 7
    assert pix[0].tolist() == [24, 25, 26, 31]
    # detector 1: row round(4.2) = 4, columns round(x + 2) = 2, 3, 4, and 9.4 is off the map
    assert pix[1].tolist() == [34, 35, 36, -1]
    np.testing.assert_allclose(c2[1], math.cos(0.6), rtol=0, atol=1e-15)
    np.testing.assert_allclose(s2[1], math.sin(0.6), rtol=0, atol=1e-15)


def test_quarter_turn_about_the_centre():
    # boresight on the centre (3.5, 3.5); a detector 2 px along +x before the turn
    # lands 2 px along +y after a +90 degree turn: (5.5, 3.5) -> pixel (6, 4)
    bore = _bore([3.5], [3.5], math.pi / 2)
    det = _dets([0.0, 1.0], [2.0, 0.0], [0.0, 0.0])
    pix, c2, s2 = expand_pointing(bore, det, 8, 8)
    assert pix[0, 0] == 6 * 8 + 4
    # 1 px along +y turns to -x: (3.5, 2.5) -> pixel (4, 3)
    assert pix[1, 0] == 4 * 8 + 3
    # psi = 0 turned by 90 degrees: cos 180 = -1, sin 180 = 0
    assert abs(c2[0, 0] + 1.0) < 1e-15 and abs(s2[0, 0]) < 1e-15


def test_pixel_edges():
    # floor(y + 1/2): -0.5 is the lower edge of pixel 0; ny - 0.5 is off the map
    bore = _bore([-0.5, -0.5000001, 7.4999999, 7.5], [0.0, 0.0, 0.0, 0.0], 0.0)
    pix, _, _ = expand_pointing(bore, _dets([0.0], [0.0], [0.0]), 8, 8)
    assert pix[0].tolist() == [0, -1, 56, -1]


def test_weights_are_the_angle_sum(rng):
    phi = rng.uniform(-0.3, 0.3, 50)
    psi = rng.uniform(0, math.pi, 7)
    bore = _bore(np.full(50, 2.0), np.full(50, 2.0), phi)
    _, c2, s2 = expand_pointing(bore, _dets(np.zeros(7), np.zeros(7), psi), 4, 4)
    ang = 2 * (psi[:, None] + phi[None, :])
    np.testing.assert_allclose(c2, np.cos(ang), rtol=0, atol=2e-15)
    np.testing.assert_allclose(s2, np.sin(ang), rtol=0, atol=2e-15)


@pytest.mark.parametrize("layout", ["hex", "line"])
def test_matches_the_generators_pointing(layout):
    inp = small_raster(ncomp=3, ny=32, nx=32, ndet=9, layout=layout, diameter=12.0,
                       drift_deg=15.0)
    pix, c2, s2 = expand_pointing(inp.bore, inp.det_off, inp.ny, inp.nx)
    assert np.array_equal(pix, inp.pix)
    assert (pix >= 0).sum() > 0.5 * pix.size and (pix < 0).any()
    # the stored weights are the float32 roundings of cos/sin 2(psi + phi)
    for w64, w32 in ((c2, inp.cos2psi), (s2, inp.sin2psi)):
        assert np.max(np.abs(w64 - w32.astype(np.float64))) <= 2.0**-24 + 1e-15


def test_oracle_scan_from_the_boresight(rng):
    inp = small_raster(ncomp=3, ny=16, nx=16, ndet=5, diameter=6.0)
    a, b = oracle.OracleScan(inp), oracle.OracleScan(boresight_only(inp))
    assert np.array_equal(a.pix, b.pix)
    np.testing.assert_array_equal(oracle.hits(a), oracle.hits(b))
    Ba = oracle.binned_blocks(a, oracle.detector_weights(a))
    mask = oracle.active_mask(a, Ba)
    x = rng.standard_normal(3 * 256) * np.tile(mask, 3)
    ya, yb = oracle.apply_A(a, x, mask), oracle.apply_A(b, x, mask)
    assert np.linalg.norm(ya - yb) <= 1e-6 * np.linalg.norm(ya)
