"""Pins of the oracle's P, P^T, N^-1, A and b against brute force, closed forms
and the invariants eq. 1-2 imply."""

import numpy as np
import pytest

import oracle
from conftest import small_raster


def _brute_P(inp, m):
    ndet, n = inp.pix.shape
    out = np.zeros((ndet, n))
    for d in range(ndet):
        for s in range(n):
            p = int(inp.pix[d, s])
            if p < 0:
                continue
            v = m[0][p]
            if inp.ncomp == 3:
                v += float(inp.cos2psi[d, s]) * m[1][p] + float(inp.sin2psi[d, s]) * m[2][p]
            out[d, s] = v
    return out


def _brute_PT(inp, tod):
    out = np.zeros((inp.ncomp, inp.ny * inp.nx))
    ndet, n = inp.pix.shape
    for d in range(ndet):
        for s in range(n):
            p = int(inp.pix[d, s])
            if p < 0:
                continue
            out[0][p] += tod[d, s]
            if inp.ncomp == 3:
                out[1][p] += float(inp.cos2psi[d, s]) * tod[d, s]
                out[2][p] += float(inp.sin2psi[d, s]) * tod[d, s]
    return out


@pytest.mark.parametrize("ncomp", [1, 3])
def test_pointing_matches_per_sample_loops(ncomp, rng):
    inp = small_raster(ncomp=ncomp, ny=4, nx=4, ndet=3, diameter=2.0)
    sc = oracle.OracleScan(inp)
    assert (inp.pix < 0).any() and (inp.pix >= 0).any()
    m = rng.standard_normal((ncomp, 16))
    v = rng.standard_normal(inp.pix.shape)
    np.testing.assert_allclose(oracle.pointing(sc, m), _brute_P(inp, m), rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.pointing_T(sc, v), _brute_PT(inp, v), rtol=0, atol=1e-12)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_pointing_adjoint(ncomp, rng):
    inp = small_raster(ncomp=ncomp, ny=16, nx=16, ndet=6)
    sc = oracle.OracleScan(inp)
    m = rng.standard_normal((ncomp, 256))
    v = rng.standard_normal(inp.pix.shape)
    lhs = np.sum(oracle.pointing(sc, m) * v)
    rhs = np.sum(m * oracle.pointing_T(sc, v))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(m) * np.linalg.norm(v))


def test_PT_of_ones_is_hit_map():
    inp = small_raster(ncomp=1, ny=16, nx=16, ndet=5)
    sc = oracle.OracleScan(inp)
    counts = np.zeros(256)
    for p in inp.pix.ravel():
        if p >= 0:
            counts[p] += 1
    np.testing.assert_array_equal(oracle.pointing_T(sc, np.ones(inp.pix.shape))[0], counts)
    np.testing.assert_array_equal(oracle.hits(sc), counts)


@pytest.mark.parametrize("n", [64, 60, 90])
def test_inv_noise_matches_dense_dft_circulant(n, rng):
    # N^-1 = F^-1 diag(iN_two_sided) F with F_fj = exp(-2 pi i j f / n), built
    # from explicit DFT matrices (the Fourier convention of eq. 11); also at
    # lengths that are not powers of two (n/2 = 30 and the odd 45)
    from synth import raster_scan
    inp = raster_scan(ncomp=1, ny=4, nx=4, ndet=2, nsamp=n, fsample=100.0, layout="hex",
                      hex_diameter_px=3.0, fknee=(1.0, 2.0), seed=(99, n))
    sc = oracle.OracleScan(inp)
    assert sc.nsamp == n
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    Finv = np.exp(2j * np.pi * np.outer(j, j) / n) / n
    v = rng.standard_normal((2, n))
    got = oracle.inv_noise(sc, v)
    for d in range(2):
        half = sc.iN[d]
        full = np.concatenate([half, half[1:n // 2][::-1]])
        Ninv = (Finv @ np.diag(full) @ F)
        assert np.abs(Ninv.imag).max() < 1e-12
        np.testing.assert_allclose(got[d], Ninv.real @ v[d], rtol=0, atol=1e-12)


def test_inv_noise_pure_tone_and_white(rng):
    inp = small_raster(ncomp=1, ny=8, nx=8, ndet=3)
    sc = oracle.OracleScan(inp)
    n = sc.nsamp
    t = np.arange(n)
    for k in (0, 1, 5, n // 2):
        tone = np.cos(2 * np.pi * k * t / n)
        out = oracle.inv_noise(sc, np.repeat(tone[None], 3, axis=0))
        for d in range(3):
            np.testing.assert_allclose(out[d], sc.iN[d, k] * tone, rtol=0, atol=1e-12)
    w = small_raster(ncomp=1, ny=8, nx=8, ndet=3, white=True)
    sw = oracle.OracleScan(w)
    v = rng.standard_normal((3, n))
    sig = w.meta["sigma"]
    expect = v / (sig.astype(np.float32).astype(np.float64)[:, None] ** 2)
    np.testing.assert_allclose(oracle.inv_noise(sw, v), v * sw.iN[:, :1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.inv_noise(sw, v), expect, rtol=1e-6)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_A_symmetric_positive(ncomp, rng):
    inp = small_raster(ncomp=ncomp, ny=16, nx=16, ndet=6)
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B)
    x = rng.standard_normal(ncomp * 256) * np.tile(mask, ncomp)
    y = rng.standard_normal(ncomp * 256) * np.tile(mask, ncomp)
    Ax, Ay = oracle.apply_A(sc, x, mask), oracle.apply_A(sc, y, mask)
    assert abs(x @ Ay - y @ Ax) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(Ay)
    assert x @ Ax > 0
    # inactive entries are zero on output
    assert np.all(Ax.reshape(ncomp, -1)[:, ~mask] == 0)


@pytest.mark.parametrize("n", [64, 90])
def test_detector_weight_is_diagonal_of_Ninv(n):
    from synth import raster_scan
    inp = raster_scan(ncomp=1, ny=4, nx=4, ndet=3, nsamp=n, fsample=100.0, layout="hex",
                      hex_diameter_px=3.0, fknee=(1.0, 2.0), seed=(98, n))
    sc = oracle.OracleScan(inp)
    e0 = np.zeros((3, n))
    e0[:, 7] = 1.0
    diag = oracle.inv_noise(sc, e0)[:, 7]
    np.testing.assert_allclose(oracle.detector_weights(sc), diag, rtol=1e-13)


def test_white_noise_binned_blocks_are_A_diagonal_blocks():
    # eq. 3-4 is exact when N is diagonal: A is then block-diagonal and its
    # pixel blocks are the binned blocks.
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=5, white=True)
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B)
    npix = 64
    Ad = oracle.dense_operator(lambda v: oracle.apply_A(sc, v, mask), 3 * npix)
    A4 = Ad.reshape(3, npix, 3, npix)
    for p in range(npix):
        if not mask[p]:
            continue
        np.testing.assert_allclose(A4[:, p, :, p], B[p], rtol=1e-12, atol=1e-12)
        off = A4[:, p, :, :].copy()
        off[:, :, p] = 0
        assert np.abs(off).max() < 1e-12 * np.abs(B[p]).max()


def test_binned_blocks_bruteforce():
    inp = small_raster(ncomp=3, ny=4, nx=4, ndet=3, diameter=2.0)
    sc = oracle.OracleScan(inp)
    wd = np.array([0.5, 1.5, 2.0])
    B = oracle.binned_blocks(sc, wd)
    ref = np.zeros((16, 3, 3))
    for d in range(3):
        for s in range(sc.nsamp):
            p = inp.pix[d, s]
            if p < 0:
                continue
            u = np.array([1.0, float(inp.cos2psi[d, s]), float(inp.sin2psi[d, s])])
            ref[p] += wd[d] * np.outer(u, u)
    np.testing.assert_allclose(B, ref, rtol=1e-13, atol=1e-13)


def test_rhs_is_A_of_signal_for_noiseless_tod(rng):
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B)
    m = rng.standard_normal((3, 64)) * mask
    d = oracle.pointing(sc, m)
    np.testing.assert_allclose(oracle.rhs(sc, d, mask), oracle.apply_A(sc, m, mask),
                               rtol=1e-12, atol=1e-12)
