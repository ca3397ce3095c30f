"""Pins of the oracle's tiled constant-correlation preconditioner: one tile
the size of the map is exactly M_C, the merge weights are a partition of
unity, white noise makes it exactly the binned preconditioner, and it is
symmetric positive definite with real tiles."""

import numpy as np
import pytest

import oracle
from oracle.tiled import TiledCirculantPrecon, axis_weights
from conftest import small_raster


def _setup(ny=16, nx=16, white=False, ndet=5):
    inp = small_raster(ncomp=3, ny=ny, nx=nx, ndet=ndet, white=white, diameter=4.0)
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    return sc, B, oracle.active_mask(sc, B)


@pytest.mark.parametrize("n,T", [(16, 16), (16, 8), (32, 8), (32, 4), (64, 16)])
def test_weights_are_a_partition_of_unity(n, T):
    orig, w = axis_weights(n, T)
    tot = np.zeros(n)
    for o, wt in zip(orig, w):
        tot[o:o + T] += wt
    np.testing.assert_allclose(tot, 1.0, rtol=0, atol=1e-14)


def test_one_tile_is_the_circulant_preconditioner(rng):
    sc, B, mask = _setup()
    Mc = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0)
    Mt = TiledCirculantPrecon(sc, mask, B, tile=16, sigma_taper=3.0)
    assert len(Mt.tiles) == 1 and Mt.tiles[0]["ref"] == Mc.ref
    r = rng.standard_normal(3 * sc.npix) * np.tile(mask, 3)
    np.testing.assert_allclose(Mt(r), Mc(r), rtol=1e-12, atol=1e-12 * np.abs(Mc(r)).max())


def test_white_noise_gives_the_binned_preconditioner(rng):
    sc, B, mask = _setup(white=True)
    Mt = TiledCirculantPrecon(sc, mask, B, tile=8, sigma_taper=2.0)
    Mb = oracle.BinnedPrecon(B, mask)
    r = rng.standard_normal(3 * sc.npix) * np.tile(mask, 3)
    np.testing.assert_allclose(Mt(r), Mb(r), rtol=1e-10, atol=1e-12)


def test_symmetric_positive_definite(rng):
    sc, B, mask = _setup(ny=32, nx=32, ndet=6)
    Mt = TiledCirculantPrecon(sc, mask, B, tile=16, sigma_taper=3.0)
    assert len(Mt.tiles) == 9
    m3 = np.tile(mask, 3)
    x, y = rng.standard_normal(3 * sc.npix) * m3, rng.standard_normal(3 * sc.npix) * m3
    a, b = x @ Mt(y), y @ Mt(x)
    assert abs(a - b) <= 1e-11 * (abs(a) + abs(b))
    assert x @ Mt(x) > 0
    # it differs from the single circulant (the tiles see different columns)
    Mc = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0)
    assert np.linalg.norm(Mt(x) - Mc(x)) > 1e-3 * np.linalg.norm(Mc(x))


def test_tile_kernels_are_rows_of_A_at_each_tiles_reference(rng):
    # Each tile's q_t(d) is Sigma_r^-T A_(r, r+d) Sigma_(r+d)^-1 at that tile's
    # OWN reference pixel r (eq. 6, eq. 10 per tile), read off the dense A:
    # a probe shared between tiles would add the other references' rows.
    sc, B, mask = _setup(ny=16, nx=16, ndet=5)
    Mt = TiledCirculantPrecon(sc, mask, B, tile=8, sigma_taper=None)
    assert len(Mt.tiles) == 9
    n = 3 * sc.npix
    A = lambda v: oracle.apply_A(sc, v, mask)  # noqa: E731
    Ad = oracle.dense_operator(A, n).reshape(3, sc.npix, 3, sc.npix)
    d = np.arange(8)
    dmi = np.where(d > 4, d - 8, d)
    for t in Mt.tiles:
        r = t["ref"]
        assert r >= 0
        ry, rx = divmod(r, 16)
        for iy in range(8):
            for ix in range(8):
                jy, jx = (ry + dmi[iy]) % 16, (rx + dmi[ix]) % 16
                j = jy * 16 + jx
                want = Mt.Siginv[r].T @ Ad[:, r, :, j] @ Mt.Siginv[j] if mask[j] else 0.0
                np.testing.assert_allclose(t["q_raw"][iy, ix], want, rtol=1e-10,
                                           atol=1e-12 * np.abs(t["q_raw"]).max())


def test_tile_floor_is_relative_to_the_tile(rng):
    # an eps that floors part of one tile's spectrum floors the count the
    # tile's own eigenvalues give (the floor of M_C applied to Q_t)
    sc, B, mask = _setup(ny=16, nx=16, ndet=5)
    M0 = TiledCirculantPrecon(sc, mask, B, tile=8, sigma_taper=2.0)
    M1 = TiledCirculantPrecon(sc, mask, B, tile=8, sigma_taper=2.0, eig_floor_rel=0.45)
    for t0, t1 in zip(M0.tiles, M1.tiles):
        K = np.conj(np.fft.fft2(t0["q"], axes=(0, 1)))
        lam = np.linalg.eigvalsh(K)
        assert t1["n_floored"] == np.count_nonzero(lam < 0.45 * lam.max())
    assert sum(t["n_floored"] for t in M1.tiles) > 0
