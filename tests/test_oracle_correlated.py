"""Pins of the oracle's inter-detector correlated inverse noise: it reduces to
the independent filter when V = 0, it equals an explicitly built dense
time-domain N^-1 (a block circulant from the per-frequency matrices), A stays
symmetric positive definite, the detector weights are that matrix's
diagonal, and the generated noise model is positive definite."""

import dataclasses

import numpy as np

import oracle
from conftest import small_raster
from synth import correlated_inverse_noise, with_correlated_noise


def _tiny(ndet=3, rank=2):
    inp = small_raster(ncomp=3, ny=4, nx=4, ndet=ndet, sweeps=1)   # 16 samples
    return with_correlated_noise(inp, rank=rank, nbins=4, seed=(1, 2))


def _dense_ninv(scan):
    """(ndet*n) x (ndet*n) matrix of N^-1 from its definition: block (d, d')
    is the circulant whose eigenvalue at two-sided frequency k is
    N^-1_{dd'}(min(k, n-k))."""
    n, nd = scan.nsamp, scan.ndet
    edges, V = scan.corr
    nk = n // 2 + 1
    Nk = np.zeros((nk, nd, nd))
    for b in range(len(edges) - 1):
        for k in range(edges[b], edges[b + 1]):
            Nk[k] = np.diag(scan.iN[:, k]) - V[b] @ V[b].T
    t = np.arange(n)
    D = np.zeros((nd * n, nd * n))
    for k in range(n):
        kk = k if k < nk else n - k
        ph = np.cos(2 * np.pi * k * (t[:, None] - t[None, :]) / n) / n
        for d in range(nd):
            for e in range(nd):
                D[d * n:(d + 1) * n, e * n:(e + 1) * n] += Nk[kk][d, e] * ph
    return D


def test_zero_correlation_is_the_independent_filter(rng):
    inp = _tiny()
    z = dataclasses.replace(inp, corr_V=np.zeros_like(inp.corr_V))
    a, b = oracle.OracleScan(z), oracle.OracleScan(dataclasses.replace(inp, corr_edges=None,
                                                                        corr_V=None))
    tod = rng.standard_normal((inp.ndet, inp.nsamp))
    np.testing.assert_allclose(oracle.inv_noise(a, tod), oracle.inv_noise(b, tod), atol=1e-13)
    np.testing.assert_allclose(oracle.detector_weights(a), oracle.detector_weights(b), rtol=1e-14)


def test_matches_dense_block_circulant(rng):
    sc = oracle.OracleScan(_tiny())
    tod = rng.standard_normal((sc.ndet, sc.nsamp))
    D = _dense_ninv(sc)
    np.testing.assert_allclose(oracle.inv_noise(sc, tod).ravel(), D @ tod.ravel(),
                               rtol=1e-11, atol=1e-11)
    # the detector weights are the time-domain diagonal
    np.testing.assert_allclose(oracle.detector_weights(sc),
                               np.diag(D).reshape(sc.ndet, sc.nsamp)[:, 0], rtol=1e-12)
    assert np.allclose(D, D.T, atol=1e-12)


def test_A_symmetric_positive_with_correlations(rng):
    inp = with_correlated_noise(small_raster(ncomp=3, ny=8, nx=8, ndet=5),
                                rank=3, nbins=8, seed=(3, 4))
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B)
    x = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    y = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    a, b = x @ oracle.apply_A(sc, y, mask), y @ oracle.apply_A(sc, x, mask)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert x @ oracle.apply_A(sc, x, mask) > 0
    # the correlation changes A
    ind = oracle.OracleScan(dataclasses.replace(inp, corr_edges=None, corr_V=None))
    assert np.linalg.norm(oracle.apply_A(sc, x, mask) - oracle.apply_A(ind, x, mask)) > \
        1e-3 * np.linalg.norm(oracle.apply_A(ind, x, mask))


def test_generated_model_is_positive_definite(rng):
    ndet, nk = 6, 129
    iN = rng.uniform(0.5, 2.0, (ndet, nk)).astype(np.float32)
    edges, V = correlated_inverse_noise(iN, 100.0, rank=3, nbins=10, beta_max=0.9, seed=(5, 6))
    assert edges[0] == 0 and edges[-1] == nk and np.all(np.diff(edges) > 0)
    for b in range(len(edges) - 1):
        for k in range(edges[b], edges[b + 1]):
            M = np.diag(iN[:, k].astype(np.float64)) - V[b].astype(np.float64) @ V[b].T
            assert np.linalg.eigvalsh(M)[0] >= 0.099 * iN[:, k].min()
