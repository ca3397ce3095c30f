"""Pins of the circulant preconditioner's eigenvalue floor.

The Implementation section needs Q invertible; the reading taken here raises
every eigenvalue of Q below eps * (the largest eigenvalue of Q) to that floor
before inverting.  Q is block circulant, so its eigenvalues are those of the
per-wavenumber blocks K(k), and the largest one is the maximum over ALL
wavenumbers.  The pin writes Q out as a dense (npix ncomp)^2 matrix (no
Fourier transforms), clamps the eigenvalues of that dense matrix directly and
inverts it; the oracle must agree in the floored count and in M_C r.

Every case here has an active floor: either the untapered circulant of a
strongly 1/f scan (negative eigenvalues at the default eps) or an eps chosen
between two of the dense eigenvalues so that a known number are raised.
Planted mistakes (the floor relative to each wavenumber's own largest
eigenvalue; the diagonal of K clamped instead of its eigenvalues; an absolute
floor; |lambda| instead of a floor) must each fail a pin.
"""

import numpy as np
import pytest

import oracle
from conftest import small_raster


def _setup(inp):
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B, 1e-3)
    return sc, B, mask


def _dense_Q(M):
    """Q[(i, a), (j, b)] = q_ab(j - i) on the periodic map (eq. 9-10)."""
    nc, ny, nx, npix = M.nc, M.ny, M.nx, M.npix
    iy, ix = np.divmod(np.arange(npix), nx)
    dy = (iy[None, :] - iy[:, None]) % ny
    dx = (ix[None, :] - ix[:, None]) % nx
    Q = M.q[dy, dx]                                   # (i, j, a, b)
    return np.transpose(Q, (0, 2, 1, 3)).reshape(npix * nc, npix * nc)


def _dense_clamped(M, eps):
    """(floored count, dense M_C) from the eigenvalues of the dense Q."""
    Q = _dense_Q(M)
    assert np.allclose(Q, Q.T, atol=1e-13 * np.abs(Q).max())
    lam, V = np.linalg.eigh(Q)
    floor = eps * lam.max()
    n = int(np.count_nonzero(lam < floor))
    Qi = (V / np.maximum(lam, floor)) @ V.T
    nc, npix = M.nc, M.npix
    # Sigma^-1 and Sigma^-T as block-diagonal matrices in (pixel, component) order
    S = np.zeros((npix * nc, npix * nc))
    for p in range(npix):
        S[p * nc:(p + 1) * nc, p * nc:(p + 1) * nc] = M.Siginv[p]
    Md = S @ Qi @ S.T
    act = np.repeat(M.mask, nc)
    Md[~act] = 0.0
    Md[:, ~act] = 0.0
    return n, Md, lam


def _apply_dense(Md, r, nc, npix):
    rp = r.reshape(nc, npix).T.reshape(-1)            # (p, a) order
    return (Md @ rp).reshape(npix, nc).T.reshape(-1)


def _pin(M, eps, rng, nrand=3):
    """(count agrees, largest relative error of M r over random r)."""
    n, Md, _ = _dense_clamped(M, eps)
    err = 0.0
    for _ in range(nrand):
        r = rng.standard_normal(M.nc * M.npix) * np.tile(M.mask, M.nc)
        want = _apply_dense(Md, r, M.nc, M.npix)
        got = M(r)
        err = max(err, np.abs(got - want).max() / np.abs(want).max())
    return n == M.n_floored, err, n


def _gap_eps(M, frac):
    """An eps that floors about `frac` of the dense eigenvalues, half way
    between two distinct consecutive ones (so rounding cannot move the count)."""
    lam = np.sort(np.linalg.eigvalsh(_dense_Q(M)))
    lmax = lam[-1]
    i = int(frac * lam.size)
    while lam[i + 1] - lam[i] < 1e-6 * lmax:
        i += 1
    return 0.5 * (lam[i] + lam[i + 1]) / lmax, i + 1


STRONG_1F = dict(ny=8, nx=8, ndet=5, fknee=(3.0, 5.0))


@pytest.mark.parametrize("ncomp", [1, 3])
def test_floor_active_untapered_matches_dense_clamp(ncomp, rng):
    # untapered q of a strongly 1/f scan has negative eigenvalues: the default
    # floor (1e-6 of the largest) must raise exactly those of the dense Q.
    sc, B, mask = _setup(small_raster(ncomp=ncomp, **STRONG_1F))
    M = oracle.CirculantPrecon(sc, mask, B, sigma_taper=None)
    ok, err, n = _pin(M, 1e-6, rng)
    assert n > 0 and M.n_floored > 0
    assert ok, (n, M.n_floored)
    assert err <= 1e-9, err


@pytest.mark.parametrize("ncomp,frac", [(1, 0.3), (3, 0.2), (3, 0.6)])
def test_floor_at_chosen_eps_matches_dense_clamp(ncomp, frac, rng):
    sc, B, mask = _setup(small_raster(ncomp=ncomp, ny=8, nx=8, ndet=5))
    M0 = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0)
    eps, nwant = _gap_eps(M0, frac)
    M = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0, eig_floor_rel=eps)
    assert M.n_floored == nwant > 0
    ok, err, n = _pin(M, eps, rng)
    assert ok, (n, M.n_floored)
    assert err <= 1e-9, err


def test_floor_relative_to_scale(rng):
    # scaling N^-1 by c scales A, q and K by c: a relative floor raises the same
    # eigenvalues and M_C scales by exactly 1/c.
    inp = small_raster(ncomp=3, **STRONG_1F)
    sc, B, mask = _setup(inp)
    M1 = oracle.CirculantPrecon(sc, mask, B, eig_floor_rel=1e-3)
    import dataclasses
    c = 32.0   # a power of two: the float32 spectrum scales exactly
    inp2 = dataclasses.replace(inp, inv_noise=(inp.inv_noise * c).astype(inp.inv_noise.dtype))
    sc2, B2, mask2 = _setup(inp2)
    assert np.array_equal(mask, mask2)
    M2 = oracle.CirculantPrecon(sc2, mask2, B2, eig_floor_rel=1e-3)
    assert M1.n_floored == M2.n_floored > 0
    r = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    # B scales by c too, so Sigma^-1 by c^-1/2 and q is scale-free: M_C scales by 1/c
    np.testing.assert_allclose(M2(r) * c, M1(r), rtol=1e-9, atol=1e-9 * np.abs(M1(r)).max())


# --------------------------------------------------------- planted mistakes

class _PerKMax(oracle.CirculantPrecon):
    @staticmethod
    def floored_inverse(K, eps):
        lam, V = np.linalg.eigh(K)
        floor = eps * lam.max(axis=-1, keepdims=True)
        n = int(np.count_nonzero(lam < floor))
        lam = np.maximum(lam, floor)
        return np.einsum("...ij,...j,...kj->...ik", V, 1.0 / lam, np.conj(V)), lam, n


class _ClampDiag(oracle.CirculantPrecon):
    @staticmethod
    def floored_inverse(K, eps):
        lam = np.linalg.eigvalsh(K)
        floor = eps * lam.max()
        Kc = K.copy()
        d = np.real(np.diagonal(K, axis1=-2, axis2=-1))
        n = int(np.count_nonzero(d < floor))
        idx = np.arange(K.shape[-1])
        Kc[..., idx, idx] = np.maximum(d, floor)
        return np.linalg.inv(Kc), None, n


class _AbsoluteFloor(oracle.CirculantPrecon):
    @staticmethod
    def floored_inverse(K, eps):
        lam, V = np.linalg.eigh(K)
        n = int(np.count_nonzero(lam < eps))
        lam = np.maximum(lam, eps)
        return np.einsum("...ij,...j,...kj->...ik", V, 1.0 / lam, np.conj(V)), lam, n


class _AbsEig(oracle.CirculantPrecon):
    @staticmethod
    def floored_inverse(K, eps):
        lam, V = np.linalg.eigh(K)
        floor = eps * lam.max()
        n = int(np.count_nonzero(lam < floor))
        lam = np.maximum(np.abs(lam), floor)
        return np.einsum("...ij,...j,...kj->...ik", V, 1.0 / lam, np.conj(V)), lam, n


def _fails_some_pin(cls, rng):
    """True if the class fails the dense-clamp pin on one of the floor cases or
    the scale pin."""
    inp = small_raster(ncomp=3, **STRONG_1F)
    sc, B, mask = _setup(inp)
    M = cls(sc, mask, B, sigma_taper=None)
    ok, err, _ = _pin(M, 1e-6, rng, nrand=1)
    if not ok or err > 1e-9:
        return True
    inp3 = small_raster(ncomp=3, ny=8, nx=8, ndet=5)
    sc3, B3, mask3 = _setup(inp3)
    eps, _ = _gap_eps(oracle.CirculantPrecon(sc3, mask3, B3, sigma_taper=3.0), 0.4)
    M3 = cls(sc3, mask3, B3, sigma_taper=3.0, eig_floor_rel=eps)
    ok, err, _ = _pin(M3, eps, rng, nrand=1)
    if not ok or err > 1e-9:
        return True
    import dataclasses
    c = 2.0 ** 13
    inp4 = dataclasses.replace(inp3, inv_noise=(inp3.inv_noise * c).astype(inp3.inv_noise.dtype))
    sc4, B4, mask4 = _setup(inp4)
    M4 = cls(sc4, mask4, B4, sigma_taper=3.0, eig_floor_rel=eps)
    ok, err, _ = _pin(M4, eps, rng, nrand=1)
    return not ok or err > 1e-9


@pytest.mark.parametrize("cls", [_PerKMax, _ClampDiag, _AbsoluteFloor, _AbsEig],
                         ids=["per-k-max", "clamp-diag", "absolute", "abs-eig"])
def test_planted_floor_mistakes_fail_a_pin(cls, rng):
    assert _fails_some_pin(cls, rng)


def test_the_oracle_itself_passes_the_mutation_harness(rng):
    assert not _fails_some_pin(oracle.CirculantPrecon, rng)
