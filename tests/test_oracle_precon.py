"""Pins of the oracle's preconditioners and PCG: exactness cases the paper's
construction implies, library PCG, dense solves and scale invariance."""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from conftest import small_raster
from synth import periodic_torus_scan, crosslinked_torus_scan


def _setup(inp, rcond=1e-3):
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B, rcond)
    A = lambda v: oracle.apply_A(sc, v, mask)  # noqa: E731
    return sc, B, mask, A


def _signal_rhs(sc, mask, A, rng):
    m = rng.standard_normal((sc.ncomp, sc.npix)) * mask
    return A(m.reshape(-1))


# ---------------------------------------------------------------- binned / Jacobi

@pytest.mark.parametrize("ncomp", [1, 3])
def test_binned_exact_for_white_noise(ncomp, rng):
    inp = small_raster(ncomp=ncomp, ny=8, nx=8, ndet=5, white=True)
    sc, B, mask, A = _setup(inp)
    M = oracle.BinnedPrecon(B, mask)
    b = _signal_rhs(sc, mask, A, rng)
    res = oracle.pcg(A, M, b, tol=1e-13, maxiter=50)
    assert res.converged and res.iters == 1, res.history


def test_jacobi_equals_binned_for_equal_weights_and_hits_for_I():
    inp = small_raster(ncomp=1, ny=8, nx=8, ndet=4, white=True, sigma_scatter=0.0)
    sc, B, mask, A = _setup(inp)
    J = oracle.binned_blocks(sc, np.ones(sc.ndet))
    np.testing.assert_array_equal(J[:, 0, 0], oracle.hits(sc))
    w = oracle.detector_weights(sc)
    assert np.allclose(w, w[0])
    Mb, Mj = oracle.BinnedPrecon(B, mask), oracle.BinnedPrecon(J, mask)
    r = np.random.default_rng(1).standard_normal(sc.npix)
    np.testing.assert_allclose(Mj(r) / w[0], Mb(r) * 1.0, rtol=1e-12)


# ---------------------------------------------------------------- circulant

def test_sym_sqrt_roots():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((10, 3, 3))
    B = X @ np.transpose(X, (0, 2, 1)) + 0.1 * np.eye(3)
    S, Si = oracle.sym_sqrt(B)
    np.testing.assert_allclose(S @ S, B, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(S, np.transpose(S, (0, 2, 1)), atol=1e-13)
    np.testing.assert_allclose(S @ Si, np.broadcast_to(np.eye(3), B.shape), atol=1e-12)


def test_reference_pixel_rule():
    ny, nx = 6, 8
    mask = np.ones(48, bool)
    assert oracle.reference_pixel(mask, ny, nx) == 3 * 8 + 4
    mask[3 * 8 + 4] = False
    # four pixels at distance 1; the smallest id is (2, 4)
    assert oracle.reference_pixel(mask, ny, nx) == 2 * 8 + 4
    mask[:] = False
    mask[0] = mask[47] = True
    # (0,0): d2 = 9+16 = 25 ; (5,7): d2 = 4+9 = 13
    assert oracle.reference_pixel(mask, ny, nx) == 47


def test_taper_minimal_image():
    g = oracle.gaussian_taper(8, 6, 2.0)
    assert g[0, 0] == 1.0
    np.testing.assert_allclose(g[1, 0], math.exp(-1 / 8))
    np.testing.assert_allclose(g[7, 0], g[1, 0])            # -1 wraps to 7
    np.testing.assert_allclose(g[4, 3], math.exp(-(16 + 9) / 8))
    assert np.all(oracle.gaussian_taper(8, 6, None) == 1.0)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_circulant_exact_on_coprime_torus(ncomp, rng):
    # PS-1: every translation of the 7x8 torus is a time shift, so A is exactly
    # (block) circulant and M_C = A^-1: PCG converges in one iteration.
    inp = periodic_torus_scan(ncomp, 7, 8, periods=6, fsample=50.0, fknee=3.0)
    sc, B, mask, A = _setup(inp)
    assert mask.all()
    M = oracle.CirculantPrecon(sc, mask, B)
    assert M.n_floored == 0
    b = _signal_rhs(sc, mask, A, rng)
    res = oracle.pcg(A, M, b, tol=1e-10, maxiter=20)
    assert res.converged and res.iters == 1, res.history
    # and the binned preconditioner is not exact here
    rb = oracle.pcg(A, oracle.BinnedPrecon(B, mask), b, tol=1e-10, maxiter=200)
    assert rb.iters > 3


@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("L", [8, 16])
def test_circulant_exact_on_crosslinked_torus(ncomp, L, rng):
    # PS-X: translations are detector permutations plus time shifts; the two
    # diagonal families give the X-shaped correlation of the paper's scans.
    inp = crosslinked_torus_scan(ncomp, L=L, periods=4, fknee=3.0)
    sc, B, mask, A = _setup(inp)
    assert mask.all()
    M = oracle.CirculantPrecon(sc, mask, B)
    b = _signal_rhs(sc, mask, A, rng)
    res = oracle.pcg(A, M, b, tol=1e-10, maxiter=20)
    assert res.converged and res.iters == 1, res.history
    # any reference pixel gives the same Q
    M2 = oracle.CirculantPrecon(sc, mask, B, ref=5 * L + 3)
    np.testing.assert_allclose(M2.q, M.q, rtol=1e-10, atol=1e-12 * np.abs(M.q).max())


@pytest.mark.parametrize("ncomp", [1, 3])
def test_circulant_white_noise_equals_binned(ncomp, rng):
    # white noise: q = delta * I, so M_C = Sigma^-1 Sigma^-T = M_B exactly.
    inp = small_raster(ncomp=ncomp, ny=8, nx=8, ndet=5, white=True)
    sc, B, mask, A = _setup(inp)
    Mc, Mb = oracle.CirculantPrecon(sc, mask, B), oracle.BinnedPrecon(B, mask)
    r = rng.standard_normal(ncomp * 64) * np.tile(mask, ncomp)
    np.testing.assert_allclose(Mc(r), Mb(r), rtol=1e-10, atol=1e-12 * np.abs(Mb(r)).max())


def test_circulant_narrow_taper_is_scaled_binned(rng):
    # sigma_taper -> 0 keeps only q(0) = A_rr / B_r: M_C = M_B / q(0), and
    # PCG is blind to the scale, so the iterates coincide.
    inp = small_raster(ncomp=1, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    Mc = oracle.CirculantPrecon(sc, mask, B, sigma_taper=1e-3)
    Mb = oracle.BinnedPrecon(B, mask)
    r = rng.standard_normal(64) * mask
    q0 = Mc.q[0, 0, 0, 0]
    np.testing.assert_allclose(Mc(r) * q0, Mb(r), rtol=1e-10, atol=1e-14)
    b = _signal_rhs(sc, mask, A, rng)
    ra = oracle.pcg(A, Mc, b, tol=1e-9, maxiter=40, keep_iterates=True)
    rb = oracle.pcg(A, Mb, b, tol=1e-9, maxiter=40, keep_iterates=True)
    assert ra.iters == rb.iters
    for xa, xb in zip(ra.iterates, rb.iterates):
        np.testing.assert_allclose(xa, xb, rtol=1e-8, atol=1e-10 * np.abs(xb).max())


@pytest.mark.parametrize("symmetrize", [True, False])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_circulant_matches_dense_block_circulant(ncomp, symmetrize, rng):
    # M_C = Sigma^-1 Q^-1 Sigma^-T with Q[(i,a),(j,b)] = q_ab(j - i) written out
    # as a dense matrix (eq. 9-12 with no Fourier transforms).
    inp = small_raster(ncomp=ncomp, ny=8, nx=8, ndet=5)
    sc, B, mask, A = _setup(inp)
    M = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0, symmetrize=symmetrize)
    assert M.n_floored == 0
    ny = nx = 8
    npix = 64
    nc = ncomp
    Q = np.zeros((npix, nc, npix, nc))
    for i in range(npix):
        iy, ix = divmod(i, nx)
        for j in range(npix):
            jy, jx = divmod(j, nx)
            Q[i, :, j, :] = M.q[(jy - iy) % ny, (jx - ix) % nx]
    Q = Q.reshape(npix * nc, npix * nc)
    if symmetrize:
        np.testing.assert_allclose(Q, Q.T, atol=1e-14 * np.abs(Q).max())
    r = rng.standard_normal(nc * npix) * np.tile(mask, nc)
    rp = r.reshape(nc, npix).T
    u = np.einsum("pba,pb->pa", M.Siginv, rp).reshape(-1)        # (p, a) order
    v = np.linalg.solve(Q, u).reshape(npix, nc)
    z = np.einsum("pab,pb->pa", M.Siginv, v)
    z[~mask] = 0
    np.testing.assert_allclose(M(r), z.T.reshape(-1), rtol=1e-9,
                               atol=1e-11 * np.abs(z).max())


def test_circulant_q_blocks_from_probe_match_dense_A(rng):
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=5)
    sc, B, mask, A = _setup(inp)
    M = oracle.CirculantPrecon(sc, mask, B, symmetrize=False)
    Ad = oracle.dense_operator(A, 3 * 64).reshape(3, 64, 3, 64)
    r = M.ref
    ry, rx = divmod(r, 8)
    for j in range(64):
        if not mask[j]:
            continue
        jy, jx = divmod(j, 8)
        blk = Ad[:, r, :, j]                   # A_{(r,a),(j,b)}
        expect = M.Siginv[r].T @ blk @ M.Siginv[j]
        np.testing.assert_allclose(M.q[(jy - ry) % 8, (jx - rx) % 8], expect,
                                   rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- PCG

def test_pcg_matches_scipy_cg_iterates(rng):
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    M = oracle.BinnedPrecon(B, mask)
    b = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    ours = oracle.pcg(A, M, b, tol=1e-30, maxiter=6, keep_iterates=True)
    n = b.size
    Aop = spla.LinearOperator((n, n), matvec=A)
    Mop = spla.LinearOperator((n, n), matvec=M)
    for k in range(1, 7):
        xs, _ = spla.cg(Aop, b, M=Mop, rtol=1e-30, atol=0.0, maxiter=k)
        np.testing.assert_allclose(ours.iterates[k - 1], xs, rtol=1e-9,
                                   atol=1e-11 * np.abs(xs).max())


def test_pcg_invariant_to_preconditioner_scale(rng):
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    M = oracle.BinnedPrecon(B, mask)
    b = _signal_rhs(sc, mask, A, rng)
    r1 = oracle.pcg(A, M, b, tol=1e-8, maxiter=200, keep_iterates=True)
    r2 = oracle.pcg(A, lambda v: 7.5 * M(v), b, tol=1e-8, maxiter=200, keep_iterates=True)
    assert r1.iters == r2.iters
    for a, c in zip(r1.iterates, r2.iterates):
        np.testing.assert_allclose(a, c, rtol=1e-9, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("ncomp", [1, 3])
def test_pcg_reaches_dense_solution(ncomp, rng):
    inp = small_raster(ncomp=ncomp, ny=8, nx=8, ndet=5, fknee=(0.3, 0.5))
    sc, B, mask, A = _setup(inp)
    idx = np.flatnonzero(np.tile(mask, ncomp))
    Ad = oracle.dense_operator(A, ncomp * 64, idx)
    np.testing.assert_allclose(Ad, Ad.T, rtol=1e-12, atol=1e-14 * np.abs(Ad).max())
    b = _signal_rhs(sc, mask, A, rng)
    xd = oracle.dense_solve(Ad, b[idx])
    for M in (oracle.BinnedPrecon(B, mask), oracle.CirculantPrecon(sc, mask, B, sigma_taper=4.0)):
        res = oracle.pcg(A, M, b, tol=1e-13, maxiter=2000)
        assert res.converged
        err = np.linalg.norm(res.x[idx] - xd) / np.linalg.norm(xd)
        assert err <= 1e-10, err


def test_pcg_finite_termination(rng):
    inp = small_raster(ncomp=1, ny=4, nx=4, ndet=3, fknee=(0.5, 0.5), diameter=1.5)
    sc, B, mask, A = _setup(inp)
    nact = int(mask.sum())
    b = _signal_rhs(sc, mask, A, rng)
    res = oracle.pcg(A, oracle.BinnedPrecon(B, mask), b, tol=0.0, maxiter=nact)
    assert res.history[-1] <= 1e-9, res.history


def test_pcg_breakdown_on_indefinite_preconditioner(rng):
    inp = small_raster(ncomp=1, ny=4, nx=4, ndet=3)
    sc, B, mask, A = _setup(inp)
    b = _signal_rhs(sc, mask, A, rng)
    res = oracle.pcg(A, lambda v: -v, b, tol=1e-8, maxiter=10)
    assert res.breakdown and not res.converged and res.iters == 0


def test_anorm_estimate_tracks_true_error(rng):
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    idx = np.flatnonzero(np.tile(mask, 3))
    Ad = oracle.dense_operator(A, 3 * 64, idx)
    b = _signal_rhs(sc, mask, A, rng)
    xd = oracle.dense_solve(Ad, b[idx])
    res = oracle.pcg(A, oracle.BinnedPrecon(B, mask), b, tol=1e-12, maxiter=300,
                     keep_iterates=True)
    est = oracle.anorm_estimate(res.alphas, res.rhos, d=4)
    # true ||x_k - x*||_A^2 for k = 1.. (iterate k-1 in the list is x_k)
    true = []
    for k in range(len(est)):
        xk = np.zeros(len(idx)) if k == 0 else res.iterates[k - 1][idx]
        e = xk - xd
        true.append(e @ Ad @ e)
    true = np.array(true)
    # a lower bound (sum of a subset of the positive terms of the exact
    # expansion, up to rounding) that tracks the truth within a modest factor
    assert np.all(est <= true * (1 + 1e-6) + 1e-12 * true[0])
    assert np.median(est / true) > 0.2


def test_flexible_beta_equals_standard_for_symmetric_M(rng):
    # with a symmetric M, r_{k+1}.M r_k = 0, so the Polak-Ribiere beta is the
    # standard one: the same iterates up to rounding
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    M = oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0)
    b = _signal_rhs(sc, mask, A, rng)
    r1 = oracle.pcg(A, M, b, tol=1e-9, maxiter=200, keep_iterates=True)
    r2 = oracle.pcg(A, M, b, tol=1e-9, maxiter=200, keep_iterates=True, flexible=True)
    assert r1.iters == r2.iters
    for a, c in zip(r1.iterates, r2.iterates):
        np.testing.assert_allclose(c, a, rtol=1e-7, atol=1e-9 * np.abs(a).max())


def test_flexible_beta_keeps_consecutive_directions_conjugate(rng):
    # for ANY M, beta = z'.(r' - r)/rho = -alpha z'.s/rho makes p_{k+1}.A p_k = 0;
    # the directions are the steps x_{k+1} - x_k.  The standard beta loses this
    # when M is not symmetric.
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=4)
    sc, B, mask, A = _setup(inp)
    Mb = oracle.BinnedPrecon(B, mask)
    n = 3 * 64
    G = np.random.default_rng(2).standard_normal((n, n)) * np.tile(mask, 3)[:, None]
    G *= np.tile(mask, 3)[None, :]
    Mns = lambda v: Mb(v) + 0.02 * Mb(G @ v)  # noqa: E731  (not symmetric)
    b = _signal_rhs(sc, mask, A, rng)

    def worst(res):
        xs = [np.zeros(n)] + res.iterates
        d = [xs[k + 1] - xs[k] for k in range(len(xs) - 1)]
        return max(abs(d[k + 1] @ A(d[k])) / np.sqrt((d[k + 1] @ A(d[k + 1])) * (d[k] @ A(d[k])))
                   for k in range(min(8, len(d) - 1)))

    rf = oracle.pcg(A, Mns, b, tol=1e-12, maxiter=12, keep_iterates=True, flexible=True)
    rs = oracle.pcg(A, Mns, b, tol=1e-12, maxiter=12, keep_iterates=True)
    assert worst(rf) <= 1e-10, worst(rf)
    assert worst(rs) > 1e-4, worst(rs)
