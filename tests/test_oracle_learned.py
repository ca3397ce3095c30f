"""Pins of the oracle's learned correction: convolutions against per-tap loops,
exact adjoints, symmetry/PSD of H^T H and of M_L - M_C, analytic gradients
against central finite differences, and the first Adam step's closed form."""

import numpy as np
import pytest

import oracle
from oracle import learned as L
from conftest import small_raster


def test_conv_same_matches_loops(rng):
    x = rng.standard_normal((3, 6, 7))
    W = rng.standard_normal((4, 3, 5, 5))
    y = L.conv_same(x, W)
    ref = np.zeros((4, 6, 7))
    for o in range(4):
        for i in range(6):
            for j in range(7):
                s = 0.0
                for c in range(3):
                    for u in range(5):
                        for v in range(5):
                            ii, jj = i + u - 2, j + v - 2
                            if 0 <= ii < 6 and 0 <= jj < 7:
                                s += W[o, c, u, v] * x[c, ii, jj]
                ref[o, i, j] = s
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def test_transpose_is_adjoint(rng):
    x = rng.standard_normal((2, 3, 9, 8))
    z = rng.standard_normal((2, 16, 9, 8))
    W = rng.standard_normal((16, 3, 5, 5))
    lhs = np.sum(L.conv_same(x, W) * z)
    rhs = np.sum(x * L.conv_same_T(z, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_HtH_symmetric_psd(rng):
    W1, W2 = L.init_weights(rng)
    W1 *= 30
    W2 *= 30
    x = rng.standard_normal((1, 3, 10, 12))
    y = rng.standard_normal((1, 3, 10, 12))
    a, b = np.sum(x * L.HtH(y, W1, W2)), np.sum(y * L.HtH(x, W1, W2))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    Hx = L.conv_same(L.conv_same(x, W1), W2)
    np.testing.assert_allclose(np.sum(x * L.HtH(x, W1, W2)), np.sum(Hx * Hx), rtol=1e-12)


def _circ():
    inp = small_raster(ncomp=3, ny=8, nx=8, ndet=5)
    sc = oracle.OracleScan(inp)
    B = oracle.binned_blocks(sc, oracle.detector_weights(sc))
    mask = oracle.active_mask(sc, B)
    return sc, mask, oracle.CirculantPrecon(sc, mask, B, sigma_taper=3.0)


def test_learned_zero_is_circulant_and_correction_is_psd(rng):
    sc, mask, Mc = _circ()
    r = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    Z1, Z2 = np.zeros((16, 3, 5, 5)), np.zeros((16, 16, 5, 5))
    np.testing.assert_array_equal(L.LearnedPrecon(Mc, Z1, Z2)(r), Mc(r))
    W1, W2 = L.init_weights(rng)
    Ml = L.LearnedPrecon(Mc, 20 * W1, 20 * W2)
    s = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    a, b = s @ Ml(r), r @ Ml(s)
    assert abs(a - b) <= 1e-11 * (abs(a) + abs(b))
    assert r @ (Ml(r) - Mc(r)) >= -1e-14 * abs(r @ Mc(r))


def test_gradient_matches_finite_differences(rng):
    P, H, W = 2, 7, 6
    R = rng.standard_normal((P, 3, H, W))
    T = rng.standard_normal((P, 3, H, W))
    E2 = rng.uniform(0.5, 2.0, P)
    W1, W2 = L.init_weights(rng)
    W1 *= 10
    W2 *= 10
    _, g1, g2 = L.loss_and_grad(R, T, E2, W1, W2)
    h = 1e-6
    for W, g, name in ((W1, g1, "W1"), (W2, g2, "W2")):
        idx = [tuple(rng.integers(0, s) for s in W.shape) for _ in range(12)]
        for ix in idx:
            Wp, Wm = W.copy(), W.copy()
            Wp[ix] += h
            Wm[ix] -= h
            args_p = (Wp, W2) if name == "W1" else (W1, Wp)
            args_m = (Wm, W2) if name == "W1" else (W1, Wm)
            fd = (L.loss_and_grad(R, T, E2, *args_p)[0] - L.loss_and_grad(R, T, E2, *args_m)[0]) / (2 * h)
            assert abs(fd - g[ix]) <= 1e-6 * max(1.0, abs(g).max()), (name, ix, fd, g[ix])


def test_first_adam_step_closed_form(rng):
    W = rng.standard_normal((4, 3, 5, 5))
    g = rng.standard_normal(W.shape)
    W1, m, v = L.adam_step(W, g, np.zeros_like(W), np.zeros_like(W), t=1, lr=1e-3)
    # bias-corrected first step: m^ = g, v^ = g^2, so W - lr g / (|g| + eps)
    np.testing.assert_allclose(W1, W - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_pair_identity(rng):
    # with the exact error in the pair, Sigma M_L r = e_w iff H^T H r_w = t
    sc, mask, Mc = _circ()
    A = lambda v: oracle.apply_A(sc, v, mask)  # noqa: E731
    x_f = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    x_k = rng.standard_normal(3 * 64) * np.tile(mask, 3)
    r_w, t, e2 = L.make_pair(A, Mc, x_f, x_k)
    e_w = L.sigma_apply(Mc, x_f - x_k)
    r = A(x_f - x_k)
    np.testing.assert_allclose(L.sigma_apply(Mc, Mc(r)) + t, e_w, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(e2, np.sum(e_w**2))
    np.testing.assert_allclose(L.unwhiten(Mc, L.sigma_apply(Mc, x_f - x_k)), x_f - x_k,
                               rtol=1e-10, atol=1e-12)
