"""Per-detector stationary noise model: white + 1/f power spectrum.

S_d(f) = sigma_d^2 * (1 + (f / f_knee,d)^alpha), alpha = -3 by default, on the
frequencies f_k = k * fsample / n of an n-sample real FFT (k = 0 .. n/2).  The
DC bin, where S diverges, takes the value of the first non-zero bin.  The
inverse spectrum 1/S is what the noise-weighting step needs; it is rounded to
float32 here so that every consumer sees bit-identical values.
"""

import numpy as np


def noise_spectrum(nsamp, fsample, sigma, fknee, alpha=-3.0):
    """Power spectrum S[d, k] (float64) for detectors with the given parameters.

    sigma, fknee: arrays of shape (ndet,). Returns shape (ndet, nsamp//2 + 1).
    """
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    fknee = np.atleast_1d(np.asarray(fknee, dtype=np.float64))
    nk = nsamp // 2 + 1
    f = np.arange(nk, dtype=np.float64) * (fsample / nsamp)
    f[0] = f[1] if nk > 1 else 1.0
    S = sigma[:, None] ** 2 * (1.0 + (f[None, :] / fknee[:, None]) ** alpha)
    return S


def inverse_spectrum(S):
    """1/S rounded to float32 (the stored inverse-noise spectrum)."""
    return (1.0 / S).astype(np.float32)


def white_inverse_spectrum(nsamp, sigma):
    """Inverse spectrum of pure white noise: 1/sigma_d^2 at every frequency."""
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    nk = nsamp // 2 + 1
    return np.repeat((1.0 / sigma**2)[:, None], nk, axis=1).astype(np.float32)


def draw_noise(S_row, rng):
    """One noise realisation with circulant covariance of spectrum S_row.

    n = irfft(sqrt(S) * rfft(w)) with w ~ N(0, 1)^n, which has covariance
    exactly F^-1 diag(S) F.
    """
    nk = S_row.shape[-1]
    nsamp = 2 * (nk - 1)
    w = rng.standard_normal(nsamp)
    return np.fft.irfft(np.sqrt(S_row) * np.fft.rfft(w), nsamp)


def correlated_inverse_noise(iN, fsample, rank=2, nbins=16, beta_max=0.9, f_atm=1.0, seed=(0, 0)):
    """Inter-detector correlated part of an inverse noise model (an
    atmosphere-like common mode plus rank-1 more modes).  The real-FFT bins
    are grouped into about `nbins` log-spaced frequency bins
    (edges[b] <= k < edges[b+1]); in bin b the inverse noise matrix is
        N^-1(k) = diag(iN[:, k]) - V_b V_b^T,
        V_b = sqrt(beta_b) diag(sqrt(min_{k in b} iN[:, k])) G_b,
    with G_b of orthonormal columns (the first the common mode 1/sqrt(ndet),
    the rest seeded random directions orthogonalised against it) and
    beta_b = beta_max / (1 + (f_b / f_atm)^2) at the bin's centre frequency
    f_b, so the correlated part dominates low frequencies.  Since
    G_b G_b^T <= I, N^-1(k) >= (1 - beta_b) diag(iN[:, k]) stays positive
    definite.  Returns (edges int32 [nb + 1], V float32 [nb][ndet][rank])."""
    iN = np.asarray(iN, dtype=np.float64)
    ndet, nk = iN.shape
    nsamp = 2 * (nk - 1)
    inner = np.unique(np.round(np.geomspace(1, nk, nbins)).astype(np.int64))
    edges = np.concatenate([[0], inner[(inner > 0) & (inner < nk)], [nk]]).astype(np.int32)
    rng = np.random.default_rng(np.random.SeedSequence(list(seed) + [77]))
    nb = len(edges) - 1
    V = np.zeros((nb, ndet, rank), np.float64)
    for b in range(nb):
        k0, k1 = int(edges[b]), int(edges[b + 1])
        fb = 0.5 * (k0 + k1 - 1) * fsample / nsamp
        beta = beta_max / (1.0 + (fb / f_atm) ** 2)
        G = np.empty((ndet, rank))
        G[:, 0] = 1.0
        G[:, 1:] = rng.standard_normal((ndet, rank - 1))
        G, _ = np.linalg.qr(G)
        dmin = iN[:, k0:k1].min(axis=1)
        V[b] = np.sqrt(beta) * np.sqrt(dmin)[:, None] * G
    return edges, V.astype(np.float32)
