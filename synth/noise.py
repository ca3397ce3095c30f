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
