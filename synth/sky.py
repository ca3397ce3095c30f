"""Flat-sky Gaussian random field skies.

Intensity has power P(k) proportional to |k|^-2 with the k = 0 mode removed,
rescaled to unit RMS; Q and U are independent fields of the same shape scaled
to RMS 0.1.  Returned in the component-major layout [ncomp][ny][nx].
"""

import numpy as np


def _grf(ny, nx, rng, index=-2.0):
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k2 = ky**2 + kx**2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (index / 4.0)  # sqrt(|k|^index)
    w = rng.standard_normal((ny, nx))
    field = np.fft.irfft2(np.fft.rfft2(w) * amp, s=(ny, nx))
    rms = np.sqrt(np.mean(field**2))
    return field / rms if rms > 0 else field


def grf_sky(ncomp, ny, nx, rng):
    comps = [_grf(ny, nx, rng)]
    for _ in range(ncomp - 1):
        comps.append(0.1 * _grf(ny, nx, rng))
    return np.stack(comps, axis=0)
