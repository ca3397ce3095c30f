"""FP64 oracle of the convergence diagnostics of the Results section (test
infrastructure only).

* map_spectra: flat-sky TT (and EE, BB) auto-spectra of a map, binned in
  multipole.  The map is zero outside the active pixels (no apodisation);
  the unnormalised 2-D DFT X(k) of each component gives, for Q and U, the E
  and B modes by the angle phi of the wavevector,
      E = Q cos 2phi + U sin 2phi,   B = -Q sin 2phi + U cos 2phi,
  and C_b = (pixel solid angle / number of pixels) x mean_{k in b} |X(k)|^2
  over the modes with ell = 2 pi |k| / (pixel size) in [b dell, (b+1) dell),
  |k| in cycles per pixel.
* spectrum_error: |C_b(x_i) - C_b(input)| in units of cosmic variance,
  sigma_b = C_b(input) sqrt(2 / N_b) with N_b = (modes in the bin) / 2, the
  independent modes of a real map.
* convergence_step: the CG step at which an error series reaches a
  threshold, the errors averaged over consecutive blocks of CG steps and
  linearly interpolated between the block centres (the Results section uses
  blocks of about 50 steps and a threshold of 0.1 cosmic variance).
"""

import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)


def map_spectra(m, mask, ny, nx, pixel_arcmin, dell, nbins):
    """m: (ncomp, ny*nx) or flat; returns (spectra (1 or 3, nbins): TT[, EE,
    BB], counts (nbins,) of modes in each bin)."""
    m = np.asarray(m, dtype=np.float64)
    nc = m.size // (ny * nx)
    planes = m.reshape(nc, ny, nx) * np.asarray(mask, dtype=np.float64).reshape(1, ny, nx)
    F = np.fft.fft2(planes)
    d = pixel_arcmin * ARCMIN
    ky = np.fft.fftfreq(ny)[:, None] * np.ones((1, nx))
    kx = np.ones((ny, 1)) * np.fft.fftfreq(nx)[None, :]
    ell = 2.0 * np.pi * np.sqrt(ky**2 + kx**2) / d
    b = np.floor(ell / dell).astype(np.int64)
    ok = b < nbins
    if nc == 3:
        phi = np.arctan2(ky, kx)
        c2, s2 = np.cos(2 * phi), np.sin(2 * phi)
        E = F[1] * c2 + F[2] * s2
        B = -F[1] * s2 + F[2] * c2
        comps = [F[0], E, B]
    else:
        comps = [F[0]]
    norm = d * d / (ny * nx)
    counts = np.bincount(b[ok], minlength=nbins).astype(np.float64)
    out = np.zeros((len(comps), nbins))
    for i, X in enumerate(comps):
        p = np.abs(X) ** 2 * norm
        s = np.bincount(b[ok], weights=p[ok], minlength=nbins)
        out[i] = np.where(counts > 0, s / np.maximum(counts, 1), 0.0)
    return out, counts


def spectrum_error(c_iter, c_input, counts):
    """|C(x_i) - C(input)| / sigma_cv per bin (nan where the bin is empty or
    the input spectrum vanishes)."""
    nind = np.asarray(counts, dtype=np.float64) / 2.0
    sig = np.asarray(c_input) * np.sqrt(2.0 / np.maximum(nind, 1e-300))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.abs(np.asarray(c_iter) - np.asarray(c_input)) / sig
    return np.where((nind > 0) & (sig > 0), e, np.nan)


def convergence_step(steps, errors, threshold=0.1, block=50):
    """First CG step where the block-averaged, linearly interpolated error
    series falls to `threshold`; None if it never does."""
    steps = np.asarray(steps, dtype=np.float64)
    errors = np.asarray(errors, dtype=np.float64)
    centres, values = [], []
    for j0 in range(0, len(steps), block):
        centres.append(steps[j0:j0 + block].mean())
        values.append(errors[j0:j0 + block].mean())
    for j, v in enumerate(values):
        if v <= threshold:
            if j == 0:
                return float(centres[0])
            c0, v0, c1 = centres[j - 1], values[j - 1], centres[j]
            return float(c0 + (v0 - threshold) * (c1 - c0) / (v0 - v))
    return None
