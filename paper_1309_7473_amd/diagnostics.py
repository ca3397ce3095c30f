"""Convergence diagnostics in the manner of the paper's Results section:
per multipole bin, the error of a PCG iterate's TT/EE/BB spectrum against the
input map's spectrum in units of cosmic variance, and the CG step at which it
falls to a threshold (0.1 cosmic variance), with the errors averaged over
blocks of CG steps (about 50 in the paper) and linearly interpolated between
block centres.  The spectra come from mm_map_spectra on the GPU, the errors
and crossing steps from the library's host functions; this module only
sequences the calls.

Cosmic variance of a bin: sigma_b = C_b(input) sqrt(2 / N_b), N_b = half the
modes of the bin (a real map's independent modes).
"""

import numpy as np


def cv_error(c_iter, c_input, counts):
    """|C(iterate) - C(input)| / sigma_cv per bin, nan for empty bins
    (mm_spectrum_cv_error)."""
    from . import mm_spectrum_cv_error
    c_iter = np.asarray(c_iter, dtype=np.float64)
    return mm_spectrum_cv_error(c_iter, np.broadcast_to(c_input, c_iter.shape), counts)


def crossing_step(steps, errors, threshold=0.1, block=50):
    """CG step where the block-averaged error first reaches `threshold`
    (interpolated between block centres), or None (mm_cv_crossing_step)."""
    from . import mm_cv_crossing_step
    return mm_cv_crossing_step(steps, errors, threshold, block)


def ps_convergence(scan, precon, b, x_input, pixel_arcmin=0.5, dell=100.0, nbins=200,
                   tol=1e-6, maxiter=1000, snap_every=1, block=50, threshold=0.1):
    """Runs PCG from zero, keeps every snap_every-th iterate and returns the
    per-bin cosmic-variance errors of each and the convergence steps."""
    import torch
    from . import mm_anorm_error_estimate
    per = scan.ncomp * scan.npix
    nsnap = maxiter // snap_every
    snaps = torch.zeros(nsnap * per, dtype=torch.float64, device=scan.device)
    res = scan.pcg(precon, b, tol=tol, maxiter=maxiter, check_every=max(1, snap_every),
                   snapshots=snaps, snap_every=snap_every, history=True)
    taken = min(res["iters"] // snap_every, nsnap)
    c_in, counts = scan.spectra(x_input, pixel_arcmin, dell, nbins)
    errs = np.zeros((taken, c_in.shape[0], nbins))
    for k in range(taken):
        c_k, _ = scan.spectra(snaps[k * per:(k + 1) * per], pixel_arcmin, dell, nbins)
        errs[k] = cv_error(c_k, c_in, counts)
    steps = np.arange(1, taken + 1) * snap_every
    conv = np.full((c_in.shape[0], nbins), np.nan)
    for c in range(c_in.shape[0]):
        for bi in range(nbins):
            e = errs[:, c, bi]
            if taken and np.all(np.isfinite(e)):
                s = crossing_step(steps, e, threshold, block)
                conv[c, bi] = np.nan if s is None else s
    return {"iters": res["iters"], "converged": res["converged"], "steps": steps,
            "errors": errs, "conv_steps": conv, "counts": counts, "c_input": c_in,
            "ell_centres": (np.arange(nbins) + 0.5) * dell,
            "anorm_est": mm_anorm_error_estimate(res["alpha"], res["rho"], 4)}
