"""The benchmark workloads as seeded synthetic scans.

Workloads (seed tag in brackets):

* "intensity_small" [1]: intensity only, 8 detectors on a cross-scan line x
  2^14 samples at 100 Hz, 64 x 64 map, white (sigma = 1) + 1/f (f_knee =
  1 Hz, index -3) noise, no scan-angle drift;
* "iqu_256det" [2]: I,Q,U, 256 detectors on a hexagonal focal plane 0.5 deg
  (60 px) across, 2^20 samples at 400 Hz, 512 x 512 map, linear scan-angle
  drift of at most +-10 deg in total, psi_d ~ U[0, pi), sigma_d log-normal
  with 10 % scatter, f_knee,d ~ U(0.5, 3) Hz, index -3;
* "iqu_1024det" [3]: the pattern of iqu_256det at 1024 detectors x 2^21
  samples on a 1024 x 1024 map (the precision study);
* "batch_64scans" [4]: 64 independent scans: per scan ndet ~ U{32..512},
  nsamp = 2^U{16..21}, square L x L maps with L = 2^U{7..10}, 4 samples per
  pixel along a sweep (so the row advance per sweep is 4 L^2 / nsamp), a hex
  focal plane max(60 px, twice the row advance) across, noise as iqu_256det;
* "iqu_256det_learned" [5]: the shape of iqu_256det for the learned
  correction (scan ids 0..7 train, 1000.. held out).

`make_workload(name, scan_id, **overrides)` draws one scan; overrides shrink
a workload for tests (e.g. ndet, nsamp, ny, nx) while keeping its recipe.
Seeds are numpy SeedSequence([tag, scan_id]) with spawned children for the
sky, focal plane, detector angles, noise parameters, drift and noise draws.
"""

from .scan import raster_scan

_IQU = dict(ncomp=3, fsample=400.0, layout="hex", hex_diameter_px=60.0, sigma=1.0,
            sigma_scatter=0.1, fknee=(0.5, 3.0), alpha=-3.0, drift_deg=10.0)

WORKLOADS = {
    "intensity_small": (1, dict(ncomp=1, ndet=8, nsamp=2**14, fsample=100.0, ny=64, nx=64,
                                layout="line", sigma=1.0, sigma_scatter=0.0, fknee=(1.0, 1.0),
                                alpha=-3.0, drift_deg=0.0)),
    "iqu_256det": (2, dict(_IQU, ndet=256, nsamp=2**20, ny=512, nx=512)),
    "iqu_1024det": (3, dict(_IQU, ndet=1024, nsamp=2**21, ny=1024, nx=1024)),
    "batch_64scans": (4, None),
    "iqu_256det_learned": (5, dict(_IQU, ndet=256, nsamp=2**20, ny=512, nx=512)),
}


def batch_scan_spec(scan_id):
    """Shape of scan `scan_id` (0..63) of the batch_64scans workload."""
    import numpy as np
    rng = np.random.default_rng(np.random.SeedSequence([4, 0, int(scan_id)]))
    ndet = int(rng.integers(32, 513))
    nsamp = 2 ** int(rng.integers(16, 22))
    side = 2 ** int(rng.integers(7, 11))
    advance = 4.0 * side * side / nsamp
    return dict(_IQU, ndet=ndet, nsamp=nsamp, ny=side, nx=side,
                hex_diameter_px=max(60.0, 2.0 * advance))


def make_workload(name, scan_id=0, **overrides):
    tag, spec = WORKLOADS[name]
    spec = batch_scan_spec(scan_id) if spec is None else dict(spec)
    spec.update(overrides)
    return raster_scan(seed=(tag, scan_id), **spec)
