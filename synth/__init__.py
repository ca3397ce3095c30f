"""Seeded synthetic inputs for the map-making tests and benchmarks.

This package only *draws inputs*: raster-scan pointing (pixel index and the
polarisation weights cos 2psi, sin 2psi), per-detector noise power spectra and
their inverses, noise realisations, and Gaussian-random-field skies.  It holds
none of the map-making arithmetic (no pointing-matrix apply, no noise filter,
no preconditioner); both the FP64 oracle and the GPU library consume what it
produces, and neither is imported here.
"""

from .scan import (  # noqa: F401
    ScanInputs,
    raster_scan,
    periodic_torus_scan,
    crosslinked_torus_scan,
    hex_focal_plane,
)
from .noise import noise_spectrum, inverse_spectrum, draw_noise  # noqa: F401
from .sky import grf_sky  # noqa: F401
from .workloads import make_workload, WORKLOADS, batch_scan_spec  # noqa: F401
