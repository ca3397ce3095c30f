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
    boresight_only,
)
from .noise import (noise_spectrum, inverse_spectrum, draw_noise,  # noqa: F401
                    correlated_inverse_noise)
from .sky import grf_sky  # noqa: F401
from .workloads import make_workload, WORKLOADS, batch_scan_spec  # noqa: F401


def with_correlated_noise(inp, rank=2, nbins=16, beta_max=0.9, f_atm=1.0, seed=(0, 0)):
    """A copy of scan inputs whose inverse noise gains the inter-detector
    correlated part of correlated_inverse_noise."""
    import dataclasses
    edges, V = correlated_inverse_noise(inp.inv_noise, inp.fsample, rank, nbins, beta_max,
                                        f_atm, seed)
    return dataclasses.replace(inp, corr_edges=edges, corr_V=V)
