"""The allocation-free spectra entry point (mm_map_spectra_noalloc) against
mm_map_spectra, through the C ABI.

Both run the same kernels on the same map.  The mode counts must be equal
exactly; the spectra to 1e-12 relative, since the binning kernel sums each
block's modes with LDS atomics, whose order (and so the last bits of a
float64 sum over at most a few thousand modes) varies from run to run
(measured 4.5e-16).  Two calls in a row,
the second on a smaller map with fewer bins (the static scratch keeps the
first call's contents, which the second must not see), then a map too
large for the scratch, which is rejected before anything runs.
"""

import numpy as np
import pytest

from gpu_common import Pair
from synth import raster_scan

pytestmark = pytest.mark.gpu


def _scan(nc, ny, nx, ndet, n, seed=5):
    sweeps = max(1, n // (4 * nx))
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(seed, sweeps))


def test_noalloc_spectra_equal_the_workspace_spectra():
    import paper_1309_7473_amd as mm
    cases = [
        # (ncomp, ny, nx, dell, nbins): the second call is smaller in every way
        (3, 64, 64, 300.0, 120),
        (3, 16, 32, 2000.0, 9),
        (1, 32, 32, 500.0, 40),
    ]
    for nc, ny, nx, dell, nbins in cases:
        pair = Pair(_scan(nc, ny, nx, 4, 2**13), tod_dtype="f64")
        x = pair.dev(np.random.default_rng(ny + nx + nc).standard_normal(nc * ny * nx))
        want, wcnt = mm.mm_map_spectra(pair.g.handle, x, 0.5, dell, nbins, nc)
        got, cnt = mm.mm_map_spectra_noalloc(pair.g.handle, x, 0.5, dell, nbins, nc)
        print(f"[noalloc nc={nc} {ny}x{nx} nbins={nbins}] max |diff| "
              f"{np.abs(got - want).max():.3e} modes {int(cnt.sum())}", flush=True)
        assert cnt.sum() > 0 and np.abs(want).max() > 0
        np.testing.assert_array_equal(cnt, wcnt)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
        # twice in a row on the same map
        got2, cnt2 = mm.mm_map_spectra_noalloc(pair.g.handle, x, 0.5, dell, nbins, nc)
        np.testing.assert_array_equal(cnt2, wcnt)
        np.testing.assert_allclose(got2, want, rtol=1e-12, atol=0)
        pair.g.close()


def test_noalloc_spectra_reject_maps_beyond_the_scratch():
    import paper_1309_7473_amd as mm
    # I,Q,U on 2048 x 2048: 3 * 2048^2 * 16 B = 201 MB > 64 MiB
    pair = Pair(_scan(3, 2048, 2048, 1, 2**14), tod_dtype="f32")
    x = pair.dev(np.zeros(3 * 2048 * 2048))
    with pytest.raises(mm.MMError, match="EINVAL"):
        mm.mm_map_spectra_noalloc(pair.g.handle, x, 0.5, 100.0, 10, 3)
    assert "too large" in mm.mm_last_error()
    # the workspace variant still serves it
    spec, cnt = mm.mm_map_spectra(pair.g.handle, x, 0.5, 100.0, 10, 3)
    assert np.all(spec == 0)
    pair.g.close()
