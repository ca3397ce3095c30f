"""GPU convergence diagnostics against the oracle: binned TT/EE/BB spectra of
masked maps (square and rectangular, I and I,Q,U), the A-norm estimate on
the device-recorded PCG scalars, and the per-bin cosmic-variance convergence
of binned and circulant PCG."""

import numpy as np
import pytest

import oracle
from oracle import diagnostics as D
from gpu_common import Pair, rel
from synth import raster_scan

pytestmark = pytest.mark.gpu


def _scan(nc, ny, nx, ndet, n, seed=77):
    sweeps = max(1, n // (4 * nx))
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(seed, sweeps))


@pytest.mark.parametrize("nc,ny,nx", [(3, 32, 32), (1, 32, 32), (3, 16, 64)])
def test_spectra_match_oracle(nc, ny, nx):
    pair = Pair(_scan(nc, ny, nx, 4, 2**13), tod_dtype="f64")
    x = np.random.default_rng(3).standard_normal(nc * ny * nx)
    for dell, nbins in ((400.0, 60), (2000.0, 8)):
        got, cnt = pair.g.spectra(pair.dev(x), 0.5, dell, nbins)
        want, wcnt = D.map_spectra(x, pair.mask, ny, nx, 0.5, dell, nbins)
        np.testing.assert_array_equal(cnt, wcnt)
        ok = wcnt > 0
        e = rel(got[:, ok], want[:, ok])
        print(f"[spectra nc={nc} {ny}x{nx} dell={dell}] rel err {e:.2e}", flush=True)
        assert e <= 1e-12
        assert np.all(got[:, ~ok] == 0)


def test_anorm_estimate_from_device_scalars():
    import paper_1309_7473_amd as mm
    pair = Pair(_scan(3, 32, 32, 4, 2**13), tod_dtype="f64")
    pair.g.build_precon("binned")
    b = pair.A_oracle(pair.masked_random(4))
    r = pair.g.pcg("binned", pair.dev(b), tol=1e-8, maxiter=300)
    est = mm.mm_anorm_error_estimate(r["alpha"], r["rho"], 4)
    # the oracle's PCG on the same system records the same scalars
    Mb = oracle.BinnedPrecon(pair.B, pair.mask)
    ro = oracle.pcg(pair.A_oracle, Mb, b, tol=1e-8, maxiter=300)
    eo = oracle.anorm_estimate(ro.alphas, ro.rhos, 4)
    n = min(len(est), len(eo), 20)
    print(f"[anorm] gpu {est[:3]} oracle {eo[:3]}", flush=True)
    assert n >= 10
    np.testing.assert_allclose(est[:n], eo[:n], rtol=1e-8)


def test_power_spectrum_convergence_binned_vs_circulant():
    from paper_1309_7473_amd import diagnostics as G
    inp = _scan(3, 32, 32, 6, 2**15)
    pair = Pair(inp, tod_dtype="f32")
    sky = (inp.sky.reshape(3, -1) * pair.mask).ravel()
    b = pair.dev(pair.A_oracle(sky))
    pair.g.build_precon("binned")
    pair.g.build_precon("circulant", sigma=3.0)
    out = {}
    for name in ("binned", "circulant"):
        d = G.ps_convergence(pair.g, name, b, pair.dev(sky), pixel_arcmin=0.5, dell=2000.0,
                             nbins=10, tol=1e-6, maxiter=400, snap_every=1, block=10)
        out[name] = d
        # one snapshot's errors against the oracle's spectra of the same map
        k = len(d["steps"]) // 2
        conv = np.nanmedian(d["conv_steps"], axis=1)
        print(f"[ps {name}] iters {d['iters']} median convergence step TT/EE/BB {conv}", flush=True)
        assert d["converged"] and np.isfinite(d["conv_steps"]).mean() > 0.5
        assert np.all(d["errors"][-1][np.isfinite(d["errors"][-1])] < 1.0)
    cin, cnt = D.map_spectra(sky, pair.mask, 32, 32, 0.5, 2000.0, 10)
    np.testing.assert_allclose(out["binned"]["c_input"][:, cnt > 0], cin[:, cnt > 0], rtol=1e-10)
