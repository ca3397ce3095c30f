"""Parity at the benchmark's full size and launch configuration.

iqu_256det: 256 detectors x 2^20 samples, 512 x 512 I,Q,U map, float32
timestream, float64 accumulation, the library's default plan (128-detector
groups, four-step 512 x 1024, angle-coded weights, pixel-major gather for
P^T) -- the scan object the benchmark times, with its 20-pixel circulant
taper.  The oracle's A-apply on the whole scan takes seconds in NumPy, so
every pixel of each output is compared, not a sample.  Tolerances as in the
smaller parity tests: A-apply 2e-6 relative L2 for a white random map and
2e-5 for the smooth sky; circulant apply 1e-4 (its probe rows come from the
float32 A-apply); every output is also held element-wise to the same
tolerance times its largest entry.  The PCG solution (tolerance 1e-6, with the
library's true-residual check and restarts) must meet 1e-6 in the true
residual ||b - A x|| / ||b|| under the oracle's float64 A.
"""

import numpy as np
import pytest

import oracle
from gpu_common import need_gpu, rel, relmax
from synth import make_workload

pytestmark = pytest.mark.gpu

TOL32_WHITE = 2e-6
TOL32_SKY = 2e-5
TAPER_PX = 20.0


@pytest.fixture(scope="module")
def full():
    mm = need_gpu()
    import torch
    inp = make_workload("iqu_256det")
    print("[full size] iqu_256det generated", flush=True)
    g = mm.Scan(inp, tod_dtype="f32")
    o = oracle.OracleScan(inp)
    B = oracle.binned_blocks(o, oracle.detector_weights(o))
    mask = oracle.active_mask(o, B)
    yield inp, g, o, B, mask, torch
    g.close()


def _to_host(torch, t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_iqu256_full_size_apply(full):
    inp, g, o, B, mask, torch = full
    info = g.info()
    print(f"[full size] plan {info}", flush=True)
    assert (info["det_group"], info["fft_m1"], info["fft_m2"]) == (128, 512, 1024)
    assert info["csr"] == 2 and info["gather_weights"] == 2
    assert np.array_equal(g.mask().cpu().numpy().astype(bool), mask)
    assert mask.sum() > 0
    nc, npix = inp.ncomp, inp.ny * inp.nx
    rnd = (np.random.default_rng(5).standard_normal((nc, npix)) * mask).ravel()
    sky = (inp.sky.reshape(nc, npix) * mask).ravel()
    for label, x, tol in (("random", rnd, TOL32_WHITE), ("sky", sky, TOL32_SKY)):
        got = _to_host(torch, g.apply_A(torch.from_numpy(x).cuda()))
        want = oracle.apply_A(o, x, mask)
        e, emax = rel(got, want), relmax(got, want)
        print(f"[full size] {label} map rel err {e:.3e} max {emax:.3e}", flush=True)
        assert e <= tol and emax <= tol, (e, emax)
        assert np.all(got.reshape(nc, -1)[:, ~mask] == 0)


def test_iqu256_full_size_circulant_and_pcg(full):
    inp, g, o, B, mask, torch = full
    nc, npix = inp.ncomp, inp.ny * inp.nx
    Mo = oracle.CirculantPrecon(o, mask, B, sigma_taper=TAPER_PX)
    g.build_precon("circulant", sigma=TAPER_PX)
    info = g.info()
    assert info["ref_pixel"] == Mo.ref
    assert info["n_floored"] == Mo.n_floored
    r = (np.random.default_rng(6).standard_normal((nc, npix)) * mask).ravel()
    got = _to_host(torch, g.apply_precon("circulant", torch.from_numpy(r).cuda()))
    want = Mo(r)
    e, emax = rel(got, want), relmax(got, want)
    print(f"[full size] circulant apply rel err {e:.3e} max {emax:.3e} "
          f"floored={info['n_floored']}", flush=True)
    assert e <= 1e-4 and emax <= 1e-4, (e, emax)
    # PCG to 1e-6 on b = A m_sky (oracle), checked under the oracle's A
    b = oracle.apply_A(o, (inp.sky.reshape(nc, npix) * mask).ravel(), mask)
    res = g.pcg("circulant", torch.from_numpy(b).cuda(), tol=1e-6, maxiter=2000, refine=2)
    x = _to_host(torch, res["x"])
    tr = np.linalg.norm(b - oracle.apply_A(o, x, mask)) / np.linalg.norm(b)
    print(f"[full size] circulant PCG iters={res['iters']} rel={res['rel_resid']:.2e} "
          f"gpu true={res['true_rel_resid']:.2e} restarts={res['restarts']} "
          f"oracle true={tr:.2e}", flush=True)
    assert res["converged"] and res["true_rel_resid"] <= 1e-6
    assert tr <= 1e-6, tr
