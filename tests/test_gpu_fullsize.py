"""Parity at the benchmark's full size and launch configuration.

iqu_256det: 256 detectors x 2^20 samples, 512 x 512 I,Q,U map, float32
timestream, float64 accumulation, the library's default plan (128-detector
groups, four-step 512 x 1024, angle-coded weights, pixel-major gather for
P^T) -- the scan object the benchmark times.  The oracle's A-apply on the
whole scan takes seconds in NumPy, so every pixel of the output is compared,
not a sample.  Tolerances as in test_gpu_apply: 2e-6 relative L2 for a white
random map, 2e-5 for the smooth sky.
"""

import numpy as np
import pytest

import oracle
from gpu_common import need_gpu, rel
from synth import make_workload

pytestmark = pytest.mark.gpu

TOL32_WHITE = 2e-6
TOL32_SKY = 2e-5


def test_iqu256_full_size_apply():
    mm = need_gpu()
    import torch
    inp = make_workload("iqu_256det")
    print("[full size] iqu_256det generated", flush=True)
    g = mm.Scan(inp, tod_dtype="f32")
    info = g.info()
    print(f"[full size] plan {info}", flush=True)
    assert (info["det_group"], info["fft_m1"], info["fft_m2"]) == (128, 512, 1024)
    assert info["csr"] == 1 and info["gather_weights"] == 2
    o = oracle.OracleScan(inp)
    B = oracle.binned_blocks(o, oracle.detector_weights(o))
    mask = oracle.active_mask(o, B)
    gmask = g.mask().cpu().numpy().astype(bool)
    assert np.array_equal(gmask, mask)
    assert mask.sum() > 0
    nc, npix = inp.ncomp, inp.ny * inp.nx
    rnd = (np.random.default_rng(5).standard_normal((nc, npix)) * mask).ravel()
    sky = (inp.sky.reshape(nc, npix) * mask).ravel()
    for label, x, tol in (("random", rnd, TOL32_WHITE), ("sky", sky, TOL32_SKY)):
        y = g.apply_A(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        want = oracle.apply_A(o, x, mask)
        e = rel(got, want)
        print(f"[full size] {label} map rel err {e:.3e}", flush=True)
        assert e <= tol, e
        assert np.all(got.reshape(nc, -1)[:, ~mask] == 0)
