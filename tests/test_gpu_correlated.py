"""Inter-detector correlated inverse noise on the GPU against the oracle:
A-apply and the right-hand side in float64 and float32, V = 0 against the
independent path, symmetry of A, the detector weights of the binned
preconditioner, and PCG to 1e-6 under the oracle's A."""

import dataclasses

import numpy as np
import pytest

import oracle
from gpu_common import Pair, rel
from synth import raster_scan, with_correlated_noise
from test_gpu_apply import make_sky, TOL64, TOL32_WHITE, TOL32_SKY

pytestmark = pytest.mark.gpu


def _scan(nc=3, ny=32, nx=32, ndet=6, n=2**14, rank=2, nbins=16, seed=77):
    inp = raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0, layout="hex",
                      hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1, fknee=(0.5, 2.0),
                      drift_deg=10.0, seed=(seed, n // (4 * nx)))
    return with_correlated_noise(inp, rank=rank, nbins=nbins, seed=(seed, 1))


CASES = [
    # (label, nc, ndet, n, rank, dtype)
    ("f64-rank2-m2=512", 3, 6, 2**14, 2, "f64"),
    ("f64-rank4-m2=512", 3, 5, 2**15, 4, "f64"),
    ("f32-rank2", 3, 6, 2**14, 2, "f32"),
    ("f32-I-rank3", 1, 4, 2**13, 3, "f32"),
    ("f64-m2=1024", 3, 3, 2**20, 2, "f64"),
    ("f32-rank6", 3, 8, 2**14, 6, "f32"),
    ("f64-rank12", 3, 14, 2**14, 12, "f64"),
    ("bf16-rank2", 3, 6, 2**14, 2, "bf16"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_correlated_apply_and_rhs_parity(case):
    label, nc, ndet, n, rank, dt = case
    inp = _scan(nc=nc, ndet=ndet, n=n, rank=rank)
    pair = Pair(inp, tod_dtype=dt)
    info = pair.g.info()
    assert info["det_group"] == ndet and info["single_pass"] == 0
    x = pair.masked_random(1)
    sky = (make_sky(nc, 32, 32) * pair.mask.reshape(1, 32, 32)).ravel()
    for name, v, t32 in (("random", x, TOL32_WHITE), ("sky", sky, TOL32_SKY)):
        e = rel(pair.A_gpu(v), pair.A_oracle(v))
        print(f"[corr {label}] A {name} rel err {e:.3e} (m1 {info['fft_m1']} m2 {info['fft_m2']})",
              flush=True)
        assert e <= {"f64": TOL64, "f32": t32, "bf16": 2.0**-8}[dt], e
    import torch
    tod = np.random.default_rng(5).standard_normal((ndet, n))
    b_want = oracle.rhs(pair.o, tod, pair.mask)
    if dt == "bf16":   # the caller hands bfloat16 data: both sides see it
        tod = torch.from_numpy(tod.astype(np.float32)).to(torch.bfloat16).double().numpy()
        b_want = oracle.rhs(pair.o, tod, pair.mask)
    tdev = torch.from_numpy(tod.astype(np.float64 if dt == "f64" else np.float32)).cuda()
    b_got = pair.host(pair.g.rhs(tdev))
    e = rel(b_got, b_want)
    print(f"[corr {label}] rhs rel err {e:.3e}", flush=True)
    assert e <= {"f64": TOL64, "f32": 3e-6, "bf16": 2 * 2.0**-8}[dt], e


def test_zero_correlation_equals_the_independent_path():
    inp = _scan()
    z = dataclasses.replace(inp, corr_V=np.zeros_like(inp.corr_V))
    ind = dataclasses.replace(inp, corr_edges=None, corr_V=None)
    a, b = Pair(z, tod_dtype="f64"), Pair(ind, tod_dtype="f64")
    x = a.masked_random(2)
    assert rel(a.A_gpu(x), b.A_gpu(x)) <= 1e-13
    # and the correlation matters for the real model
    c = Pair(inp, tod_dtype="f64")
    assert rel(c.A_gpu(x), b.A_gpu(x)) > 1e-3


def test_correlated_A_symmetric_and_binned_weights():
    inp = _scan(rank=3)
    pair = Pair(inp, tod_dtype="f64")
    x, y = pair.masked_random(3), pair.masked_random(4)
    a, b = x @ pair.A_gpu(y), y @ pair.A_gpu(x)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    # binned preconditioner from the diagonal of the correlated N^-1
    pair.g.build_precon("binned")
    r = pair.masked_random(5)
    want = oracle.BinnedPrecon(pair.B, pair.mask)(r)
    got = pair.host(pair.g.apply_precon("binned", pair.dev(r)))
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("precon", ["binned", "circulant"])
def test_correlated_pcg(precon):
    inp = _scan(ndet=6, n=2**15, rank=2)
    pair = Pair(inp, tod_dtype="f64")
    sky = (inp.sky.reshape(3, -1) * pair.mask).ravel()
    b = pair.A_oracle(sky)
    if precon == "circulant":
        pair.g.build_precon("circulant", sigma=3.0)
    else:
        pair.g.build_precon("binned")
    r = pair.g.pcg(precon, pair.dev(b), tol=1e-6, maxiter=2000)
    x = pair.host(r["x"])
    t = rel(pair.A_oracle(x), b)
    line = f"[corr pcg {precon}] iters {r['iters']} true resid {t:.2e}"
    if precon == "binned":
        ro = oracle.pcg(pair.A_oracle, oracle.BinnedPrecon(pair.B, pair.mask), b, tol=1e-6,
                        maxiter=2000)
        line += f" oracle iters {ro.iters}"
        assert abs(r["iters"] - ro.iters) <= max(2, 0.05 * ro.iters)
    print(line, flush=True)
    assert r["converged"] and t <= 1.5e-6
