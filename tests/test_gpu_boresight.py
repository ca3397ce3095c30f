"""GPU parity of the pointing computed from the boresight model (each
sample's pixel and weights formed inside the kernels from the boresight track
and the detector offsets) against the oracle, which expands the same model in
float64 on the CPU.

Pixel decisions are integer results: the mask, hit counts and every
pixel-dependent output must agree exactly with the oracle's expansion (both
sides evaluate the same float64 expressions without fused multiply-add).
Tolerances otherwise as for stored pointing: float64 path 1e-12, float32
2e-6 (white map); bfloat16 storage 4e-3 (2^-8, rounded three times).
"""

import numpy as np
import pytest

import oracle
from gpu_common import Pair, rel, need_gpu
from synth import raster_scan, boresight_only, make_workload

pytestmark = pytest.mark.gpu

CASES = [
    # label, ncomp, ny, nx, ndet, nsamp, dtype, acc, det_group, fft_m1
    ("single-f64-I", 1, 16, 16, 5, 2**10, "f64", "f64", 0, 0),
    ("single-f32-IQU", 3, 16, 16, 5, 2**12, "f32", "f64", 0, 0),
    ("single-f64-IQU", 3, 16, 16, 3, 2**13, "f64", "f64", 0, 0),
    ("min-n-I", 1, 8, 8, 6, 32, "f64", "f64", 0, 0),
    ("fourstep-f64-IQU", 3, 32, 32, 3, 2**16, "f64", "f64", 2, 0),
    ("fourstep-f32-IQU-ragged", 3, 32, 32, 5, 2**15, "f32", "f64", 2, 0),
    ("fourstep-f32-I-m1=512", 1, 32, 32, 2, 2**18, "f32", "f64", 1, 512),
    ("fourstep-f32-IQU-m2=2048", 3, 32, 32, 3, 2**15, "f32", "f64", 3, 8),
    ("fourstep-f32x2-IQU", 3, 32, 32, 4, 2**15, "f32", "f32x2", 0, 0),
    ("fourstep-bf16-IQU", 3, 32, 32, 4, 2**15, "bf16", "f64", 0, 0),
]
TOL = {"f64": 1e-12, "f32": 2e-6, "bf16": 4e-3}


def _inputs(nc, ny, nx, ndet, n, seed):
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(91, seed))


@pytest.mark.parametrize("scatter,csr", [("auto", 2), ("samples", 1)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_boresight_apply_rhs_and_binned(case, scatter, csr):
    # auto: the run-length index (pixel-major angles from the model's weights
    # on the float paths, the model's float64 weights on the float64 path);
    # samples: the per-sample index
    label, nc, ny, nx, ndet, n, dt, acc, G, m1 = case
    inp = boresight_only(_inputs(nc, ny, nx, ndet, n, ndet))
    pair = Pair(inp, tod_dtype=dt, acc=acc, det_group=G, fft_m1=m1, scatter=scatter)
    info = pair.g.info()
    print(f"[boresight {label} {scatter}] {info}", flush=True)
    assert info["csr"] == csr
    # mask: integer decisions, exact
    mask = pair.host(pair.g.mask()).astype(bool)
    assert np.array_equal(mask, pair.mask), "active pixels differ from the oracle's"
    assert pair.mask.sum() > 0
    x = pair.masked_random(1)
    e = rel(pair.A_gpu(x), pair.A_oracle(x))
    # right-hand side of a noise-free timestream
    tod = oracle.pointing(pair.o, x.reshape(nc, -1))
    b_want = oracle.rhs(pair.o, tod, pair.mask)
    b_got = pair.host(pair.g.rhs(pair.torch.from_numpy(tod)))
    eb = rel(b_got, b_want)
    # binned preconditioner from the on-the-fly weights
    r = pair.masked_random(2)
    eM = rel(pair.host(pair.g.apply_precon("binned", pair.dev(r))),
             oracle.BinnedPrecon(pair.B, pair.mask)(r))
    print(f"[boresight {label}] A {e:.2e} rhs {eb:.2e} binned {eM:.2e}", flush=True)
    tol = TOL[dt]
    assert e <= tol and eb <= 2 * tol
    assert eM <= (1e-12 if dt != "bf16" else 1e-12)


def test_boresight_equals_stored_pointing_on_the_gpu():
    """Same scan, both pointing modes on the GPU, float64 path: identical
    masks and hit structure; results differ only by the float32 rounding of
    the stored weights."""
    inp = _inputs(3, 32, 32, 5, 2**15, 3)
    a = Pair(inp, tod_dtype="f64")
    b = Pair(boresight_only(inp), tod_dtype="f64")
    assert np.array_equal(a.host(a.g.mask()), b.host(b.g.mask()))
    assert a.g.info()["n_active"] == b.g.info()["n_active"]
    x = a.masked_random(4)
    e = rel(b.A_gpu(x), a.A_gpu(x))
    print(f"[boresight vs stored f64] {e:.2e}", flush=True)
    assert 0 < e <= 3e-7


@pytest.mark.parametrize("precon", ["binned", "circulant"])
def test_boresight_pcg(precon):
    inp = _inputs(3, 32, 32, 6, 2**15, 5)
    pair = Pair(boresight_only(inp), tod_dtype="f64")
    m = np.random.default_rng(3).standard_normal((3, 32 * 32)) * pair.mask
    b = pair.A_oracle(m.ravel())
    if precon == "circulant":
        pair.g.build_precon("circulant", sigma=3.0)
        M = oracle.CirculantPrecon(pair.o, pair.mask, pair.B, sigma_taper=3.0)
    else:
        M = oracle.BinnedPrecon(pair.B, pair.mask)
    ro = oracle.pcg(pair.A_oracle, M, b, tol=1e-8, maxiter=2000)
    rg = pair.g.pcg(precon, pair.dev(b), tol=1e-8, maxiter=2000)
    x = pair.host(rg["x"])
    tr = np.linalg.norm(b - pair.A_oracle(x)) / np.linalg.norm(b)
    print(f"[boresight pcg {precon}] oracle {ro.iters} gpu {rg['iters']} true {tr:.2e}", flush=True)
    assert rg["converged"] and ro.converged and abs(rg["iters"] - ro.iters) <= 1 and tr <= 1e-7


def test_boresight_at_full_launch_geometry():
    """iqu_256det's shape (2^20 samples, 512 x 512, 60 px focal plane) with 16
    detectors, float32: against the stored-pointing GPU path, which the
    oracle validates at this geometry, and against the oracle on the mask."""
    inp = make_workload("iqu_256det", ndet=16)
    need_gpu()
    import paper_1309_7473_amd as mm
    import torch
    sa = mm.Scan(inp, tod_dtype="f32")
    sb = mm.Scan(boresight_only(inp), tod_dtype="f32")
    ma = sa.mask()
    assert torch.equal(ma, sb.mask())
    assert sa.info()["fft_m1"] == sb.info()["fft_m1"]
    x = torch.from_numpy(inp.sky.ravel().copy()).cuda() * ma.repeat(3).double()
    ya, yb = sa.apply_A(x), sb.apply_A(x)
    torch.cuda.synchronize()
    e = rel(yb.cpu().numpy(), ya.cpu().numpy())
    print(f"[boresight full geometry] rel to stored {e:.2e}", flush=True)
    assert e <= 2e-5
    sa.close()
    sb.close()


def test_boresight_errors():
    mm = need_gpu()
    import torch
    inp = _inputs(3, 16, 16, 3, 2**12, 9)
    with pytest.raises(mm.MMError, match="EINVAL"):
        mm.Scan(boresight_only(inp), scatter="atomic")
    bad = boresight_only(inp)
    bad.bore = bad.bore.copy()
    bad.bore[1, 7] = np.nan
    with pytest.raises(mm.MMError, match="non-finite"):
        mm.Scan(bad)
    # stored pointing passed together with the boresight mode is rejected
    s = mm.Scan(boresight_only(inp))
    d = s.desc
    d.pix = s.inv_noise.data_ptr()
    with pytest.raises(mm.MMError, match="must be NULL"):
        mm.mm_create_scan(d)
    d.pix = None
    d.bore = s.bore.data_ptr() + 8
    with pytest.raises(mm.MMError, match="aligned"):
        mm.mm_create_scan(d)
    d.bore = None
    with pytest.raises(mm.MMError, match="required"):
        mm.mm_create_scan(d)
    torch.cuda.synchronize()
    s.close()
