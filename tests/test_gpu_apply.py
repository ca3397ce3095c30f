"""GPU parity of the A-apply and the right-hand side against the FP64 oracle.

Tolerances (relative L2, GPU vs oracle on identical inputs):
  float64 timestream path: 1e-12;
  float32 timestream path: 2e-6 for a white random map (the FFT/filter
  rounding of ~1e-7 relative, grown by log2 n stages) and 2e-5 for a smooth
  sky map, whose filtered timestream is small next to the timestream itself
  because 1/N(f) removes most of its low-frequency power.
"""

import numpy as np
import pytest

import oracle
from conftest import small_raster
from gpu_common import Pair, rel, relmax, need_gpu
from synth import make_workload, raster_scan

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_WHITE = 2e-6
TOL32_SKY = 2e-5


def _check_apply(pair, tol, seed=0, label=""):
    assert pair.mask.sum() > 0, "no active pixel: the comparison would be vacuous"
    x = pair.masked_random(seed)
    got, want = pair.A_gpu(x), pair.A_oracle(x)
    e, emax = rel(got, want), relmax(got, want)
    print(f"[apply {label}] rel err random map = {e:.3e} max {emax:.3e}", flush=True)
    assert e <= tol and emax <= tol, (e, emax)
    # inactive pixels are zero
    assert np.all(got.reshape(pair.nc, -1)[:, ~pair.mask] == 0)
    return e


CASES = [
    # (label, ncomp, ny, nx, ndet, nsamp, dtype, det_group, fft_m1)
    ("single-f32-I", 1, 16, 16, 5, 2**10, "f32", 0, 0),
    ("single-f32-IQU", 3, 16, 16, 5, 2**12, "f32", 0, 0),
    ("single-f64-IQU", 3, 16, 16, 3, 2**13, "f64", 0, 0),
    ("min-n", 1, 8, 8, 1, 16, "f32", 0, 0),
    ("min-n-IQU", 3, 8, 8, 6, 32, "f64", 0, 0),
    ("single-max-f32", 3, 32, 32, 6, 2**14, "f32", 0, 0),
    ("fourstep-f32-ragged", 3, 32, 32, 5, 2**15, "f32", 2, 0),
    ("fourstep-f32-m1=16", 3, 32, 32, 3, 2**15, "f32", 0, 16),
    ("fourstep-f32-m1=512", 1, 32, 32, 2, 2**18, "f32", 1, 512),
    ("fourstep-f32-m1=1024", 3, 32, 32, 5, 2**18, "f32", 2, 1024),
    ("fourstep-f64", 3, 32, 32, 3, 2**16, "f64", 2, 0),
    ("fourstep-f64-m1=8", 1, 16, 16, 2, 2**15, "f64", 0, 8),
    # rows of 512 and 1024 bins take one wavefront a row in pass 2, rows
    # of 2048 bins two
    ("fourstep-f32-m2=512", 3, 32, 32, 3, 2**15, "f32", 0, 32),
    ("fourstep-f32-m2=2048", 3, 32, 32, 3, 2**15, "f32", 3, 8),
    ("fourstep-f64-m2=512", 3, 32, 32, 3, 2**15, "f64", 0, 32),
    ("fourstep-f64-m2=1024", 3, 32, 32, 5, 2**15, "f64", 2, 16),
    ("fourstep-f64-m2=2048", 3, 32, 32, 3, 2**15, "f64", 0, 8),
]


@pytest.mark.parametrize("scatter", ["auto", "atomic", "samples"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_apply_A_parity(case, scatter):
    label, nc, ny, nx, ndet, n, dt, G, m1 = case
    if scatter != "auto" and not label.startswith("fourstep"):
        pytest.skip("the one-kernel path has only the atomic scatter")
    sweeps = max(1, n // (4 * nx))
    inp = raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                      layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                      fknee=(0.5, 2.0), drift_deg=10.0, seed=(77, sweeps))
    pair = Pair(inp, tod_dtype=dt, det_group=G, fft_m1=m1, scatter=scatter)
    info = pair.g.info()
    print(label, info, flush=True)
    want_csr = 0 if not label.startswith("fourstep") else {"auto": 2, "atomic": 0,
                                                              "samples": 1}[scatter]
    assert info["csr"] == want_csr
    if m1:
        assert info["fft_m1"] == m1
    tol = TOL64 if dt == "f64" else TOL32_WHITE
    _check_apply(pair, tol, label=label)
    sky = make_sky(nc, ny, nx) * pair.mask.reshape(1, ny, nx)
    want = pair.A_oracle(sky.ravel())
    assert np.linalg.norm(want) > 0
    got = pair.A_gpu(sky.ravel())
    e, emax = rel(got, want), relmax(got, want)
    print(f"[apply {label}] rel err sky map = {e:.3e} max {emax:.3e}", flush=True)
    tol = TOL64 if dt == "f64" else TOL32_SKY
    assert e <= tol and emax <= tol, (e, emax)


def make_sky(nc, ny, nx):
    from synth import grf_sky
    return grf_sky(nc, ny, nx, np.random.default_rng(5))


def test_intensity_small_full_size_f64():
    inp = make_workload("intensity_small")
    pair = Pair(inp, tod_dtype="f64")
    assert pair.g.info()["single_pass"] == 1
    assert pair.g.info()["n_active"] == int(pair.mask.sum())
    _check_apply(pair, TOL64, label="intensity_small")
    sky = (inp.sky * pair.mask.reshape(1, 64, 64)).ravel()
    assert rel(pair.A_gpu(sky), pair.A_oracle(sky)) <= TOL64


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_rhs_parity(dt):
    inp = small_raster(ncomp=3, ny=32, nx=32, ndet=4, sweeps=256)  # n = 2^15, four-step
    pair = Pair(inp, tod_dtype=dt, det_group=3)
    rng = np.random.default_rng(3)
    noise = np.stack([np.fft.irfft(np.sqrt(inp.spectrum[d]) * np.fft.rfft(
        rng.standard_normal(inp.nsamp)), inp.nsamp) for d in range(inp.ndet)])
    d = oracle.pointing(pair.o, inp.sky) + noise
    d = d.astype(np.float32 if dt == "f32" else np.float64)
    want = oracle.rhs(pair.o, d.astype(np.float64), pair.mask)
    got = pair.host(pair.g.rhs(pair.torch.from_numpy(d).cuda()))
    e = rel(got, want)
    print(f"[rhs {dt}] rel err = {e:.3e}", flush=True)
    assert e <= (TOL64 if dt == "f64" else TOL32_SKY)


def test_A_symmetric_on_gpu_f64():
    inp = small_raster(ncomp=3, ny=32, nx=32, ndet=6, sweeps=256)
    pair = Pair(inp, tod_dtype="f64", det_group=4)
    x, y = pair.masked_random(1), pair.masked_random(2)
    Ax, Ay = pair.A_gpu(x), pair.A_gpu(y)
    assert abs(x @ Ay - y @ Ax) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(Ay)


def test_mask_and_hits_match_oracle():
    inp = small_raster(ncomp=3, ny=16, nx=16, ndet=4, diameter=4.0)
    pair = Pair(inp, tod_dtype="f32")
    m = pair.host(pair.g.mask())
    np.testing.assert_array_equal(m.astype(bool), pair.mask)


def test_collision_stress_long_runs():
    # intensity only, so that every hit pixel is an unknown: every sample of
    # detector 0 in one pixel, detector 1 alternating between two pixels,
    # detector 2 entirely off the map, detector 3 an ordinary raster
    inp = small_raster(ncomp=1, ny=16, nx=16, ndet=4, sweeps=128)  # n = 8192
    inp.pix[0, :] = 5 * 16 + 7
    inp.pix[1, :] = np.where(np.arange(inp.nsamp) % 2 == 0, 3, 200)
    inp.pix[2, :] = -1
    for dt, tol in (("f32", TOL32_WHITE), ("f64", TOL64)):
        pair = Pair(inp, tod_dtype=dt)
        assert pair.mask[5 * 16 + 7] and pair.mask[3] and pair.mask[200]
        _check_apply(pair, tol, label=f"collision-{dt}")
    # the same on the four-step pipeline, both forms of P^T
    inp2 = small_raster(ncomp=1, ny=16, nx=16, ndet=4, sweeps=512)  # n = 2^15
    inp2.pix[0, :] = 5 * 16 + 7
    inp2.pix[1, :] = np.where(np.arange(inp2.nsamp) % 2 == 0, 3, 200)
    inp2.pix[2, :] = -1
    for scatter in ("auto", "atomic"):
        pair = Pair(inp2, tod_dtype="f64", det_group=2, scatter=scatter)
        _check_apply(pair, TOL64, label=f"collision-fourstep-{scatter}")
    # I,Q,U: six detectors with distinct angles share one pixel for all samples
    inp3 = small_raster(ncomp=3, ny=8, nx=8, ndet=6, sweeps=64)
    inp3.pix[:3, :] = 3 * 8 + 4
    pair = Pair(inp3, tod_dtype="f64")
    assert pair.mask[3 * 8 + 4]
    _check_apply(pair, TOL64, label="collision-IQU")


@pytest.mark.parametrize("scatter,csr", [("auto", 2), ("samples", 1)])
def test_apply_A_bitwise_repeatable(scatter, csr):
    inp = small_raster(ncomp=3, ny=32, nx=32, ndet=5, sweeps=256)
    pair = Pair(inp, tod_dtype="f32", det_group=2, scatter=scatter)
    assert pair.g.info()["csr"] == csr
    x = pair.dev(pair.masked_random(8))
    y1 = pair.host(pair.g.apply_A(x))
    y2 = pair.host(pair.g.apply_A(x))
    assert np.array_equal(y1, y2)


def test_longest_timestream_takes_wavefront_rows():
    # nsamp = 2^22: the automatic split is 1024 x 2048 (rows for the
    # one-wavefront pass 2), not 512 x 4096
    n = 2**22
    inp = raster_scan(ncomp=3, ny=32, nx=32, ndet=3, nsamp=n, fsample=400.0, layout="hex",
                      hex_diameter_px=6.0, sigma_scatter=0.1, fknee=(0.5, 2.0), drift_deg=10.0,
                      seed=(77, 22))
    pair = Pair(inp, tod_dtype="f32")
    info = pair.g.info()
    assert (info["fft_m1"], info["fft_m2"]) == (1024, 2048), info
    _check_apply(pair, TOL32_WHITE, label="n=2^22")


def test_invalid_pixel_rejected():
    mm = need_gpu()
    inp = small_raster(ncomp=1, ny=8, nx=8, ndet=2)
    inp.pix[1, 7] = 64  # == npix: out of range
    with pytest.raises(mm.MMError) as ei:
        mm.Scan(inp)
    assert ei.value.status == mm.MM_EINVAL


def test_iqu256_detector_subset():
    """Config 2's recipe and the benchmark's launch geometry (n = 2^20,
    512 x 512, 16 detectors per group, four-step 512 x 1024) on a 16-detector
    draw, small enough for the oracle."""
    inp = make_workload("iqu_256det", ndet=16)
    pair = Pair(inp, tod_dtype="f32")
    info = pair.g.info()
    assert (info["fft_m1"], info["fft_m2"], info["fft_cols"], info["det_group"]) == (512, 1024, 16, 16)
    _check_apply(pair, TOL32_WHITE, label="iqu256-subset")
    sky = (inp.sky * pair.mask.reshape(1, 512, 512)).ravel()
    e = rel(pair.A_gpu(sky), pair.A_oracle(sky))
    print(f"[iqu256 subset] sky rel err = {e:.3e}", flush=True)
    assert e <= TOL32_SKY


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_apply_parity_wide_column_tiles(dt):
    # 32 columns x 512 rows per pass-1/3 block: 16 elements per thread
    n = 2**18
    inp = raster_scan(ncomp=3, ny=32, nx=32, ndet=3, nsamp=n, fsample=100.0, layout="hex",
                      hex_diameter_px=6.0, sigma_scatter=0.1, fknee=(0.5, 2.0), drift_deg=10.0,
                      seed=(77, n // 128))
    pair = Pair(inp, tod_dtype=dt, fft_m1=512, fft_cols=32)
    info = pair.g.info()
    assert (info["fft_m1"], info["fft_cols"]) == (512, 32)
    x = pair.masked_random(1)
    e = rel(pair.A_gpu(x), pair.A_oracle(x))
    print(f"[apply wide tiles {dt}] rel err {e:.3e}", flush=True)
    assert e <= (TOL32_WHITE if dt == "f32" else 2.0**-8)


def test_gather_weight_encodings():
    """Unit-norm weights (stored, or from the boresight model) go into the
    pixel index as 4-byte angles on the float32 and bfloat16 paths; other
    weights keep float32 pairs, the float64 path pairs or (boresight) model
    weights, I only none; every encoding matches the oracle."""
    import dataclasses
    from synth import boresight_only
    inp = raster_scan(ncomp=3, ny=32, nx=32, ndet=4, nsamp=2**15, fsample=100.0,
                      layout="hex", hex_diameter_px=6.0, sigma_scatter=0.1,
                      fknee=(0.5, 2.0), drift_deg=10.0, seed=(78, 1))
    scaled = dataclasses.replace(inp, cos2psi=(inp.cos2psi * np.float32(0.95)),
                                 sin2psi=(inp.sin2psi * np.float32(0.95)))
    cases = [("unit f32", inp, "f32", 2, TOL32_WHITE),
             ("unit bf16", inp, "bf16", 2, 4e-3),
             ("efficiency 0.95 f32", scaled, "f32", 0, TOL32_WHITE),
             ("unit f64", inp, "f64", 0, TOL64),
             ("boresight f32", boresight_only(inp), "f32", 2, TOL32_WHITE),
             ("boresight f64", boresight_only(inp), "f64", 1, TOL64)]
    for label, data, dt, code, tol in cases:
        pair = Pair(data, tod_dtype=dt)
        info = pair.g.info()
        assert info["gather_weights"] == code, (label, info)
        e = _check_apply(pair, tol, seed=3, label=f"weights {label}")
        print(f"[gather weights {label}] code {code} rel {e:.2e}", flush=True)
    pair = Pair(raster_scan(ncomp=1, ny=16, nx=16, ndet=3, nsamp=2**15, fsample=100.0,
                            seed=(78, 2)), tod_dtype="f32")
    assert pair.g.info()["gather_weights"] == -1
