"""Precision modes against the oracle: bfloat16 storage of the timestream and
of the pass buffers between the FFT kernels (float32 math), and compensated
float32 pairs in place of float64 for the pixel accumulation of P^T and the
PCG inner products.

Tolerances.  bfloat16 keeps 8 significant bits, unit roundoff U = 2^-8.  The
four-step pipeline rounds three times (after pass 1, pass 2 and pass 3), each
at most U relative per element; the FFTs are unitary up to scale, so each
stage adds at most U norm-wise, about U/sqrt(3) in rms for uncorrelated
rounding, and the three stages add in quadrature to about U.  The filter
re-weights frequencies, which can raise the error of a smooth map's output
relative to the output; A-apply is held to U and the right-hand side (white
timestream, all three stages carry its full power) to 2U.  The compensated
pairs carry about 48 bits, so they must agree with the float64 accumulation
to 1e-13 relative and with the oracle to the tolerance of the timestream
arithmetic."""

import numpy as np
import pytest

from gpu_common import Pair, rel
from synth import raster_scan
from test_gpu_apply import make_sky, TOL64, TOL32_WHITE, TOL32_SKY

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8


def _scan(nc, ny, nx, ndet, n, seed=77):
    sweeps = max(1, n // (4 * nx))
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(seed, sweeps))


def _maps(pair):
    nc, ny, nx = pair.inp.ncomp, pair.inp.ny, pair.inp.nx
    x = pair.masked_random(1)
    sky = (make_sky(nc, ny, nx) * pair.mask.reshape(1, ny, nx)).ravel()
    return x, sky


def _rhs_pair(pair, round_bf16):
    import torch
    inp = pair.inp
    tod = np.random.default_rng(5).standard_normal((inp.ndet, inp.nsamp)).astype(np.float32)
    if round_bf16:  # the caller hands bfloat16 data; both sides see the same values
        tod = torch.from_numpy(tod).to(torch.bfloat16).float().numpy()
    import oracle
    want = oracle.rhs(pair.o, tod.astype(np.float64), pair.mask)
    got = pair.host(pair.g.rhs(torch.from_numpy(tod).cuda()))
    return rel(got, want)


BF16_CASES = [
    # (label, ncomp, ny, nx, ndet, nsamp, acc)
    ("fourstep-IQU", 3, 32, 32, 3, 2**15, "f64"),
    ("fourstep-IQU-m2=1024", 3, 32, 32, 4, 2**16, "f64"),
    ("fourstep-I-f32x2", 1, 32, 32, 3, 2**15, "f32x2"),
    ("onekernel-gather-IQU", 3, 16, 16, 5, 2**12, "f32x2"),
    # rows of 2048 bins: two wavefronts a row in pass 2
    ("fourstep-IQU-m2=2048", 3, 32, 32, 3, 2**15, "f64", 8),
]


@pytest.mark.parametrize("case", BF16_CASES, ids=[c[0] for c in BF16_CASES])
def test_bf16_storage_parity(case):
    label, nc, ny, nx, ndet, n, acc = case[:7]
    m1 = case[7] if len(case) > 7 else 0
    inp = _scan(nc, ny, nx, ndet, n)
    pair = Pair(inp, tod_dtype="bf16", acc=acc, fft_m1=m1)
    ref = Pair(inp, tod_dtype="f32", acc=acc, fft_m1=m1)
    if m1:
        assert pair.g.info()["fft_m1"] == m1
    x, sky = _maps(pair)
    for name, v in (("random", x), ("sky", sky)):
        want = pair.A_oracle(v)
        e = rel(pair.A_gpu(v), want)
        e32 = rel(ref.A_gpu(v), want)
        print(f"[bf16 {label}] A {name}: rel err {e:.3e} (f32 storage {e32:.3e})", flush=True)
        assert e <= U_BF16, e
        # the rounding is really there: far above the float32 path's error
        assert e > 20 * e32, (e, e32)
    eb = _rhs_pair(pair, round_bf16=True)
    print(f"[bf16 {label}] rhs rel err {eb:.3e}", flush=True)
    assert eb <= 2 * U_BF16, eb


def test_bf16_one_kernel_scatter_keeps_float_buffers():
    # without a pass buffer (one-kernel filter, atomic scatter) bfloat16 only
    # changes what rhs reads: A-apply equals float32 storage up to the order
    # of the float64 atomic additions
    inp = _scan(3, 16, 16, 5, 2**12)
    pair = Pair(inp, tod_dtype="bf16")
    ref = Pair(inp, tod_dtype="f32")
    assert pair.g.info()["single_pass"] == 1 and pair.g.info()["csr"] == 0
    x, _ = _maps(pair)
    assert rel(pair.A_gpu(x), ref.A_gpu(x)) <= 1e-14
    assert _rhs_pair(pair, round_bf16=True) <= TOL32_WHITE


F32X2_CASES = [
    # (label, ncomp, ny, nx, ndet, nsamp, tod dtype)
    ("fourstep-f32", 3, 32, 32, 3, 2**15, "f32"),
    ("fourstep-f64", 3, 32, 32, 4, 2**16, "f64"),
    ("onekernel-f64", 3, 16, 16, 5, 2**12, "f64"),
    ("onekernel-I-f32", 1, 16, 16, 5, 2**12, "f32"),
]


@pytest.mark.parametrize("case", F32X2_CASES, ids=[c[0] for c in F32X2_CASES])
def test_compensated_accumulation_parity(case):
    label, nc, ny, nx, ndet, n, dt = case
    inp = _scan(nc, ny, nx, ndet, n)
    pair = Pair(inp, tod_dtype=dt, acc="f32x2")
    ref = Pair(inp, tod_dtype=dt, acc="f64")
    assert pair.g.info()["csr"] >= 1
    x, sky = _maps(pair)
    for name, v, tol32 in (("random", x, TOL32_WHITE), ("sky", sky, TOL32_SKY)):
        want = pair.A_oracle(v)
        got = pair.A_gpu(v)
        e = rel(got, want)
        d = rel(got, ref.A_gpu(v))
        print(f"[f32x2 {label}] A {name}: vs oracle {e:.3e}, vs float64 accumulation {d:.3e}",
              flush=True)
        assert e <= (TOL64 if dt == "f64" else tol32), e
        assert d <= 1e-13, d
    e = _rhs_pair(pair, round_bf16=False)
    assert e <= (TOL64 if dt == "f64" else TOL32_WHITE), e


def test_compensated_pcg_matches_float64():
    inp = _scan(3, 32, 32, 4, 2**16)
    a = Pair(inp, tod_dtype="f64", acc="f64")
    c = Pair(inp, tod_dtype="f64", acc="f32x2")
    _, sky = _maps(a)
    b = a.A_oracle(sky)
    out = []
    for p in (a, c):
        p.g.build_precon("binned")
        res = p.g.pcg("binned", p.dev(b), tol=1e-6, maxiter=500)
        x = p.host(res["x"])
        out.append((res["iters"], res["converged"], x, rel(p.A_oracle(x), b)))
    (ia, ca, xa, ta), (ic, cc, xc, tc) = out
    print(f"[pcg f32x2] iters {ic} (float64 {ia}); true resid {tc:.3e} ({ta:.3e}); "
          f"map diff {rel(xc, xa):.3e}", flush=True)
    assert ca and cc
    assert abs(ic - ia) <= 1
    assert tc <= 1.01e-6
    assert rel(xc, xa) <= 1e-8


def test_bf16_pcg_reports_its_map_error():
    # the recursion converges; the true residual and the map error show what
    # bfloat16 storage costs (per Stokes component)
    inp = _scan(3, 32, 32, 4, 2**16)
    p = Pair(inp, tod_dtype="bf16")
    _, sky = _maps(p)
    b = p.A_oracle(sky)
    p.g.build_precon("binned")
    res = p.g.pcg("binned", p.dev(b), tol=1e-6, maxiter=500)
    x = p.host(res["x"])
    true = rel(p.A_oracle(x), b)
    errs = [rel(x.reshape(3, -1)[k], sky.reshape(3, -1)[k]) for k in range(3)]
    print(f"[pcg bf16] iters {res['iters']} true resid {true:.3e} "
          f"map err I,Q,U {errs[0]:.3e} {errs[1]:.3e} {errs[2]:.3e}", flush=True)
    assert res["converged"]
    assert true <= U_BF16
    assert all(np.isfinite(errs)) and max(errs) < 1.0
