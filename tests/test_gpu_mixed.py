"""GPU parity of the filter for timestream lengths that are not powers of
two, n = 2^a 3^b 5^c (mixed-radix LDS FFT on the one-kernel path), against
the oracle, whose N^-1 is numpy's FFT of any length (pinned against a dense
DFT circulant at such lengths).  Tolerances as for powers of two: float64
1e-12, float32 2e-6 (white map)."""

import numpy as np
import pytest

import oracle
from gpu_common import Pair, rel
from synth import raster_scan

pytestmark = pytest.mark.gpu

CASES = [
    # label, ncomp, ny, nx, ndet, nsamp, dtype, acc
    ("n30-odd-M-f64", 1, 8, 8, 3, 30, "f64", "f64"),
    ("n96-f64-IQU", 3, 8, 8, 6, 96, "f64", "f64"),
    ("n1000-f64-IQU", 3, 16, 16, 5, 1000, "f64", "f64"),
    ("n1000-f32-IQU", 3, 16, 16, 5, 1000, "f32", "f64"),
    ("n6144-f32-IQU", 3, 16, 16, 4, 6144, "f32", "f64"),
    ("n12000-f64-I", 1, 32, 32, 3, 12000, "f64", "f64"),
    ("n13122-3pow8-f32-IQU", 3, 32, 32, 6, 2 * 3**8, "f32", "f64"),
    ("n16000-f32-IQU-gather", 3, 32, 32, 4, 16000, "f32", "f32x2"),
    ("n15000-bf16-IQU", 3, 32, 32, 4, 15000, "bf16", "f64"),
    # four-step: rows 2^l, the factors 3 and 5 in the columns
    ("fourstep-3x2^14-f32-IQU", 3, 32, 32, 4, 3 * 2**14, "f32", "f64"),
    ("fourstep-15x2^14-f64-IQU", 3, 32, 32, 5, 15 * 2**14, "f64", "f64"),
    ("fourstep-2x3^5x2^12-f32-I", 1, 32, 32, 2, 2 * 3**5 * 2**12, "f32", "f64"),
    ("fourstep-2x5^4x2^10-f32-IQU", 3, 32, 32, 3, 2 * 5**4 * 2**10, "f32", "f64"),
    ("fourstep-45x2^12-bf16-IQU", 3, 32, 32, 4, 45 * 2**12, "bf16", "f64"),
    ("fourstep-75x2^10-f32x2-IQU", 3, 32, 32, 4, 75 * 2**10, "f32", "f32x2"),
]
TOL = {"f64": 1e-12, "f32": 2e-6, "bf16": 4e-3}


def _inputs(nc, ny, nx, ndet, n):
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(93, n))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mixed_length_apply_and_rhs(case):
    label, nc, ny, nx, ndet, n, dt, acc = case
    pair = Pair(_inputs(nc, ny, nx, ndet, n), tod_dtype=dt, acc=acc)
    info = pair.g.info()
    print(f"[mixed {label}] {info}", flush=True)
    assert info["single_pass"] == (0 if label.startswith("fourstep") else 1)
    assert pair.mask.sum() > 0
    x = pair.masked_random(1)
    e = rel(pair.A_gpu(x), pair.A_oracle(x))
    tod = np.random.default_rng(n).standard_normal((ndet, n))
    b_want = oracle.rhs(pair.o, tod, pair.mask)
    b_got = pair.host(pair.g.rhs(pair.torch.from_numpy(tod)))
    eb = rel(b_got, b_want)
    print(f"[mixed {label}] A {e:.2e} rhs {eb:.2e}", flush=True)
    assert e <= TOL[dt] and eb <= 2 * TOL[dt]


def test_mixed_length_pcg():
    n = 2 * 3 * 5 * 2**7   # 3840
    pair = Pair(_inputs(3, 16, 16, 6, n), tod_dtype="f64")
    m = np.random.default_rng(2).standard_normal((3, 256)) * pair.mask
    b = pair.A_oracle(m.ravel())
    ro = oracle.pcg(pair.A_oracle, oracle.BinnedPrecon(pair.B, pair.mask), b, tol=1e-9,
                    maxiter=2000)
    rg = pair.g.pcg("binned", pair.dev(b), tol=1e-9, maxiter=2000)
    x = pair.host(rg["x"])
    tr = np.linalg.norm(b - pair.A_oracle(x)) / np.linalg.norm(b)
    print(f"[mixed pcg n={n}] oracle {ro.iters} gpu {rg['iters']} true {tr:.2e}", flush=True)
    assert rg["converged"] and abs(rg["iters"] - ro.iters) <= 1 and tr <= 1e-8


def test_mixed_length_fourstep_pcg():
    n = 2 * 3 * 5 * 2**12   # 122880: four-step, columns of 60
    pair = Pair(_inputs(3, 32, 32, 6, n), tod_dtype="f64")
    assert pair.g.info()["single_pass"] == 0 and pair.mask.sum() > 500
    m = np.random.default_rng(4).standard_normal((3, 1024)) * pair.mask
    b = pair.A_oracle(m.ravel())
    ro = oracle.pcg(pair.A_oracle, oracle.BinnedPrecon(pair.B, pair.mask), b, tol=1e-9,
                    maxiter=2000)
    rg = pair.g.pcg("binned", pair.dev(b), tol=1e-9, maxiter=2000)
    x = pair.host(rg["x"])
    tr = np.linalg.norm(b - pair.A_oracle(x)) / np.linalg.norm(b)
    print(f"[mixed four-step pcg n={n}] oracle {ro.iters} gpu {rg['iters']} true {tr:.2e}",
          flush=True)
    assert rg["converged"] and abs(rg["iters"] - ro.iters) <= 1 and tr <= 1e-8
