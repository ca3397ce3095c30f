"""The autotuner on the GPU: it times real plans, its choice builds a scan
whose A-apply matches the oracle, and the scan runs the chosen plan."""

import pytest

from gpu_common import Pair, rel
from synth import raster_scan
from test_gpu_apply import TOL32_WHITE

pytestmark = pytest.mark.gpu


def test_autotuned_plan_is_used_and_correct(tmp_path):
    from paper_1309_7473_amd import autotune
    inp = raster_scan(ncomp=3, ny=32, nx=32, ndet=4, nsamp=2**16, fsample=100.0, layout="hex",
                      hex_diameter_px=6.0, sigma_scatter=0.1, fknee=(0.5, 2.0), drift_deg=10.0,
                      seed=(77, 128))
    best = autotune.tune(inp, tod_dtype="f32", reps=3, cache_path=str(tmp_path / "t.json"),
                         verbose=True)
    assert best in autotune.candidates(inp.nsamp, inp.ndet, "f32")
    pair = Pair(inp, tod_dtype="f32", **best)
    info = pair.g.info()
    assert (info["fft_m1"], info["fft_cols"], info["det_group"]) == \
        (best["fft_m1"], best["fft_cols"], best["det_group"])
    x = pair.masked_random(1)
    e = rel(pair.A_gpu(x), pair.A_oracle(x))
    print(f"[autotune] {best}: rel err {e:.2e}", flush=True)
    assert e <= TOL32_WHITE
