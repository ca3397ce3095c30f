"""Host logic of the plan autotuner: candidate plans, choice of the fastest,
the per-shape cache (GPU timing replaced by an injected timer)."""

import math
from types import SimpleNamespace

import numpy as np

from paper_1309_7473_amd import autotune as at


def _inputs(ndet=4, nsamp=2**16, nc=3, ny=32, nx=32):
    return SimpleNamespace(ncomp=nc, ny=ny, nx=nx, pix=np.zeros((ndet, nsamp), np.int32))


def test_candidates_follow_the_plan_rules():
    assert at.candidates(2**14, 8) == []          # one-kernel plan: nothing to tune
    c = at.candidates(2**21, 256, "f32")
    logM = 20
    l1s = sorted({int(math.log2(p["fft_m1"])) for p in c})
    assert l1s == list(range(max(2, logM - 12), min(10, logM - 5) + 1))
    assert {p["fft_cols"] for p in c} == {8, 16}
    # automatic group ~512 MiB of pass buffer, half and a quarter of it
    assert {p["det_group"] for p in c} == {64, 32, 16}
    assert {p["det_group"] for p in at.candidates(2**21, 256, "bf16")} == {128, 64, 32}


def test_tune_picks_the_fastest_and_caches(tmp_path):
    inp = _inputs()
    calls = []

    def timer(plan):
        calls.append(plan)
        if plan["fft_cols"] == 8 and plan["fft_m1"] == 16:
            raise RuntimeError("rejected")
        return 1.0 + 0.01 * plan["fft_m1"] - 0.001 * plan["fft_cols"] + 0.0001 * plan["det_group"]

    path = str(tmp_path / "tune.json")
    best = at.tune(inp, cache_path=path, timer=timer)
    ok = [p for p in at.candidates(2**16, 4) if not (p["fft_cols"] == 8 and p["fft_m1"] == 16)]
    want = min(ok, key=lambda p: 1.0 + 0.01 * p["fft_m1"] - 0.001 * p["fft_cols"]
               + 0.0001 * p["det_group"])
    assert best == want
    n = len(calls)
    again = at.tune(inp, cache_path=path, timer=timer)
    assert again == best and len(calls) == n      # served from the cache
    other = at.tune(_inputs(ndet=8), cache_path=path, timer=timer)
    assert len(calls) > n and other                # a new shape is timed


def test_one_kernel_shape_returns_empty(tmp_path):
    assert at.tune(_inputs(nsamp=2**12), cache_path=str(tmp_path / "t.json"),
                   timer=lambda p: 1.0) == {}
