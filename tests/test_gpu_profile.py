"""The library's per-stage timing: every stage while enabled, only the
selected stages after mm_profile_stages, nothing inside a captured graph."""

import pytest

from conftest import small_raster
from gpu_common import Pair

pytestmark = pytest.mark.gpu


def test_profile_stages_select_what_is_timed():
    import paper_1309_7473_amd as mm
    inp = small_raster(ncomp=3, ny=32, nx=32, ndet=4, sweeps=256)   # 2^15 samples: four-step
    pair = Pair(inp, tod_dtype="f32")
    h = pair.g.handle
    x = pair.dev(pair.masked_random(0))
    mm.mm_profile_enable(h, True)
    mm.mm_profile_read(h)
    pair.g.apply_A(x)
    allp = mm.mm_profile_read(h)
    for k in ("pass1", "pass2", "pass3", "reduce", "apply_A"):
        assert allp[k][1] >= 1, (k, allp)
    mm.mm_profile_stages(h, ["reduce"])
    pair.g.apply_A(x)
    one = mm.mm_profile_read(h)
    assert set(k for k, v in one.items() if v[1] > 0) == {"reduce"}, one
    assert one["reduce"][1] == allp["reduce"][1] and one["reduce"][0] > 0
    mm.mm_profile_stages(h, None)
    pair.g.apply_A(x)
    again = mm.mm_profile_read(h)
    assert again["pass1"][1] == allp["pass1"][1]
    mm.mm_profile_enable(h, False)
