"""Pass 1's chunk-coded pointing against the uncoded form and the oracle.

With stored I,Q,U pointing whose weights are angles (float32 and bfloat16
four-step paths), pass 1 may read each 64-sample chunk of a detector as a
header (the chunk's smallest on-map pixel, a linear angle trend) and one
4-byte word a sample (16-bit pixel offset, 0xFFFF off the map; 16-bit offset
from the trend).  It decodes exactly the stored pixel and angle, so its
A-apply must equal the uncoded one (pointing_code = "off") bit for bit, and
match the oracle at the float32 tolerance.  A scan with any chunk that does
not fit (on-map pixels spread over more than 65534 ids, or angles 2^15 or
more steps of 2 pi / 2^32 off the trend) keeps the uncoded form.
"""

import dataclasses

import numpy as np
import pytest

from gpu_common import Pair, need_gpu, rel, relmax
from synth import make_workload, raster_scan

pytestmark = pytest.mark.gpu

TOL32 = 2e-6
TOLBF16 = 4e-3
CODED, UNCODED = 3, 2   # mm_scan_info.pass1_pointing


def _raster(ny=32, nx=32, ndet=5, n=2**15, seed=(81, 1)):
    return raster_scan(ncomp=3, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=6.0, sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=seed)


def _coded_equals_uncoded(inp, dt, want_code, tol, label, **kw):
    """Builds the scan twice (automatic coding, coding off); checks the
    pointing source each reports, bitwise equality of the two A-applies and
    the oracle parity of the automatic one."""
    mm = need_gpu()
    pair = Pair(inp, tod_dtype=dt, **kw)
    off = mm.Scan(inp, tod_dtype=dt, pointing_code="off", **kw)
    try:
        assert pair.mask.sum() > 0, "no active pixel: the comparison would be vacuous"
        assert pair.g.info()["pass1_pointing"] == want_code, (label, pair.g.info())
        assert off.info()["pass1_pointing"] == UNCODED
        x = pair.masked_random(4)
        xd = pair.dev(x)
        y_auto = pair.host(pair.g.apply_A(xd))
        y_off = pair.host(off.apply_A(xd))
        assert np.array_equal(y_auto, y_off), label
        want = pair.A_oracle(x)
        e, emax = rel(y_auto, want), relmax(y_auto, want)
        print(f"[pointing code {label}] code {want_code} rel {e:.2e} max {emax:.2e}", flush=True)
        assert e <= tol and emax <= tol, (e, emax)
    finally:
        off.close()
        pair.g.close()


@pytest.mark.parametrize("dt,tol", [("f32", TOL32), ("bf16", TOLBF16)])
def test_coded_pointing_is_bitwise_the_stored_one(dt, tol):
    # ragged detector groups (5 detectors in groups of 2)
    _coded_equals_uncoded(_raster(), dt, CODED, tol, f"raster {dt}", det_group=2)


def test_coded_pointing_chunk_edges():
    inp = _raster(ndet=3)
    pix = inp.pix.copy()
    pix[0, 64:128] = -1         # a chunk wholly off the map
    pix[0, 128:191] = -1        # a chunk with one on-map sample, its last (slope 0)
    pix[1, 128:192:3] = -1      # off-map samples inside a chunk
    pix[2, 0] = -1              # the trend through later samples
    pix[2, 63] = -1             # the last sample of the first chunk
    _coded_equals_uncoded(dataclasses.replace(inp, pix=pix), "f32", CODED, TOL32, "chunk edges")


def _one_far_sample(shift):
    """A 16 x 16 raster drawn into a 256 x 512 map (ids up to 15 * 512 + 15),
    with one sample of one chunk moved to (the chunk's smallest on-map id) +
    shift: that chunk then spans exactly `shift` ids."""
    inp = _raster(ny=16, nx=16, ndet=4, seed=(82, 1))
    y, x = np.divmod(inp.pix.astype(np.int64), 16)
    pix = np.where(inp.pix >= 0, y * 512 + x, -1)
    c = next(c for c in range(inp.nsamp // 64) if (pix[1, 64 * c:64 * c + 64] >= 0).sum() >= 2)
    ch = pix[1, 64 * c:64 * c + 64]             # a view: a chunk of detector 1
    on = np.flatnonzero(ch >= 0)
    i_min = on[np.argmin(ch[on])]
    j = on[on != i_min][0]
    lo = ch[i_min]
    ch[j] = lo + shift
    assert ch[ch >= 0].max() - ch[ch >= 0].min() == shift
    return dataclasses.replace(inp, ny=256, nx=512, pix=pix.astype(np.int32), sky=None)


@pytest.mark.parametrize("shift,code", [(65534, CODED), (65535, UNCODED),
                                        (200 * 512 + 300, UNCODED)])
def test_pixel_span_limit(shift, code):
    _coded_equals_uncoded(_one_far_sample(shift), "f32", code, TOL32, f"span {shift}")


def test_jumping_angles_keep_the_stored_form():
    inp = _raster(ndet=3)
    rng = np.random.default_rng(83)
    c2, s2 = inp.cos2psi.copy(), inp.sin2psi.copy()
    th = rng.uniform(0.0, 2 * np.pi, 64)
    # one chunk of one detector, on the map
    c = next(c for c in range(4, inp.nsamp // 64) if (inp.pix[2, 64 * c:64 * c + 64] >= 0).all())
    c2[2, 64 * c:64 * c + 64] = np.cos(th).astype(np.float32)
    s2[2, 64 * c:64 * c + 64] = np.sin(th).astype(np.float32)
    _coded_equals_uncoded(dataclasses.replace(inp, cos2psi=c2, sin2psi=s2), "f32", UNCODED,
                          TOL32, "jumping angles")


def test_bench_geometry_is_coded_and_bitwise():
    # the iqu_256det recipe on 16 detectors: n = 2^20, 512 x 512, four-step
    # 512 x 1024, one group
    inp = make_workload("iqu_256det", ndet=16)
    _coded_equals_uncoded(inp, "f32", CODED, TOL32, "iqu256 subset")
