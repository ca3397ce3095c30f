"""Graph-replayed PCG iterations and batched solves of several scans.

A captured iteration runs the same kernels in the same order as the eager
loop, and every kernel of the gather path has a fixed summation order, so a
graph solve must reproduce the eager solve bit for bit: each replay is
checked implicitly, since one wrong replay would change every later iterate.
The host polls the device scalars (a synchronisation) between replays.  A
batch interleaves independent solves on forked streams and must return what
each scan's own solve returns."""

import numpy as np
import pytest

from gpu_common import Pair, rel
from synth import batch_scan_spec, make_workload, raster_scan

pytestmark = pytest.mark.gpu


def _scan(nc, ny, nx, ndet, n, seed=77, white=False):
    sweeps = max(1, n // (4 * nx))
    return raster_scan(ncomp=nc, ny=ny, nx=nx, ndet=ndet, nsamp=n, fsample=100.0,
                       layout="hex", hex_diameter_px=min(6.0, ny / 3), sigma_scatter=0.1,
                       fknee=(0.5, 2.0), drift_deg=10.0, seed=(seed, sweeps), white=white)


def _rhs(pair, seed=3):
    sky = pair.masked_random(seed)
    return pair.A_oracle(sky)


@pytest.mark.parametrize("precon", ["binned", "circulant"])
@pytest.mark.parametrize("every", [1, 5])
def test_graph_solve_reproduces_eager_solve(precon, every):
    inp = _scan(3, 32, 32, 3, 2**15)
    pair = Pair(inp, tod_dtype="f32")
    assert pair.g.info()["csr"] == 2
    if precon == "circulant":
        pair.g.build_precon("circulant", sigma=3.0)
    else:
        pair.g.build_precon("binned")
    b = pair.dev(_rhs(pair))
    eager = pair.g.pcg(precon, b, tol=1e-6, maxiter=400, check_every=every)
    graph = pair.g.pcg(precon, b, tol=1e-6, maxiter=400, check_every=every, graph=True)
    xe, xg = pair.host(eager["x"]), pair.host(graph["x"])
    print(f"[graph {precon} every={every}] iters eager {eager['iters']} graph {graph['iters']}",
          flush=True)
    assert eager["converged"] and graph["converged"]
    assert graph["iters"] == eager["iters"]
    np.testing.assert_array_equal(graph["history"], eager["history"])
    np.testing.assert_array_equal(xg, xe)
    # and the answer is right
    assert rel(pair.A_oracle(xg), pair.host(b)) <= 1.5e-6


def test_graph_solve_on_the_atomic_path_agrees():
    # float64 atomics add in varying order: compare to rounding, not bits
    inp = _scan(3, 16, 16, 5, 2**12)
    pair = Pair(inp, tod_dtype="f64")
    assert pair.g.info()["csr"] == 0
    pair.g.build_precon("binned")
    b = pair.dev(_rhs(pair))
    eager = pair.g.pcg("binned", b, tol=1e-8, maxiter=400)
    graph = pair.g.pcg("binned", b, tol=1e-8, maxiter=400, graph=True, check_every=4)
    assert abs(graph["iters"] - eager["iters"]) <= 1
    assert rel(pair.host(graph["x"]), pair.host(eager["x"])) <= 1e-9


def _batch_pairs():
    return [
        Pair(_scan(1, 16, 16, 4, 2**12, seed=1), tod_dtype="f32", acc="f32x2"),
        Pair(_scan(3, 16, 16, 5, 2**13, seed=2), tod_dtype="f64", acc="f32x2"),
        Pair(_scan(3, 32, 32, 3, 2**15, seed=3), tod_dtype="f32"),
        Pair(_scan(3, 32, 32, 4, 2**16, seed=4), tod_dtype="f64"),
    ]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single_solves(graph):
    import paper_1309_7473_amd as mm
    pairs = _batch_pairs()
    bs = []
    for k, p in enumerate(pairs):
        assert p.g.info()["csr"] >= 1
        p.g.build_precon("binned")
        bs.append(p.dev(_rhs(p, seed=10 + k)))
    singles = [p.g.pcg("binned", b, tol=1e-6, maxiter=500) for p, b in zip(pairs, bs)]
    out = mm.pcg_batch([p.g for p in pairs], "binned", bs, tol=1e-6, maxiter=500,
                       check_every=4, graph=graph)
    for p, b, s1, r in zip(pairs, bs, singles, out):
        print(f"[batch graph={graph}] iters single {s1['iters']} batch {r['iters']}", flush=True)
        assert s1["iters"] > 5   # a real solve, not an empty mask
        assert r["status"] == mm.MM_OK and r["converged"]
        assert r["iters"] == s1["iters"]
        np.testing.assert_array_equal(p.host(r["x"]), p.host(s1["x"]))
        assert rel(p.A_oracle(p.host(r["x"])), p.host(b)) <= 1.5e-6


def test_batch_reports_each_status_and_rejects_duplicates():
    import paper_1309_7473_amd as mm
    pairs = _batch_pairs()[:2]
    bs = []
    for k, p in enumerate(pairs):
        p.g.build_precon("binned")
        bs.append(p.dev(_rhs(p, seed=20 + k)))
    out = mm.pcg_batch([p.g for p in pairs], "binned", bs, tol=1e-12, maxiter=3)
    assert all(r["status"] == mm.MM_ENOCONV and r["iters"] == 3 for r in out)
    with pytest.raises(mm.MMError):
        mm.pcg_batch([pairs[0].g, pairs[0].g], "binned", [bs[0], bs[0]])


def test_batch_of_batch64_shaped_scans():
    # four scans of the batched workload's recipe, shrunk so the oracle can
    # check each answer: detectors / 16, samples / 16, map side / 4 (the
    # samples per pixel and the row advance per sweep stay as drawn)
    import paper_1309_7473_amd as mm
    pairs = []
    for sid in range(4):
        sp = batch_scan_spec(sid)
        inp = make_workload("batch_64scans", sid, ndet=max(4, sp["ndet"] // 16), nsamp=sp["nsamp"] // 16,
                          ny=sp["ny"] // 4, nx=sp["nx"] // 4,
                          hex_diameter_px=sp["hex_diameter_px"] / 4)
        pairs.append(Pair(inp, tod_dtype="f32"))
    bs = []
    for k, p in enumerate(pairs):
        p.g.build_precon("binned")
        bs.append(p.dev(_rhs(p, seed=30 + k)))
    out = mm.pcg_batch([p.g for p in pairs], "binned", bs, tol=1e-6, maxiter=5000,
                       check_every=8, graph=True)
    for p, b, r in zip(pairs, bs, out):
        x = p.host(r["x"])
        t = rel(p.A_oracle(x), p.host(b))
        print(f"[batch_64scans] {p.inp.ndet} det x {p.inp.nsamp} on {p.inp.ny}^2: "
              f"iters {r['iters']} true resid {t:.2e}", flush=True)
        assert r["converged"] and t <= 2e-6
