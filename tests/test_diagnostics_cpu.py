"""Host logic of the package's convergence diagnostics against the oracle's
independent implementation, and the A-norm estimate entry point (host only,
no GPU needed)."""

import numpy as np

import oracle
from oracle import diagnostics as D


def test_cv_error_matches_oracle(rng):
    from paper_1309_7473_amd import diagnostics as G
    c_in = np.abs(rng.standard_normal((3, 40)))
    c_in[1, 5] = 0.0
    counts = rng.integers(0, 50, 40).astype(float)
    c_it = c_in * (1 + 0.1 * rng.standard_normal((3, 40)))
    a = G.cv_error(c_it, c_in, counts)
    b = D.spectrum_error(c_it, c_in, counts)
    np.testing.assert_array_equal(np.isnan(a), np.isnan(b))
    np.testing.assert_allclose(a[~np.isnan(a)], b[~np.isnan(b)], rtol=1e-14)


def test_crossing_step_matches_oracle(rng):
    from paper_1309_7473_amd import diagnostics as G
    steps = np.arange(1, 301)
    for _ in range(20):
        e = np.exp(-steps / rng.uniform(20, 200)) * rng.uniform(0.5, 5) \
            * (1 + 0.2 * rng.standard_normal(steps.size))
        for block in (1, 10, 50):
            a = G.crossing_step(steps, e, 0.1, block)
            b = D.convergence_step(steps, e, 0.1, block)
            assert (a is None) == (b is None)
            if a is not None:
                assert abs(a - b) <= 1e-9 * max(1.0, abs(b))


def test_anorm_entry_point_matches_oracle(rng):
    import paper_1309_7473_amd as mm
    a, r = rng.uniform(0.1, 2, 37), rng.uniform(0.01, 3, 37)
    np.testing.assert_allclose(mm.mm_anorm_error_estimate(a, r, 4), oracle.anorm_estimate(a, r, 4),
                               rtol=1e-15)
    assert mm.mm_anorm_error_estimate(a[:2], r[:2], 4).size == 0
