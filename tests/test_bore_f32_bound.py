"""The float32 pixel evaluation that pass 1 uses for boresight pointing on
the float paths decides a pixel only when its error bound keeps p + 1/2 away
from an integer; these CPU checks replay its float32 operations (numpy
float32, each operation rounded once, no fused multiply-add, as the kernel
is compiled) and require every decided pixel to equal the float64
definition, on random scans and on samples placed within 1e-7 .. 1e-3 px of
pixel edges."""

import numpy as np
import pytest

from oracle.boresight import expand_pointing

F = np.float32


def _f32_pixels(bore, det, ny, nx):
    yb, xb, c, s = (np.asarray(v) for v in bore[:4])
    cy64, cx64 = (ny - 1) / 2.0, (nx - 1) / 2.0
    Y = F(yb - cy64)[None, :]
    X = F(xb - cx64)[None, :]
    c, s = F(c)[None, :], F(s)[None, :]
    dy, dx = F(det[0])[:, None], F(det[1])[:, None]
    cy, cx = F(0.5) * F(ny - 1), F(0.5) * F(nx - 1)
    ry = Y + dy
    rx = X + dx
    py = (cy + s * rx) + c * ry
    px = (cx + c * rx) - s * ry
    com = F(4) * (np.abs(rx) + np.abs(ry)) + np.abs(X) + np.abs(Y) + np.abs(dx) + np.abs(dy)
    ty = F(1.1920929e-07) * (cy + com + F(2) * np.abs(py))
    tx = F(1.1920929e-07) * (cx + com + F(2) * np.abs(px))
    vy, vx = py + F(0.5), px + F(0.5)
    fy, fx = np.floor(vy), np.floor(vx)
    dyy = np.minimum(vy - fy, fy + F(1) - vy)
    dxx = np.minimum(vx - fx, fx + F(1) - vx)
    decided = (dyy > ty) & (dxx > tx)
    on = (fy >= 0) & (fy < ny) & (fx >= 0) & (fx < nx)
    pix = np.where(on, fy.astype(np.int64) * nx + fx.astype(np.int64), -1)
    for a in (ry, rx, py, px, ty, tx, vy, vx, dyy, dxx):
        assert a.dtype == np.float32
    return np.where(decided, pix, -2)


def _bore(yb, xb, phi):
    return np.stack([yb, xb, np.cos(phi), np.sin(phi), np.cos(2 * phi), np.sin(2 * phi)])


@pytest.mark.parametrize("n_map", [64, 512, 4096])
def test_decided_pixels_equal_the_float64_definition(n_map, rng):
    nsamp, ndet = 200_000, 8
    yb = rng.uniform(-40, n_map + 40, nsamp)
    xb = rng.uniform(-40, n_map + 40, nsamp)
    phi = rng.uniform(-0.2, 0.2, nsamp)
    det = np.stack([rng.uniform(-30, 30, ndet), rng.uniform(-30, 30, ndet),
                    np.ones(ndet), np.zeros(ndet)])
    bore = _bore(yb, xb, phi)
    p64, _, _ = expand_pointing(bore, det, n_map, n_map)
    p32 = _f32_pixels(bore, det, n_map, n_map)
    dec = p32 != -2
    assert np.array_equal(p32[dec], p64[dec])
    assert dec.mean() > 0.99          # the float64 fallback stays rare


@pytest.mark.parametrize("eps", [1e-7, 1e-6, 1e-5, 1e-4, 1e-3])
def test_samples_at_pixel_edges(eps, rng):
    """Boresights placed so that the unturned detector sits eps from a pixel
    edge (either side) on one axis: the float32 path must defer or agree."""
    n_map, nsamp = 512, 100_000
    k = rng.integers(0, n_map, nsamp).astype(np.float64)
    side = rng.choice([-1.0, 1.0], nsamp)
    yb = k - 0.5 + side * eps
    xb = rng.uniform(0, n_map - 1, nsamp)
    phi = rng.choice([0.0, 1e-9, -1e-9, 0.05], nsamp)
    det = np.stack([np.array([0.0, 0.25, -7.5]), np.array([0.0, 3.0, 0.125]),
                    np.ones(3), np.zeros(3)])
    bore = _bore(yb, xb, phi)
    p64, _, _ = expand_pointing(bore, det, n_map, n_map)
    p32 = _f32_pixels(bore, det, n_map, n_map)
    dec = p32 != -2
    assert np.array_equal(p32[dec], p64[dec])
    if eps <= 1e-5:
        assert (~dec[0][phi == 0.0]).all()   # within the bound: always deferred
