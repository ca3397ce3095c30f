"""FP64 oracle of the tiled (position-dependent) constant-correlation
preconditioner that the Summary section proposes (test infrastructure only).

The section only sketches it: cover the map with overlapping tiles, apply the
constant-correlation preconditioner to each tile, merge.  Readings:

* Tiles are T x T (T a power of two dividing into the map at stride T/2):
  origins 0, T/2, 2 T/2, ..., n - T along each axis.
* Merge by a partition of unity: along an axis a tile's weight is
  sin^2(pi (u + 1/2) / T) at offset u inside the tile, except that the outer
  half of the first and the last tile weigh 1 (no neighbour there) and a
  tile spanning the whole axis weighs 1.  Two overlapping tiles' weights sum
  to one (sin^2 + cos^2); the 2-D weight is the product W_t.
  M_T r = Sigma^-1 [ sum_t sqrt(W_t) F_t^-1 K_t^-1 F_t sqrt(W_t) ] Sigma^-T r,
  a sum of symmetric positive semi-definite terms that is positive definite
  where the tiles' M_t are.
* Tile t's reference pixel is the active pixel of the tile nearest its
  centre (o + T/2 on each axis), smallest id on ties; a tile without active
  pixels contributes nothing.
* Probing: each tile's constant-correlation kernel comes from the rows of A
  at that tile's own reference pixel (eq. 6): ncomp A-applies per tile, one
  unit vector at a time, exactly as for M_C.
* K_t is built exactly like M_C's K but on the tile's own periodic T x T
  displacement grid: q_t(d) = Sigma_r^-T C_(r+d) Sigma_(r+d)^-1 with r + d
  taken modulo the map, zero for inactive pixels, Gaussian taper on the
  minimal-image displacement, symmetrised, conj FFT2, Hermitian eigenvalue
  floor relative to the tile's largest eigenvalue (the same floor as M_C's,
  applied to the tile's own Q_t).
With T equal to the map size there is one tile of weight one and M_T = M_C.
"""

import numpy as np

from .operators import apply_A
from .precon import CirculantPrecon, sym_sqrt, gaussian_taper


def tile_origins(n, T):
    if T > n or n % (T // 2) != 0 or T & (T - 1):
        raise ValueError("tile size must be a power of two <= n with n a multiple of T/2")
    return list(range(0, n - T + 1, T // 2))


def axis_weights(n, T):
    """Per tile along one axis: the weight of offsets u = 0..T-1."""
    orig = tile_origins(n, T)
    u = np.arange(T)
    w = []
    for i, o in enumerate(orig):
        if len(orig) == 1:
            w.append(np.ones(T))
            continue
        s = np.sin(np.pi * (u + 0.5) / T) ** 2
        if i == 0:
            s = np.where(u < T // 2, 1.0, s)
        if i == len(orig) - 1:
            s = np.where(u >= T // 2, 1.0, s)
        w.append(s)
    return orig, w


def tile_reference(mask, nx, oy, ox, T):
    cy, cx = oy + T // 2, ox + T // 2
    best, bd = -1, None
    for y in range(oy, oy + T):
        for x in range(ox, ox + T):
            p = y * nx + x
            if not mask[p]:
                continue
            d = (y - cy) ** 2 + (x - cx) ** 2
            if bd is None or d < bd or (d == bd and p < best):
                best, bd = p, d
    return best


class TiledCirculantPrecon:
    def __init__(self, scan, mask, B, tile, sigma_taper=None, eig_floor_rel=1e-6):
        nc, ny, nx = scan.ncomp, scan.ny, scan.nx
        npix = ny * nx
        T = int(tile)
        self.nc, self.ny, self.nx, self.npix, self.T = nc, ny, nx, npix, T
        self.mask = mask
        self.Siginv = np.zeros((npix, nc, nc))
        _, Si = sym_sqrt(B[mask])
        self.Siginv[mask] = Si
        oys, wys = axis_weights(ny, T)
        oxs, wxs = axis_weights(nx, T)
        self.tiles = []
        for iy, oy in enumerate(oys):
            for ix, ox in enumerate(oxs):
                W = np.outer(wys[iy], wxs[ix])
                ref = tile_reference(mask, nx, oy, ox, T)
                self.tiles.append(dict(iy=iy, ix=ix, oy=oy, ox=ox, W=W, ref=ref, Kinv=None))
        # the rows of A at every tile's own reference pixel (eq. 6)
        C = {}
        for t in self.tiles:
            if t["ref"] < 0:
                continue
            C[id(t)] = np.zeros((nc, nc, npix))
            for g in range(nc):
                e = np.zeros((nc, npix))
                e[g, t["ref"]] = 1.0
                C[id(t)][g] = apply_A(scan, e, mask).reshape(nc, npix)
        taper = gaussian_taper(T, T, sigma_taper)
        d = np.arange(T)
        dmi = np.where(d > T // 2, d - T, d)              # minimal image on the tile
        for t in self.tiles:
            if t["ref"] < 0:
                continue
            r = t["ref"]
            ry, rx = divmod(r, nx)
            jy = (ry + dmi[:, None]) % ny
            jx = (rx + dmi[None, :]) % nx
            j = (jy * nx + jx)                             # (T, T) pixel of r + d
            Cj = np.transpose(C[id(t)], (2, 0, 1))[j]       # (T, T, g, b)
            q = np.einsum("ga,yxgb,yxbc->yxac", self.Siginv[r], Cj, self.Siginv[j])
            q[~mask[j]] = 0.0
            t["q_raw"] = q.copy()
            q *= taper[:, :, None, None]
            qm = q[(-d) % T][:, (-d) % T]
            q = 0.5 * (q + np.transpose(qm, (0, 1, 3, 2)))
            t["q"] = q
            K = np.conj(np.fft.fft2(q, axes=(0, 1)))
            t["Kinv"], _, t["n_floored"] = CirculantPrecon.floored_inverse(K, eig_floor_rel)

    def __call__(self, rvec):
        nc, ny, nx, npix, T = self.nc, self.ny, self.nx, self.npix, self.T
        rp = np.asarray(rvec, dtype=np.float64).reshape(nc, npix).T
        u = np.einsum("pba,pb->pa", self.Siginv, rp).T.reshape(nc, ny, nx)   # Sigma^-T r
        acc = np.zeros((nc, ny, nx))
        for t in self.tiles:
            if t["Kinv"] is None:
                continue
            sw = np.sqrt(t["W"])
            sl = (slice(None), slice(t["oy"], t["oy"] + T), slice(t["ox"], t["ox"] + T))
            uh = np.fft.fft2(u[sl] * sw, axes=(1, 2))
            vh = np.einsum("yxab,byx->ayx", t["Kinv"], uh)
            acc[sl] += np.fft.ifft2(vh, axes=(1, 2)).real * sw
        z = np.einsum("pab,pb->pa", self.Siginv, acc.reshape(nc, npix).T)
        z[~self.mask] = 0.0
        return z.T.reshape(-1)
