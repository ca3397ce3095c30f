"""Seeded scanning patterns and the nearest-pixel pointing they induce.

Conventions shared by every consumer:

* Maps are [ncomp][ny][nx], x fastest; pixel id p = y * nx + x.
* Pixel centres sit at integer coordinates; a sample at (y, x) falls in pixel
  (floor(y + 1/2), floor(x + 1/2)), and off-map samples get pix = -1.
* The timestream and the pointing arrays are detector-major [ndet][nsamp].
* A detector responds to T + cos(2 psi) Q + sin(2 psi) U; the weights are
  computed in float64 and stored as float32.

The raster is a constant-speed boustrophedon sweep along x covering all
columns at 0.25 px/sample (4 * nx samples per sweep), advancing in y between
sweeps so that the sweeps cover the rows evenly.  An optional slow linear
drift phi(t) rotates the whole pattern (boresight track and focal plane) about
the map centre, and adds phi(t) to every detector angle.
"""

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class ScanInputs:
    ncomp: int
    ny: int
    nx: int
    ndet: int
    nsamp: int
    fsample: float
    pix: np.ndarray                  # int32 [ndet][nsamp], -1 = off-map
    cos2psi: np.ndarray | None       # float32 [ndet][nsamp] (None if ncomp == 1)
    sin2psi: np.ndarray | None       # float32 [ndet][nsamp]
    inv_noise: np.ndarray            # float32 [ndet][nsamp//2 + 1]
    spectrum: np.ndarray             # float64 [ndet][nsamp//2 + 1] (for noise draws)
    sky: np.ndarray | None = None    # float64 [ncomp][ny][nx]
    meta: dict = field(default_factory=dict)
    # inter-detector correlated part of N^-1 (None: detectors independent):
    # real-FFT bins edges[b] <= k < edges[b+1] share V[b] (float32 [ndet][rank])
    corr_edges: np.ndarray | None = None   # int32 [nbins + 1]
    corr_V: np.ndarray | None = None       # float32 [nbins][ndet][rank]
    # the pointing model the per-sample pointing was expanded from (raster
    # scans): boresight float64 [6][nsamp] = y_b, x_b (pixel coordinates),
    # cos phi, sin phi, cos 2phi, sin 2phi of the scan-angle drift about the map
    # centre; detectors float64 [4][ndet] = dy, dx (offsets before rotation),
    # cos 2psi, sin 2psi.  pix/cos2psi/sin2psi may be None when these are given.
    bore: np.ndarray | None = None
    det_off: np.ndarray | None = None

    @property
    def npix(self):
        return self.ny * self.nx

    @property
    def nsamples(self):
        return self.ndet * self.nsamp


def hex_focal_plane(ndet, diameter_px, rotation=0.0):
    """Offsets (dy, dx) of the ndet hexagonal-lattice points nearest the centre,
    scaled so that the outermost detector sits at diameter_px / 2, and rotated
    by `rotation` radians.  Returns two float64 arrays of shape (ndet,)."""
    if ndet == 1:
        return np.zeros(1), np.zeros(1)
    r = int(math.ceil(math.sqrt(ndet))) + 2
    pts = []
    for j in range(-r, r + 1):
        for i in range(-r, r + 1):
            x = i + 0.5 * j
            y = j * math.sqrt(3.0) / 2.0
            pts.append((round(x * x + y * y, 9), math.atan2(y, x), x, y))
    pts.sort()
    sel = np.array([(p[2], p[3]) for p in pts[:ndet]])
    x, y = sel[:, 0], sel[:, 1]
    x = x - x.mean()
    y = y - y.mean()
    rmax = np.sqrt(x * x + y * y).max()
    s = (diameter_px / 2.0) / rmax if rmax > 0 else 1.0
    c, sn = math.cos(rotation), math.sin(rotation)
    dx = s * (c * x - sn * y)
    dy = s * (sn * x + c * y)
    return dy, dx


def raster_boresight(nsamp, ny, nx, samples_per_px=4):
    """Boresight track (y, x) in pixel coordinates, float64 arrays (nsamp,)."""
    lsw = samples_per_px * nx
    t = np.arange(nsamp, dtype=np.int64)
    sweep = t // lsw
    tau = t % lsw
    nsweep = -(-nsamp // lsw)
    adv = ny / nsweep
    x = (tau + 0.5) * (nx / lsw) - 0.5
    x = np.where(sweep % 2 == 0, x, (nx - 1) - x)
    y = sweep * adv + (adv - 1.0) / 2.0
    return y, x


def _pointing_rows(ny, nx, yb, xb, dy, dx, phi, psi, ncomp, progress=None):
    cy, cx = (ny - 1) / 2.0, (nx - 1) / 2.0
    ndet, nsamp = len(dy), len(yb)
    pix = np.empty((ndet, nsamp), np.int32)
    cos2 = np.empty((ndet, nsamp), np.float32) if ncomp == 3 else None
    sin2 = np.empty((ndet, nsamp), np.float32) if ncomp == 3 else None
    cphi, sphi = np.cos(phi), np.sin(phi)
    for d in range(ndet):
        ry = (yb - cy) + dy[d]
        rx = (xb - cx) + dx[d]
        py = cy + sphi * rx + cphi * ry
        px = cx + cphi * rx - sphi * ry
        iy = np.floor(py + 0.5).astype(np.int64)
        ix = np.floor(px + 0.5).astype(np.int64)
        ok = (iy >= 0) & (iy < ny) & (ix >= 0) & (ix < nx)
        pix[d] = np.where(ok, iy * nx + ix, -1)
        if ncomp == 3:
            ang = 2.0 * (psi[d] + phi)
            cos2[d] = np.cos(ang)
            sin2[d] = np.sin(ang)
        if progress and (d + 1) % 128 == 0:
            progress(d + 1, ndet)
    return pix, cos2, sin2


def raster_scan(*, ncomp, ny, nx, ndet, nsamp, fsample, layout="hex",
                hex_diameter_px=60.0, sigma=1.0, sigma_scatter=0.0,
                fknee=(1.0, 1.0), alpha=-3.0, drift_deg=0.0, seed=(0, 0),
                white=False, with_sky=True, progress=None):
    """A seeded raster scan.

    layout: "line" puts detector d at cross-scan offset d px (no along-scan
    offset); "hex" uses hex_focal_plane with a seeded lattice rotation.
    sigma_scatter: sigma_d = sigma * exp(sigma_scatter * N(0, 1)).
    fknee: (lo, hi), f_knee,d ~ U(lo, hi).  drift_deg: total scan-angle drift
    is U(-drift_deg, drift_deg) degrees over the scan.  white: pure white noise.
    progress: optional callable(done, ndet), called every 128 detectors.
    """
    from .noise import noise_spectrum, inverse_spectrum, white_inverse_spectrum
    from .sky import grf_sky

    ss = np.random.SeedSequence(list(seed))
    c_sky, c_fp, c_psi, c_par, c_drift, c_noise = ss.spawn(6)
    r_fp = np.random.default_rng(c_fp)
    r_psi = np.random.default_rng(c_psi)
    r_par = np.random.default_rng(c_par)
    r_drift = np.random.default_rng(c_drift)

    if layout == "line":
        dy = np.arange(ndet, dtype=np.float64)
        dx = np.zeros(ndet)
    elif layout == "hex":
        dy, dx = hex_focal_plane(ndet, hex_diameter_px,
                                 rotation=r_fp.uniform(0.0, math.pi / 3.0))
    else:
        raise ValueError(layout)
    psi = r_psi.uniform(0.0, math.pi, ndet)
    sig = sigma * np.exp(sigma_scatter * r_par.standard_normal(ndet))
    fk = r_par.uniform(fknee[0], fknee[1], ndet)
    dphi = math.radians(r_drift.uniform(-drift_deg, drift_deg)) if drift_deg else 0.0

    yb, xb = raster_boresight(nsamp, ny, nx)
    t = np.arange(nsamp, dtype=np.float64)
    phi = dphi * (t / nsamp - 0.5)
    pix, cos2, sin2 = _pointing_rows(ny, nx, yb, xb, dy, dx, phi, psi, ncomp, progress)
    bore = np.stack([yb, xb, np.cos(phi), np.sin(phi), np.cos(2 * phi), np.sin(2 * phi)])
    det_off = np.stack([dy, dx, np.cos(2 * psi), np.sin(2 * psi)])

    S = noise_spectrum(nsamp, fsample, sig, fk, alpha)
    if white:
        iN = white_inverse_spectrum(nsamp, sig)
        S = np.repeat((sig**2)[:, None], S.shape[1], axis=1)
    else:
        iN = inverse_spectrum(S)
    sky = grf_sky(ncomp, ny, nx, np.random.default_rng(c_sky)) if with_sky else None
    meta = dict(psi=psi, sigma=sig, fknee=fk, dphi=dphi, dy=dy, dx=dx,
                noise_seed=c_noise, layout=layout)
    return ScanInputs(ncomp, ny, nx, ndet, nsamp, fsample, pix, cos2, sin2,
                      iN, S, sky, meta, bore=np.ascontiguousarray(bore),
                      det_off=np.ascontiguousarray(det_off))


def boresight_only(inp):
    """A copy of raster-scan inputs that carries its pointing only as the
    boresight model (pix, cos2psi and sin2psi dropped)."""
    import dataclasses
    if inp.bore is None or inp.det_off is None:
        raise ValueError("these inputs carry no boresight model")
    return dataclasses.replace(inp, pix=None, cos2psi=None, sin2psi=None)


def _identical_spectra(ndet, nsamp, fsample, sigma, fknee, alpha, white):
    from .noise import noise_spectrum, inverse_spectrum, white_inverse_spectrum
    sig = np.full(ndet, float(sigma))
    if white:
        S = np.full((ndet, nsamp // 2 + 1), float(sigma) ** 2)
        return S, white_inverse_spectrum(nsamp, sig)
    S = noise_spectrum(nsamp, fsample, sig, np.full(ndet, float(fknee)), alpha)
    return S, inverse_spectrum(S)


def periodic_torus_scan(ncomp, ny=7, nx=8, periods=4, fsample=100.0,
                        sigma=1.0, fknee=2.0, alpha=-3.0, white=False):
    """Coprime-torus scan: pix(t) = (t mod ny, t mod nx), with gcd(ny, nx) = 1
    and nsamp a multiple of ny*nx, so every map translation is a time shift.
    I-only uses one detector; IQU uses three co-pointed detectors with
    psi = 0, pi/3, 2pi/3.  All detectors share one spectrum."""
    if math.gcd(ny, nx) != 1:
        raise ValueError("torus sides must be coprime")
    nsamp = ny * nx * periods
    if nsamp % 2:
        nsamp *= 2
    t = np.arange(nsamp)
    row = ((t % ny) * nx + (t % nx)).astype(np.int32)
    ndet = 1 if ncomp == 1 else 3
    pix = np.repeat(row[None, :], ndet, axis=0)
    cos2 = sin2 = None
    psi = np.array([0.0, math.pi / 3, 2 * math.pi / 3])[:ndet]
    if ncomp == 3:
        cos2 = np.repeat(np.cos(2 * psi)[:, None], nsamp, axis=1).astype(np.float32)
        sin2 = np.repeat(np.sin(2 * psi)[:, None], nsamp, axis=1).astype(np.float32)
    S, iN = _identical_spectra(ndet, nsamp, fsample, sigma, fknee, alpha, white)
    return ScanInputs(ncomp, ny, nx, ndet, nsamp, fsample, pix, cos2, sin2, iN, S,
                      None, dict(psi=psi, layout="torus"))


def crosslinked_torus_scan(ncomp, L=8, periods=4, fsample=100.0, sigma=1.0,
                           fknee=2.0, alpha=-3.0, white=False,
                           psi_families=(0.0, math.pi / 3, 2 * math.pi / 3)):
    """L x L torus scanned by two diagonal detector families:
    family 1 detector d hits ((d + t) mod L, t mod L), family 2 hits
    ((d - t) mod L, t mod L), d = 0 .. L-1.  Every map translation is a
    detector permutation plus a time shift, and the two families cross-link
    each pixel.  For IQU a third family co-points with family 1; each family
    has its own detector angle.  nsamp is a multiple of L; spectra identical."""
    nsamp = L * periods
    if nsamp % 2:
        nsamp *= 2
    t = np.arange(nsamp)
    fams = [(+1, psi_families[0]), (-1, psi_families[1])]
    if ncomp == 3:
        fams.append((+1, psi_families[2]))
    rows, psis = [], []
    for sgn, ps in fams:
        for d in range(L):
            y = (d + sgn * t) % L
            x = t % L
            rows.append((y * L + x).astype(np.int32))
            psis.append(ps)
    pix = np.stack(rows)
    ndet = pix.shape[0]
    psi = np.array(psis)
    cos2 = sin2 = None
    if ncomp == 3:
        cos2 = np.repeat(np.cos(2 * psi)[:, None], nsamp, axis=1).astype(np.float32)
        sin2 = np.repeat(np.sin(2 * psi)[:, None], nsamp, axis=1).astype(np.float32)
    S, iN = _identical_spectra(ndet, nsamp, fsample, sigma, fknee, alpha, white)
    return ScanInputs(ncomp, L, L, ndet, nsamp, fsample, pix, cos2, sin2, iN, S,
                      None, dict(psi=psi, layout="crosslinked-torus"))
