"""FP64 pointing, noise and map-making operators (test infrastructure only).

Follows the linear data model d = P m + n and the map-making equation
(P^T N^-1 P) m = P^T N^-1 d of the Introduction (eq. 1 and eq. 2):

* P has one non-zero per row (nearest-pixel pointing, the footnote to eq. 1)
  with weights (1, cos 2psi, sin 2psi) for T, Q, U (Test setup section);
  pix = -1 marks an off-map sample, whose row of P is zero.
* N is stationary, so N^-1 is circulant in time: N^-1 v = irfft(iN * rfft(v))
  per detector with iN = 1/S(f) on the n/2+1 real-FFT frequencies, with no
  padding or apodisation.  With inter-detector correlations (the ACT-like
  noise model of the Test setup section) N^-1 is a matrix over detectors at
  each frequency: N^-1(k) = diag(iN[:, k]) - V_b V_b^T for the frequency bin b
  holding k, applied to the vector of all detectors' spectra at k.
* The unknowns are restricted to the active pixels (hit, and for I,Q,U with
  a well-conditioned binned block); inactive entries are zero on input and
  output of every operator.

Maps are arrays of shape (ncomp, npix), pixel id p = y * nx + x.
"""

import numpy as np

DET_CHUNK = 8


class OracleScan:
    """Read-only view of one scan's inputs in the oracle's own terms.

    The pointing weights and inverse spectra arrive as float32 and are used
    as the float64 numbers they represent.  Inputs without pix carry the
    boresight model instead (bore, det_off), which boresight.expand_pointing
    turns into float64 per-sample pointing.
    """

    def __init__(self, inputs):
        self.ncomp = int(inputs.ncomp)
        self.ny = int(inputs.ny)
        self.nx = int(inputs.nx)
        self.npix = self.ny * self.nx
        if getattr(inputs, "pix", None) is None:
            # pointing given only as the boresight model: expand it here
            from .boresight import expand_pointing
            self.pix, c2, s2 = expand_pointing(inputs.bore, inputs.det_off, self.ny, self.nx)
            self.cos2psi = c2 if self.ncomp == 3 else None
            self.sin2psi = s2 if self.ncomp == 3 else None
        else:
            self.pix = np.asarray(inputs.pix)
            self.cos2psi = None if inputs.cos2psi is None else np.asarray(inputs.cos2psi)
            self.sin2psi = None if inputs.sin2psi is None else np.asarray(inputs.sin2psi)
        self.ndet, self.nsamp = self.pix.shape
        self.iN = np.asarray(inputs.inv_noise, dtype=np.float64)
        if self.iN.shape != (self.ndet, self.nsamp // 2 + 1):
            raise ValueError("inverse spectrum must be [ndet][nsamp/2+1]")
        edges = getattr(inputs, "corr_edges", None)
        self.corr = None
        if edges is not None:
            V = np.asarray(inputs.corr_V, dtype=np.float64)
            edges = np.asarray(edges, dtype=np.int64)
            if edges[0] != 0 or edges[-1] != self.nsamp // 2 + 1 or np.any(np.diff(edges) <= 0):
                raise ValueError("correlation bins must tile 0..nsamp/2")
            if V.shape[:2] != (len(edges) - 1, self.ndet):
                raise ValueError("V must be [nbins][ndet][rank]")
            self.corr = (edges, V)
        if self.ncomp not in (1, 3):
            raise ValueError("ncomp must be 1 or 3")

    def det_range(self, dets):
        return range(self.ndet) if dets is None else dets

    def weights(self, d0, d1):
        """Pointing weights w[alpha, d, s] for detectors d0..d1-1 (float64)."""
        w = np.ones((self.ncomp, d1 - d0, self.nsamp))
        if self.ncomp == 3:
            w[1] = self.cos2psi[d0:d1]
            w[2] = self.sin2psi[d0:d1]
        return w


def _chunks(n, step=DET_CHUNK):
    for a in range(0, n, step):
        yield a, min(n, a + step)


def pointing(scan, m, d0=0, d1=None):
    """P m for detectors d0..d1-1: t[d, s] = sum_alpha w[alpha,d,s] m[alpha, pix[d,s]]
    (eq. 1; one pixel per sample).  m: (ncomp, npix).  Returns (d1-d0, nsamp)."""
    d1 = scan.ndet if d1 is None else d1
    m = np.asarray(m, dtype=np.float64).reshape(scan.ncomp, scan.npix)
    pix = scan.pix[d0:d1]
    hit = pix >= 0
    safe = np.where(hit, pix, 0)
    w = scan.weights(d0, d1)
    tod = np.zeros((d1 - d0, scan.nsamp))
    for a in range(scan.ncomp):
        tod += w[a] * m[a][safe]
    tod[~hit] = 0.0
    return tod


def pointing_T(scan, tod, d0=0, d1=None):
    """P^T t for detectors d0..d1-1: y[alpha, p] = sum over samples with
    pix = p of w[alpha,d,s] t[d,s].  Returns (ncomp, npix)."""
    d1 = scan.ndet if d1 is None else d1
    pix = scan.pix[d0:d1]
    hit = pix >= 0
    w = scan.weights(d0, d1)
    y = np.zeros((scan.ncomp, scan.npix))
    p = pix[hit]
    for a in range(scan.ncomp):
        y[a] = np.bincount(p, weights=(w[a] * tod)[hit], minlength=scan.npix)
    return y


def inv_noise(scan, tod, d0=0, d1=None):
    """N^-1 t per detector as a circulant filter: irfft(iN_d * rfft(t_d)).
    With correlations tod must hold every detector (d0 = 0, d1 = ndet): at
    each frequency k of bin b, F[:, k] <- iN[:, k] F[:, k] - V_b (V_b^T F[:, k])."""
    d1 = scan.ndet if d1 is None else d1
    f = np.fft.rfft(np.asarray(tod, dtype=np.float64), axis=1)
    if scan.corr is None:
        f *= scan.iN[d0:d1]
    else:
        assert d0 == 0 and d1 == scan.ndet, "correlated noise couples all detectors"
        edges, V = scan.corr
        g = f * scan.iN
        for b in range(len(edges) - 1):
            k0, k1 = edges[b], edges[b + 1]
            g[:, k0:k1] -= V[b] @ (V[b].T @ f[:, k0:k1])
        f = g
    return np.fft.irfft(f, scan.nsamp, axis=1)


def detector_weights(scan):
    """w_d = (N^-1)_tt, the diagonal of each detector's circulant N^-1, i.e.
    the mean of its eigenvalues over all n two-sided frequencies (the
    N^-1_tt of eq. 3-4).  Equals 1/sigma^2 for white noise."""
    n = scan.nsamp
    out = np.empty(scan.ndet)
    diag = scan.iN.copy()
    if scan.corr is not None:   # diagonal of N^-1(k): iN_d(k) - sum_j V_b[d, j]^2
        edges, V = scan.corr
        for b in range(len(edges) - 1):
            diag[:, edges[b]:edges[b + 1]] -= (V[b] ** 2).sum(axis=1)[:, None]
    for d in range(scan.ndet):
        half = diag[d]
        two_sided = np.concatenate([half, half[1:n // 2][::-1]])
        assert two_sided.size == n
        out[d] = two_sided.mean()
    return out


def hits(scan):
    """Number of samples falling in each pixel."""
    p = scan.pix[scan.pix >= 0]
    return np.bincount(p, minlength=scan.npix)


def binned_blocks(scan, det_weight):
    """B_p = sum over samples in p of w_d u u^T, u = (1, cos 2psi, sin 2psi)
    (eq. 3-4; eq. 7 for the polarised blocks).  Returns (npix, nc, nc)."""
    nc = scan.ncomp
    B = np.zeros((scan.npix, nc, nc))
    for d0, d1 in _chunks(scan.ndet):
        pix = scan.pix[d0:d1]
        hit = pix >= 0
        p = pix[hit]
        w = scan.weights(d0, d1)
        wd = np.broadcast_to(np.asarray(det_weight, dtype=np.float64)[d0:d1, None],
                             pix.shape)[hit]
        for a in range(nc):
            for b in range(nc):
                B[:, a, b] += np.bincount(p, weights=wd * w[a][hit] * w[b][hit],
                                          minlength=scan.npix)
    return B


def active_mask(scan, B, rcond=1e-3):
    """Active pixels: hit at least once and, for I,Q,U, binned block with
    lambda_min / lambda_max >= rcond."""
    h = hits(scan)
    act = h > 0
    if scan.ncomp == 3:
        lam = np.linalg.eigvalsh(B)
        ok = np.zeros(scan.npix, bool)
        pos = lam[:, -1] > 0
        ok[pos] = lam[pos, 0] / lam[pos, -1] >= rcond
        act &= ok
    return act


def _groups(scan):
    # correlated noise couples all detectors: one group
    return [(0, scan.ndet)] if scan.corr is not None else list(_chunks(scan.ndet))


def apply_A(scan, x, mask):
    """A x = P^T N^-1 P x (eq. 2) on the active set.  x: (ncomp*npix,) or
    (ncomp, npix); returns the same flat shape (ncomp*npix,)."""
    xm = np.asarray(x, dtype=np.float64).reshape(scan.ncomp, scan.npix) * mask
    y = np.zeros((scan.ncomp, scan.npix))
    for d0, d1 in _groups(scan):
        t = pointing(scan, xm, d0, d1)
        t = inv_noise(scan, t, d0, d1)
        y += pointing_T(scan, t, d0, d1)
    return (y * mask).reshape(-1)


def rhs(scan, d, mask):
    """b = P^T N^-1 d (eq. 2) on the active set.  d: (ndet, nsamp)."""
    y = np.zeros((scan.ncomp, scan.npix))
    for d0, d1 in _groups(scan):
        t = inv_noise(scan, np.asarray(d[d0:d1], dtype=np.float64), d0, d1)
        y += pointing_T(scan, t, d0, d1)
    return (y * mask).reshape(-1)
