"""FP64 preconditioners for the map-making equation (test infrastructure only).

* Binned (eq. 3-4): M_B^-1 = P^T diag(N^-1_tt) P, block-diagonal in pixels.
* Jacobi (eq. 5): the same with N = a I, a = 1.
* Circulant / constant correlation (Implementation section, eq. 7-12; the
  Regularization and Polarization sections, eq. 13): A ~ Sigma^T Q Sigma with
  Sigma^T Sigma = the binned blocks, Q circulant built from the rows of A at
  one reference pixel, applied through 2-D FFTs.

Readings where the paper is silent: Sigma is the symmetric square root of the
binned block; the reference pixel is (ny//2, nx//2) or the nearest active
pixel (smallest id on ties); q is tapered by an isotropic Gaussian of the
minimal-image displacement, symmetrised as (q(d) + q(-d)^T)/2, and the
per-wavenumber Hermitian blocks get an eigenvalue floor of eps * the largest
eigenvalue over all wavenumbers.
"""

import numpy as np

from .operators import apply_A


class BinnedPrecon:
    """z_p = B_p^-1 r_p on active pixels, 0 elsewhere (eq. 3-5)."""

    def __init__(self, B, mask):
        self.nc = B.shape[1]
        self.npix = B.shape[0]
        self.mask = mask
        self.Binv = np.zeros_like(B)
        self.Binv[mask] = np.linalg.inv(B[mask])

    def __call__(self, r):
        rp = np.asarray(r, dtype=np.float64).reshape(self.nc, self.npix).T
        z = np.einsum("pab,pb->pa", self.Binv, rp)
        return z.T.reshape(-1)


def sym_sqrt(B):
    """Symmetric square root and inverse square root of SPD blocks (npix,n,n)."""
    lam, V = np.linalg.eigh(B)
    if np.any(lam <= 0):
        raise ValueError("sym_sqrt needs positive definite blocks")
    S = np.einsum("pij,pj,pkj->pik", V, np.sqrt(lam), V)
    Si = np.einsum("pij,pj,pkj->pik", V, 1.0 / np.sqrt(lam), V)
    return S, Si


def reference_pixel(mask, ny, nx):
    """The pixel nearest the map centre (Implementation section): (ny//2, nx//2)
    if active, else the nearest active pixel in Euclidean distance, smallest
    pixel id on ties."""
    cy, cx = ny // 2, nx // 2
    c = cy * nx + cx
    if mask[c]:
        return c
    p = np.arange(ny * nx)
    d2 = (p // nx - cy) ** 2 + (p % nx - cx) ** 2
    d2 = np.where(mask, d2, np.iinfo(np.int64).max)
    return int(np.argmin(d2))  # first minimum = smallest id


def minimal_image(n):
    """Displacements 0..n-1 mapped to the minimal image in (-n/2, n/2]."""
    d = np.arange(n)
    return np.where(d > n // 2, d - n, d)


def gaussian_taper(ny, nx, sigma):
    """g(dy, dx) = exp(-(dy~^2 + dx~^2) / (2 sigma^2)) on the displacement grid,
    dy~, dx~ minimal images (Regularization section).  sigma <= 0 or None: 1."""
    if sigma is None or sigma <= 0 or not np.isfinite(sigma):
        return np.ones((ny, nx))
    dy = minimal_image(ny)[:, None].astype(np.float64)
    dx = minimal_image(nx)[None, :].astype(np.float64)
    return np.exp(-(dy**2 + dx**2) / (2.0 * sigma**2))


class CirculantPrecon:
    """The constant-correlation preconditioner M_C (eq. 8-13).

    Build: Sigma_p = B_p^(1/2); probe c_g = A e_(r,g) for g < ncomp (eq. 6);
    q(d)_ab = [Sigma_r^-T C_j Sigma_j^-1]_ab with j = r + d (mod the map),
    (C_j)_gb = c_g[b, j], zero for inactive j (eq. 10, eq. 13); taper;
    symmetrise; K(k) = conj(FFT2 q)(k) (eq. 11); Hermitian eigenvalue floor;
    store K(k)^-1.
    Apply (eq. 12): z = Sigma^-1 F^-1 K^-1 F Sigma^-T r.
    """

    def __init__(self, scan, mask, B, sigma_taper=None, symmetrize=True,
                 eig_floor_rel=1e-6, ref=None):
        nc, ny, nx = scan.ncomp, scan.ny, scan.nx
        npix = ny * nx
        self.nc, self.ny, self.nx, self.npix = nc, ny, nx, npix
        self.mask = mask
        self.Sigma = np.zeros((npix, nc, nc))
        self.Siginv = np.zeros((npix, nc, nc))
        S, Si = sym_sqrt(B[mask])
        self.Sigma[mask] = S
        self.Siginv[mask] = Si
        self.ref = reference_pixel(mask, ny, nx) if ref is None else int(ref)
        r = self.ref
        # probe rows: C[g, b, j] = (A e_(r,g))[b, j]
        C = np.zeros((nc, nc, npix))
        for g in range(nc):
            e = np.zeros((nc, npix))
            e[g, r] = 1.0
            C[g] = apply_A(scan, e, mask).reshape(nc, npix)
        self.probe = C
        # q on the displacement grid
        ry, rx = divmod(r, nx)
        jy, jx = np.divmod(np.arange(npix), nx)
        dy = (jy - ry) % ny
        dx = (jx - rx) % nx
        Cj = np.transpose(C, (2, 0, 1))                      # (j, g, b)
        qj = np.einsum("ga,jgb,jbc->jac", self.Siginv[r], Cj, self.Siginv)
        qj[~mask] = 0.0
        q = np.zeros((ny, nx, nc, nc))
        q[dy, dx] = qj
        q *= gaussian_taper(ny, nx, sigma_taper)[:, :, None, None]
        if symmetrize:
            qm = q[(-np.arange(ny)) % ny][:, (-np.arange(nx)) % nx]   # q(-d)
            q = 0.5 * (q + np.transpose(qm, (0, 1, 3, 2)))
        self.q = q
        qhat = np.fft.fft2(q, axes=(0, 1))                   # (ky, kx, a, b)
        K = np.conj(qhat)
        self.K = K
        self.n_floored = 0
        if symmetrize:
            self.Kinv, self.lam, self.n_floored = self.floored_inverse(K, eig_floor_rel)
        else:
            self.lam = None
            self.Kinv = np.linalg.inv(K)

    @staticmethod
    def floored_inverse(K, eig_floor_rel):
        """Positive definite inverse of the Hermitian blocks K(k) (reading of
        the Implementation section, which needs Q invertible): every
        eigenvalue of every block is raised to at least eig_floor_rel times
        the largest eigenvalue over ALL wavenumbers (the largest eigenvalue of
        the whole block-circulant Q), then K^-1 = V diag(1/lam) V^H.
        Returns (K^-1, the floored eigenvalues, how many were raised)."""
        lam, V = np.linalg.eigh(K)
        floor = eig_floor_rel * lam.max()
        n_floored = int(np.count_nonzero(lam < floor))
        lam = np.maximum(lam, floor)
        Kinv = np.einsum("...ij,...j,...kj->...ik", V, 1.0 / lam, np.conj(V))
        return Kinv, lam, n_floored

    def __call__(self, rvec):
        nc, ny, nx, npix = self.nc, self.ny, self.nx, self.npix
        rp = np.asarray(rvec, dtype=np.float64).reshape(nc, npix).T      # (p, a)
        u = np.einsum("pba,pb->pa", self.Siginv, rp)                    # Sigma^-T r
        uh = np.fft.fft2(u.T.reshape(nc, ny, nx), axes=(1, 2))          # (a, ky, kx)
        vh = np.einsum("yxab,byx->ayx", self.Kinv, uh)
        v = np.fft.ifft2(vh, axes=(1, 2)).real.reshape(nc, npix).T      # (p, a)
        z = np.einsum("pab,pb->pa", self.Siginv, v)                     # Sigma^-1 v
        z[~self.mask] = 0.0
        return z.T.reshape(-1)
