"""FP64 expansion of a boresight pointing model into per-sample pointing
(test infrastructure only).

The data model of the Introduction (eq. 1) has each sample see one pixel
through the telescope's pointing; the Test setup section builds it from the
scanning pattern of the telescope and the detectors' places and polarisation
angles in the focal plane.  Reading used here (flat sky, pixel units):

* the boresight of sample t sits at (y_b(t), x_b(t)) in pixel coordinates and
  the focal plane is turned by the scan angle phi(t) about the map centre
  (c_y, c_x) = ((ny - 1) / 2, (nx - 1) / 2);
* detector d sits at offset (dy_d, dx_d) from the boresight before the turn
  and has polarisation angle psi_d;
* its position is the turned offset point
      ry = (y_b - c_y) + dy_d,  rx = (x_b - c_x) + dx_d,
      py = (c_y + sin(phi) rx) + cos(phi) ry,
      px = (c_x + cos(phi) rx) - sin(phi) ry,
  in float64 in that order (each sum and product rounded once), and its
  pixel is (floor(py + 1/2), floor(px + 1/2)), none (-1) off the map;
* its weights for Q and U are cos 2(psi_d + phi) and sin 2(psi_d + phi), from
  the given cos/sin of 2 psi_d and 2 phi by the angle-sum identities.

Inputs: bore float64 [6][nsamp] = y_b, x_b, cos phi, sin phi, cos 2phi,
sin 2phi; det_off float64 [4][ndet] = dy, dx, cos 2psi, sin 2psi.
"""

import numpy as np


def expand_pointing(bore, det_off, ny, nx):
    """Returns pix int32 [ndet][nsamp] and the weights cos 2(psi + phi),
    sin 2(psi + phi) as float64 [ndet][nsamp]."""
    bore = np.asarray(bore, dtype=np.float64)
    det_off = np.asarray(det_off, dtype=np.float64)
    yb, xb, c, s, c2, s2 = bore
    dy, dx, c2p, s2p = det_off
    cy, cx = (ny - 1) / 2.0, (nx - 1) / 2.0
    ry = (yb - cy)[None, :] + dy[:, None]
    rx = (xb - cx)[None, :] + dx[:, None]
    py = (cy + s[None, :] * rx) + c[None, :] * ry
    px = (cx + c[None, :] * rx) - s[None, :] * ry
    fy = np.floor(py + 0.5)
    fx = np.floor(px + 0.5)
    on = (fy >= 0) & (fy < ny) & (fx >= 0) & (fx < nx)
    pix = np.where(on, fy * nx + fx, -1).astype(np.int32)
    cos2 = c2p[:, None] * c2[None, :] - s2p[:, None] * s2[None, :]
    sin2 = s2p[:, None] * c2[None, :] + c2p[:, None] * s2[None, :]
    return pix, cos2, sin2
