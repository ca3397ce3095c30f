"""FP64 oracle of the learned linear correction to the circulant preconditioner
(test infrastructure only; not part of the paper).

M_L r = M_C r + Sigma^-1 H^T H Sigma^-T r with H = C2 o C1, where C1 (3 -> 16
channels) and C2 (16 -> 16) are 5 x 5 "same" correlations with zero padding
and no bias, and H^T = C1^T o C2^T is the exact adjoint (the correlation with
the spatially flipped kernel and swapped channels).  The four layers are
C1, C2, C2^T, C1^T (3 -> 16 -> 16 -> 16 -> 3); the weight tying makes M_L
symmetric, and M_L - M_C = (H Sigma^-T)^T (H Sigma^-T) is positive
semi-definite, so M_L is SPD whenever M_C is and plain PCG stays valid.

Training pairs come from circulant PCG iterates x_k and a converged x_f:
e = x_f - x_k, r = A e, r_w = Sigma^-T r, e_w = Sigma e and the target
t = e_w - Sigma M_C r, so that Sigma M_L r = Sigma M_C r + H^T H r_w matches
e_w.  Loss: mean over pairs of ||H^T H r_w - t||^2 / ||e_w||^2.  Adam on the
two weight tensors.
"""

import numpy as np

KS = 5
HALF = KS // 2


def conv_same(x, W):
    """y[o, i, j] = sum_{c,u,v} W[o, c, u, v] x[c, i+u-2, j+v-2] (zero outside).
    x: (..., Cin, H, W) ; W: (Cout, Cin, 5, 5)."""
    H, Wd = x.shape[-2:]
    pad = [(0, 0)] * (x.ndim - 2) + [(HALF, HALF), (HALF, HALF)]
    xp = np.pad(x, pad)
    out = np.zeros(x.shape[:-3] + (W.shape[0], H, Wd))
    for u in range(KS):
        for v in range(KS):
            out += np.einsum("oc,...chw->...ohw", W[:, :, u, v], xp[..., u:u + H, v:v + Wd])
    return out


def flip_T(W):
    """Kernel of the adjoint correlation: swapped channels, flipped taps."""
    return np.transpose(W, (1, 0, 2, 3))[:, :, ::-1, ::-1]


def conv_same_T(z, W):
    """Adjoint of conv_same(., W): (C^T z)[c, i, j] = sum_{o,u,v} W[o,c,u,v] z[o, i-u+2, j-v+2]."""
    return conv_same(z, flip_T(W))


def HtH(x, W1, W2):
    return conv_same_T(conv_same_T(conv_same(conv_same(x, W1), W2), W2), W1)


def wgrad(P, Q):
    """dW[o, c, u, v] = sum_{b,i,j} P[b, o, i, j] Q[b, c, i+u-2, j+v-2]."""
    H, Wd = Q.shape[-2:]
    Qp = np.pad(Q, [(0, 0), (0, 0), (HALF, HALF), (HALF, HALF)])
    g = np.zeros((P.shape[1], Q.shape[1], KS, KS))
    for u in range(KS):
        for v in range(KS):
            g[:, :, u, v] = np.einsum("bohw,bchw->oc", P, Qp[:, :, u:u + H, v:v + Wd])
    return g


def loss_and_grad(R, T, E2, W1, W2):
    """R, T: (P, 3, H, W) whitened residuals and targets; E2: (P,) ||e_w||^2.
    Returns the loss and its gradients with respect to W1 and W2 (chain rule
    through the four tied layers)."""
    P = R.shape[0]
    a1 = conv_same(R, W1)
    a2 = conv_same(a1, W2)
    a3 = conv_same_T(a2, W2)
    y = conv_same_T(a3, W1)
    d = y - T
    L = float(np.mean(np.sum(d * d, axis=(1, 2, 3)) / E2))
    gy = (2.0 / P) * d / E2[:, None, None, None]
    g_a3 = conv_same(gy, W1)              # adjoint of C1^T
    g_a2 = conv_same(g_a3, W2)            # adjoint of C2^T
    g_a1 = conv_same_T(g_a2, W2)          # adjoint of C2
    dW1 = wgrad(g_a1, R) + wgrad(a3, gy)
    dW2 = wgrad(g_a2, a1) + wgrad(a2, g_a3)
    return L, dW1, dW2


def adam_step(W, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); t is the 1-based step number."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return W - lr * mh / (np.sqrt(vh) + eps), m, v


def init_weights(rng, cin=3, hidden=16):
    """N(0, (0.1 / sqrt(fan_in))^2) for both tensors (H = 0 is a stationary
    point of H^T H, so training cannot start there)."""
    W1 = rng.standard_normal((hidden, cin, KS, KS)) * 0.1 / np.sqrt(cin * KS * KS)
    W2 = rng.standard_normal((hidden, hidden, KS, KS)) * 0.1 / np.sqrt(hidden * KS * KS)
    return W1, W2


def whiten(circ, r):
    """Sigma^-T r as an image (nc, ny, nx)."""
    rp = np.asarray(r, dtype=np.float64).reshape(circ.nc, circ.npix).T
    u = np.einsum("pba,pb->pa", circ.Siginv, rp)
    return u.T.reshape(circ.nc, circ.ny, circ.nx)


def unwhiten(circ, img):
    """Sigma^-1 applied to an image (nc, ny, nx); masked, flat map."""
    vp = np.asarray(img, dtype=np.float64).reshape(circ.nc, circ.npix).T
    z = np.einsum("pab,pb->pa", circ.Siginv, vp)
    z[~circ.mask] = 0.0
    return z.T.reshape(-1)


def sigma_apply(circ, x):
    """Sigma x = B^(1/2) x per pixel, as an image."""
    xp = np.asarray(x, dtype=np.float64).reshape(circ.nc, circ.npix).T
    y = np.einsum("pab,pb->pa", circ.Sigma, xp)
    return y.T.reshape(circ.nc, circ.ny, circ.nx)


class LearnedPrecon:
    """M_L r = M_C r + Sigma^-1 H^T H Sigma^-T r."""

    def __init__(self, circ, W1, W2):
        self.circ, self.W1, self.W2 = circ, W1, W2

    def __call__(self, r):
        c = self.circ
        corr = unwhiten(c, HtH(whiten(c, r)[None], self.W1, self.W2)[0])
        return c(r) + corr


def make_pair(apply_A, circ, x_f, x_k):
    """(r_w, t, ||e_w||^2) of one training pair from a converged x_f and an
    iterate x_k."""
    e = (np.asarray(x_f) - np.asarray(x_k)).reshape(-1)
    r = apply_A(e)
    r_w = whiten(circ, r)
    e_w = sigma_apply(circ, e)
    t = e_w - sigma_apply(circ, circ(r))
    return r_w, t, float(np.sum(e_w * e_w))
