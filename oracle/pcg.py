"""Preconditioned conjugate gradients in FP64 (test infrastructure only).

The textbook PCG the paper solves eq. 2 with (Introduction and its footnote on
preconditioning), started from x0 = 0 and stopped when the recursive residual
satisfies ||r||_2 <= tol ||b||_2; the iteration count is the number of
A-applies inside the loop.  Breakdown (p.Ap <= 0 or r.z <= 0, or a non-finite
scalar) stops the solve with the last good iterate.

flexible=True takes the Polak-Ribiere form of beta, z_{k+1}.(r_{k+1} - r_k) /
r_k.z_k, in place of r_{k+1}.z_{k+1} / r_k.z_k.  The two agree in exact
arithmetic when M is symmetric; the flexible form keeps the search directions
conjugate when M is only nearly symmetric (a preconditioner evaluated in
reduced precision), at the price of one more inner product.

Also the error A-norm estimate quoted with the residual A-norm figure in the
Results section: ||x_k - x||_A^2 ~ sum_{j=k}^{k+d-1} alpha_j r_j.z_j, d = 4
(with preconditioning r_j.z_j takes the place of ||r_j||^2).
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    history: list = field(default_factory=list)   # ||r_k|| / ||b||, k = 0..iters
    alphas: list = field(default_factory=list)
    rhos: list = field(default_factory=list)      # r_k . z_k
    iterates: list | None = None


def pcg(apply_A, apply_M, b, tol=1e-6, maxiter=5000, x0=None, keep_iterates=False,
        flexible=False):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    res = PCGResult(x, 0, False, False, iterates=[] if keep_iterates else None)
    if bnorm == 0.0:
        res.converged = True
        res.history.append(0.0)
        return res
    res.history.append(np.linalg.norm(r) / bnorm)
    if res.history[-1] <= tol:
        res.converged = True
        return res
    z = apply_M(r)
    p = z.copy()
    rho = float(r @ z)
    res.rhos.append(rho)
    for it in range(1, maxiter + 1):
        s = apply_A(p)
        ps = float(p @ s)
        if not (np.isfinite(ps) and np.isfinite(rho)) or ps <= 0.0 or rho <= 0.0:
            res.breakdown = True
            break
        alpha = rho / ps
        x = x + alpha * p
        r_old = r
        r = r - alpha * s
        res.iters = it
        res.alphas.append(alpha)
        res.history.append(np.linalg.norm(r) / bnorm)
        if keep_iterates:
            res.iterates.append(x.copy())
        if res.history[-1] <= tol:
            res.converged = True
            break
        z = apply_M(r)
        rho_new = float(r @ z)
        beta = (float(z @ (r - r_old)) if flexible else rho_new) / rho
        p = z + beta * p
        rho = rho_new
        res.rhos.append(rho)
    res.x = x
    return res


def anorm_estimate(alphas, rhos, d=4):
    """Estimates e_k ~ ||x_k - x||_A^2 = sum_{j=k}^{k+d-1} alpha_j rho_j for every
    k with k+d-1 inside the recorded iterations."""
    a = np.asarray(alphas, dtype=np.float64)
    r = np.asarray(rhos[: len(a)], dtype=np.float64)
    terms = a * r
    n = len(terms) - d + 1
    return np.array([terms[k:k + d].sum() for k in range(max(n, 0))])
