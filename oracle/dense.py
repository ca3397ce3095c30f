"""Dense A from unit-vector probes and a direct solve (test infrastructure only).

Each column of A is one A-apply on a unit map, A_ij = (A e_i)_j (eq. 6).  On
tiny maps the full matrix restricted to the active unknowns is Cholesky-solved,
giving the exact m* = A^-1 b that every convergent PCG reaches.
"""

import numpy as np
import scipy.linalg


def dense_operator(apply, n, index=None):
    """Matrix of a linear map given as a function, on the unknowns `index`
    (default all n)."""
    idx = np.arange(n) if index is None else np.asarray(index)
    M = np.zeros((len(idx), len(idx)))
    for c, i in enumerate(idx):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, c] = apply(e)[idx]
    return M


def dense_solve(A, b):
    """Cholesky solve of the SPD system A x = b."""
    c, low = scipy.linalg.cho_factor(A)
    return scipy.linalg.cho_solve((c, low), b)
