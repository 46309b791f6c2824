"""Newton-system reference -- TEST INFRASTRUCTURE ONLY.

Solves (I - h gamma J) x = b per state with LAPACK LU (scipy getrf/getrs) and
iterative refinement whose residuals are formed in extended precision
(numpy.longdouble), until the correction is below 1e-17 relative; also returns
the infinity-norm condition number of A.  J comes from the oracle's own
Jacobian, never from the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def newton_reference(J: np.ndarray, h: np.ndarray, gamma: float, rhs: np.ndarray,
                     max_iter: int = 20):
    """J: (N*N, n) row-major per state; h: (n,); rhs: (N, n).
    Returns x (N, n), kappa_inf (n,)."""
    NN, n = J.shape
    N = int(round(NN ** 0.5))
    x = np.empty((N, n))
    kappa = np.empty(n)
    for s in range(n):
        Js = J[:, s].reshape(N, N)
        A = np.eye(N) - h[s] * gamma * Js
        lu = sla.lu_factor(A)
        b = rhs[:, s]
        xs = sla.lu_solve(lu, b)
        Al = A.astype(np.longdouble)
        bl = b.astype(np.longdouble)
        xl = xs.astype(np.longdouble)
        for _ in range(max_iter):
            r = bl - Al @ xl
            d = sla.lu_solve(lu, r.astype(np.float64))
            xl = xl + d.astype(np.longdouble)
            if np.max(np.abs(d)) <= 1e-17 * np.max(np.abs(xl.astype(np.float64))):
                break
        x[:, s] = xl.astype(np.float64)
        kappa[s] = np.linalg.cond(A, np.inf)
    return x, kappa
