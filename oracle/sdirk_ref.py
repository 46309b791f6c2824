"""Implicit integrator step reference -- TEST INFRASTRUCTURE ONLY.

One step of the three-stage, L-stable, stiffly accurate singly diagonally
implicit Runge-Kutta method of order 3 (Alexander, 1977), whose diagonal
coefficient gamma is the root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6,
gamma = 0.43586652150845899942: the gamma of the Newton matrix I - h gamma J
that the paper gives as the motivation for fast Jacobians (Sec. 1).

Stage i solves z_i = h sum_{j<i} a_ij f(y + z_j) + h gamma f(y + z_i) by
simplified Newton with the matrix I - h gamma J(y), starting from z_i = 0,
for a fixed number of iterations; the step returns y + z_3 (stiffly accurate:
the last stage is the solution).  Written generically over f and J so that
the method itself is pinned on problems with known solutions; the chemistry
callers pass the oracle's own RHS and Jacobian.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0.43586652150845899942
A21 = (1.0 - GAMMA) / 2.0
B1 = -(6.0 * GAMMA ** 2 - 16.0 * GAMMA + 1.0) / 4.0
B2 = (6.0 * GAMMA ** 2 - 20.0 * GAMMA + 5.0) / 4.0
# Butcher tableau (lower triangular), nodes and weights
A = np.array([[GAMMA, 0.0, 0.0], [A21, GAMMA, 0.0], [B1, B2, GAMMA]])
C = A.sum(axis=1)
B = A[2].copy()


def sdirk3_step(f, jac, y: np.ndarray, h: float, newton_iters: int = 4):
    """f(y) -> dy/dt, jac(y) -> df/dy (dense); returns (y_next, last Newton
    increment max-norm of each stage)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    M = np.eye(n) - h * GAMMA * jac(y)
    F = []
    dn = []
    z = np.zeros(n)
    for i in range(3):
        base = np.zeros(n)
        for j in range(i):
            base = base + h * A[i, j] * F[j]
        z = np.zeros(n)
        d = np.zeros(n)
        for _ in range(newton_iters):
            g = base + h * GAMMA * f(y + z) - z          # -G(z)
            d = np.linalg.solve(M, g)
            z = z + d
        dn.append(float(np.max(np.abs(d))))
        F.append(f(y + z))
    return y + z, dn


def sdirk3_step_states(ref, phi: np.ndarray, p: np.ndarray, h: np.ndarray, newton_iters: int = 4):
    """The step for each state (column) of phi [N, n] at constant pressure
    p [n] with step h [n], with the oracle mechanism `ref` (RefMech)."""
    N, n = phi.shape
    out = np.empty_like(phi)
    dn = np.empty((3, n))
    for s in range(n):
        ps = p[s:s + 1]

        def f(y):
            return ref.eval_rates(y.reshape(N, 1), ps)["dphi"][:, 0]

        def jac(y):
            return np.asarray(ref.eval_jacobian(y.reshape(N, 1), ps)).reshape(N, N)

        out[:, s], d = sdirk3_step(f, jac, phi[:, s], float(h[s]), newton_iters)
        dn[:, s] = d
    return out, dn
