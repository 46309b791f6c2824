"""Seeded thermochemical states and Newton inputs.

State layout matches the library's: phi[j, s] with j = 0 the temperature and
j = 1..N-1 the mass fractions Y_1..Y_{N-1} (the last species' mass fraction is
implied), p[s] in Pa; the state index is the fastest-varying one.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from .mechgen import ATM, WORKLOADS, STATE_SEED_BASE

NEWTON_GAMMA = 0.4358665


def draw_states(seed: int, n_species: int, n_states: int, T=(800.0, 2200.0),
                P_atm=(1.0, 50.0), dirichlet=0.3) -> Tuple[np.ndarray, np.ndarray]:
    """T ~ U[T], p ~ U[P_atm] atm, Y ~ Dirichlet(alpha) over all N species."""
    rng = np.random.default_rng(seed)
    T_s = rng.uniform(T[0], T[1], size=n_states)
    p_s = rng.uniform(P_atm[0], P_atm[1], size=n_states) * ATM
    Y = rng.dirichlet(np.full(n_species, dirichlet), size=n_states)  # (S, N)
    phi = np.empty((n_species, n_states), dtype=np.float64)
    phi[0] = T_s
    phi[1:] = Y[:, : n_species - 1].T
    return np.ascontiguousarray(phi), p_s


def config_states(cfg_id: int, n_states: int | None = None):
    c = WORKLOADS[cfg_id]
    n = c["n_states"] if n_states is None else n_states
    return draw_states(STATE_SEED_BASE + cfg_id, c["n_species"], n, c["T"],
                       c["P_atm"], c["dirichlet"])


def draw_newton_inputs(seed: int, n_species: int, n_states: int,
                       h_range=(1e-9, 1e-5)):
    """Per-state step size h (log-uniform) and right-hand side b ~ N(0, 1),
    b laid out [N][n_states]."""
    rng = np.random.default_rng(seed)
    h = np.exp(rng.uniform(np.log(h_range[0]), np.log(h_range[1]), size=n_states))
    rhs = rng.standard_normal((n_species, n_states))
    return h, np.ascontiguousarray(rhs)


def conditioned_steps(seed: int, jac_rows: np.ndarray, c_range=(1.0, 3.0e3),
                      gamma: float = NEWTON_GAMMA) -> np.ndarray:
    """Per-state step h_s = c_s / (gamma ||J_s||_inf) with c_s log-uniform on
    c_range, so that I - h gamma J stays solvable (kappa_inf roughly c^2).
    jac_rows: absolute row sums of each state's Jacobian, shape (N, n)."""
    rng = np.random.default_rng(seed)
    n = jac_rows.shape[1]
    c = np.exp(rng.uniform(np.log(c_range[0]), np.log(c_range[1]), size=n))
    return c / (gamma * np.max(jac_rows, axis=0))


def pasr_fresh(mech, T_in: float, seed: int, inert_fraction: float = 0.72) -> np.ndarray:
    """Fresh inflow composition of a premixed PaSR (App. C) for a synthetic
    mechanism, shaped like a fuel/air mixture: the inert last species carries
    `inert_fraction` of the mass (the N2 of air), three seeded species share
    the rest, every other species holds a trace of 1e-9.  Returns
    [T_in, Y_1..Y_{N-1}]."""
    rng = np.random.default_rng(seed)
    N = mech.n_species
    Y = np.full(N, 1e-9)
    major = rng.choice(N - 1, 3, replace=False)
    Y[major] = rng.dirichlet(np.full(3, 2.0)) * (1.0 - inert_fraction)
    Y[N - 1] = 0.0
    Y[N - 1] = 1.0 - Y.sum()
    return np.concatenate([[T_in], Y[:-1]])
