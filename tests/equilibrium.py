"""Constructed chemical-equilibrium states (test input helper).

For a temperature T and element potentials lambda_e, the concentrations
  [X_k] = (p_atm / R T) exp(-G_k/RT + sum_e a_ek lambda_e),
with G_k/RT = H_k/RT - S_k/R from the species' NASA-7 polynomials (Sec. 2.2),
satisfy prod_k [X_k]^nu_ki = K_c,i for every element-balanced reaction
(Sec. 2.3.1), so every K_c-reversible reaction has R_f = R_r.  The potentials
are shifted by a common lambda_0, found by bisection, so that the pressure
R T sum [X_k] lands on a chosen value: every species holds at least one atom,
so the pressure grows monotonically with lambda_0.

Evaluated in mpmath (40 digits) so that the states are at equilibrium to well
below FP64 rounding of the rates.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

R = 8314.462618
PATM = 101325.0


def _g_over_RT(sp, T):
    c = [mp.mpf(v) for v in (sp.low if T <= sp.tmid else sp.high)]
    Tm = mp.mpf(T)
    H = Tm * (c[0] + Tm * (c[1] / 2 + Tm * (c[2] / 3 + Tm * (c[3] / 4 + c[4] / 5 * Tm)))) + c[5]
    S = c[0] * mp.log(Tm) + Tm * (c[1] + Tm * (c[2] / 2 + Tm * (c[3] / 3 + c[4] / 4 * Tm))) + c[6]
    return H / Tm - S


def equilibrium_states(mech, n, seed, T=(900.0, 2100.0), P_atm=(1.0, 50.0), spread=2.0):
    """n equilibrium states of the mechanism: phi[N][n] (T, Y_1..Y_{N-1}), p[n]."""
    mp.mp.dps = 40
    rng = np.random.default_rng(seed)
    a = mech.element_matrix()
    W = mech.molecular_weights()
    N = mech.n_species
    natoms = a.sum(axis=0)
    assert np.all(natoms > 0)
    phi = np.empty((N, n))
    p = np.empty(n)
    for s in range(n):
        Ts = float(rng.uniform(*T))
        lam = rng.uniform(-spread, spread, size=a.shape[0])
        target = mp.mpf(float(rng.uniform(*P_atm)) * PATM)
        base = [-_g_over_RT(sp, Ts) + sum(int(a[e, k]) * lam[e] for e in range(a.shape[0]))
                for k, sp in enumerate(mech.species)]
        c0 = mp.mpf(PATM) / (R * mp.mpf(Ts))

        def conc(l0):
            return [c0 * mp.exp(b + int(natoms[k]) * l0) for k, b in enumerate(base)]

        def pres(l0):
            return R * mp.mpf(Ts) * mp.fsum(conc(l0))

        lo, hi = mp.mpf(-400), mp.mpf(400)
        for _ in range(200):
            mid = (lo + hi) / 2
            if pres(mid) < target:
                lo = mid
            else:
                hi = mid
        X = conc((lo + hi) / 2)
        rho = mp.fsum(x * mp.mpf(float(w)) for x, w in zip(X, W))
        Y = [x * mp.mpf(float(w)) / rho for x, w in zip(X, W)]
        phi[0, s] = Ts
        phi[1:, s] = [float(y) for y in Y[:-1]]
        p[s] = float(R * mp.mpf(Ts) * mp.fsum(X))
    return np.ascontiguousarray(phi), p
