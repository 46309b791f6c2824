"""Oracle of the PaSR mixing fractional step (App. C) -- test infrastructure only.

Plain per-particle loops: mixture enthalpy h = sum_k Y_k h_k(T) from the
oracle's NASA-7 polynomials (Sec. 2.2), pairwise relaxation
x_s <- x_s - w (x_s - x_q) of (h, Y_1..Y_N), and the temperature from the
mixed enthalpy by Newton's method.
"""
from __future__ import annotations

import numpy as np

R = 8314.462618


def mixture_enthalpy(ref, W, T, Y):
    """Mass-specific enthalpy and heat capacity of composition Y (all N) at T."""
    cpR, hRT, _ = ref.species_thermo(T)
    h = float(np.sum(Y * hRT * R * T / W))
    cp = float(np.sum(Y * cpR * R / W))
    return h, cp


def temperature_from_enthalpy(ref, W, h, Y, T0, tol=1e-13, max_iter=100):
    T = T0
    for _ in range(max_iter):
        hh, cp = mixture_enthalpy(ref, W, T, Y)
        dT = (h - hh) / cp
        T += dT
        if abs(dT) <= tol * T:
            break
    return T


def mix_pairs(ref, W, phi, partner, w):
    """phi [N, n] (T, Y_1..Y_{N-1}); partner [n]; returns the mixed states."""
    N, n = phi.shape
    out = phi.copy()
    for s in range(n):
        q = int(partner[s])
        if q < 0:
            continue
        Ys = np.append(phi[1:, s], 1.0 - phi[1:, s].sum())
        Yq = np.append(phi[1:, q], 1.0 - phi[1:, q].sum())
        hs, _ = mixture_enthalpy(ref, W, phi[0, s], Ys)
        hq, _ = mixture_enthalpy(ref, W, phi[0, q], Yq)
        Ym = Ys - w * (Ys - Yq)
        hm = hs - w * (hs - hq)
        T0 = phi[0, s] - w * (phi[0, s] - phi[0, q])
        out[0, s] = temperature_from_enthalpy(ref, W, hm, Ym, T0)
        out[1:, s] = Ym[:-1]
    return out
