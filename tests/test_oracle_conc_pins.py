"""Pins of the oracle's constant-volume, concentration-based form (Sec. 3.3:
the formulation with molar concentrations as state variables, whose Jacobian
is sparse; planned in Sec. 6).

State Phi_C = {T, [X_1], ..., [X_N]}, d[X_k]/dt = wdot_k and
dT/dt = -sum U_k wdot_k / sum [X_k] C_v,k at constant volume.  The analytical
Jacobian is pinned by
  * the complex-step derivative of the oracle's RHS (every reaction class,
    PLOG and Chebyshev pressure dependence, absent colliders);
  * mass and element conservation of every Jacobian column;
  * the energy identity of the temperature row;
  * the chain rule to the (separately pinned) constant-pressure, mass-fraction
    Jacobian at the same state: d wdot / dY at fixed T, p equals the
    concentration-form block times d[X]/dY, and likewise for d wdot / dT.
"""
import numpy as np
import pytest

from conftest import ALL_KINDS, BLENDED, species_collider_mech, tiny, zero_collider_states
from synth import config_mechanism, config_states, draw_states

R = 8314.462618


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def conc_states(mech, phi, p):
    """(T, p, Y_1..Y_{N-1}) -> Phi_C = (T, [X_1..X_N])."""
    W = mech.molecular_weights()
    Y = np.vstack([phi[1:], 1 - phi[1:].sum(axis=0)])
    rho = p / (R * phi[0] * (Y / W[:, None]).sum(axis=0))
    return np.vstack([phi[:1], rho * Y / W[:, None]])


def enorm(A, B):
    sc = np.max(np.abs(B), axis=0)
    sc[sc == 0] = 1
    return np.linalg.norm((A - B) / sc, axis=0) / np.linalg.norm(B / sc, axis=0)


CASES = [(k, {k: 2, "elementary": 1}) for k in ALL_KINDS] + [(f"mixed{s}", None) for s in range(4)]


@pytest.mark.parametrize("name,kinds", CASES, ids=[c[0] for c in CASES])
def test_conc_jacobian_matches_complex_step(Ref, name, kinds):
    if kinds is None:
        s = int(name[5:])
        rng = np.random.default_rng(910 + s)
        kinds = {k: int(rng.integers(0, 2)) for k in ALL_KINDS}
        kinds["elementary"] += 2
        mech = tiny(720 + s, kinds, n_species=8, reactive_last=(s % 2 == 0),
                    rev_mix={"kc": 2, "explicit": 1, "irrev": 1})
    else:
        mech = tiny(540 + ALL_KINDS.index(name), kinds, rev_mix={"kc": 1.0})
    phi, p = draw_states(21, mech.n_species, 40, T=(700.0, 2400.0), P_atm=(0.3, 80.0), dirichlet=0.5)
    m = Ref(text=mech.to_text())
    c = conc_states(mech, phi, p)
    J, Jcs = m.eval_jacobian_conc(c), m.eval_jacobian_conc_cs(c)
    assert np.all(np.isfinite(J))
    e = enorm(J, Jcs)
    assert e.max() < 1e-12, (name, e.max())


@pytest.mark.parametrize("cfg,n", [(0, 30), (1, 6), (2, 3)])
def test_conc_jacobian_full_mechanisms(Ref, cfg, n):
    mech = config_mechanism(cfg)
    phi, p = config_states(cfg, n)
    m = Ref(text=mech.to_text())
    c = conc_states(mech, phi, p)
    e = enorm(m.eval_jacobian_conc(c), m.eval_jacobian_conc_cs(c))
    assert e.max() < 1e-11, e.max()


@pytest.mark.parametrize("kind", BLENDED)
def test_conc_absent_collider(Ref, kind):
    mech, m_sp = species_collider_mech(kind, 150 + BLENDED.index(kind))
    phi, p = zero_collider_states(mech, m_sp, 9)
    m = Ref(text=mech.to_text())
    c = conc_states(mech, phi, p)
    c[1 + m_sp] = np.where(phi[1 + m_sp] == 0, 0.0, c[1 + m_sp])
    J, Jcs = m.eval_jacobian_conc(c), m.eval_jacobian_conc_cs(c)
    assert np.all(np.isfinite(J))
    assert enorm(J, Jcs).max() < 1e-12


def test_conc_conservation_and_energy(Ref):
    mech = config_mechanism(1)
    N = mech.n_species
    phi, p = config_states(1, 8)
    m = Ref(text=mech.to_text())
    c = conc_states(mech, phi, p)
    J = m.eval_jacobian_conc(c).reshape(N + 1, N + 1, -1)
    f = m.eval_rhs_conc(c)
    W = mech.molecular_weights()
    a = mech.element_matrix()
    rows = J[1:]                                         # d wdot_k / d Phi_j
    scale = np.abs(W[:, None, None] * rows).sum(axis=0)
    assert np.all(np.abs((W[:, None, None] * rows).sum(axis=0)) <= 1e-13 * scale)
    for e in range(a.shape[0]):
        s_e = (a[e][:, None, None] * rows)
        assert np.all(np.abs(s_e.sum(axis=0)) <= 1e-13 * np.abs(s_e).sum(axis=0) + 1e-300)
    # energy identity: D J_0j + dD/dPhi_j f_0 + sum U_k J_kj + sum dU_k/dPhi_j wdot_k = 0
    for s in range(c.shape[1]):
        T = c[0, s]
        cpR, hRT, _ = m.species_thermo(T)
        U, Cv = R * T * (hRT - 1), R * (cpR - 1)
        h = 1e-3
        cpp, _, _ = m.species_thermo(T + h)
        cpm, _, _ = m.species_thermo(T - h)
        dCv = R * (cpp - cpm) / (2 * h)
        C = c[1:, s]
        D = (C * Cv).sum()
        dD = np.concatenate([[(C * dCv).sum()], Cv])
        dUw = np.concatenate([[(Cv * f[1:, s]).sum()], np.zeros(N)])
        lhs = D * J[0, :, s] + dD * f[0, s] + U @ J[1:, :, s] + dUw
        gross = np.abs(D * J[0, :, s]) + np.abs(U) @ np.abs(J[1:, :, s])
        assert np.all(np.abs(lhs) <= 1e-8 * gross), np.max(np.abs(lhs) / gross)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_chain_rule_to_mass_fraction_form(Ref, cfg):
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, 5)
    m = Ref(text=mech.to_text())
    c = conc_states(mech, phi, p)
    Jc = m.eval_jacobian_conc(c).reshape(N + 1, N + 1, -1)
    Jp = m.eval_jacobian(phi, p).reshape(N, N, -1)
    wdot = m.eval_rates(phi, p)["wdot"]
    W = mech.molecular_weights()
    for s in range(phi.shape[1]):
        T, C = phi[0, s], c[1:, s]
        rho = (C * W).sum()
        Wmix = rho / C.sum()
        v = 1 / W[:-1] - 1 / W[-1]
        # d[X_l]/dY_j at fixed T, p (j = 1..N-1) and d[X_l]/dT at fixed p, Y
        dC = np.zeros((N, N - 1))
        for j in range(N - 1):
            dC[:, j] = -C * Wmix * v[j]
            dC[j, j] += rho / W[j]
            dC[N - 1, j] -= rho / W[N - 1]
        dwdY_conc = Jc[1:, 1:, s] @ dC
        dwdT_conc = Jc[1:, 0, s] + Jc[1:, 1:, s] @ (-C / T)
        # the same derivatives from the constant-pressure, mass-fraction Jacobian
        wd = wdot[:, s]
        dwdY_mass = rho / W[:-1, None] * (Jp[1:, 1:, s] - (W[:-1] * wd[:-1])[:, None] * (R * T / p[s]) * v[None, :])
        dwdT_mass = rho / W[:-1] * (Jp[1:, 0, s] - W[:-1] * wd[:-1] / (rho * T))
        sc = np.abs(Jc[1:, 1:, s]) @ np.abs(dC)
        assert np.all(np.abs(dwdY_conc[:-1] - dwdY_mass) <= 1e-10 * sc[:-1] + 1e-300)
        scT = np.abs(Jc[1:, 0, s]) + np.abs(Jc[1:, 1:, s]) @ np.abs(C / T)
        assert np.all(np.abs(dwdT_conc[:-1] - dwdT_mass) <= 1e-10 * scT[:-1] + 1e-300)
