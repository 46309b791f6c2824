"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: the Jacobian is checked against
complex-step and extended-precision Richardson finite differences of the RHS;
K_c against the paper's second (B_k) formula path; NASA thermo against the
thermodynamic derivative relations; rate expressions against special cases that
reduce to closed forms (trigonometric Chebyshev identity, PLOG grid points,
falloff limits, Troe A = 0, SRI P_r = 1); net rates against constructed chemical
equilibrium and element/mass conservation.  A plausible slip anywhere in the
oracle (a dropped term, a wrong sign or index) fails at least one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from conftest import ALL_KINDS, tiny
from synth import ATM, draw_states

R = 8314.462618
PATM = 101325.0


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def enorm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def per_state_enorm(J, Jref, N):
    return np.array([enorm(J[:, s], Jref[:, s]) for s in range(J.shape[1])])


# ------------------------------------------------------------------ Jacobian
@pytest.mark.parametrize("kind", ALL_KINDS)
@pytest.mark.parametrize("rev", ["kc", "explicit", "irrev"])
def test_jacobian_vs_complex_step_each_class(Ref, kind, rev):
    """Sec. 3.1 analytical Jacobian equals the complex-step derivative of the RHS
    (Sec. 2) for each reaction class alone, with each reverse-rate treatment."""
    mech = tiny(101 + ALL_KINDS.index(kind), {kind: 2, "elementary": 1},
                rev_mix={rev: 1.0})
    m = Ref(text=mech.to_text())
    phi, p = draw_states(7, m.n_species, 12, T=(700.0, 2400.0), P_atm=(0.3, 80.0),
                         dirichlet=0.6)
    J = m.eval_jacobian(phi, p)
    Jcs = m.eval_jacobian_cs(phi, p)
    assert per_state_enorm(J, Jcs, m.n_species).max() < 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_jacobian_vs_complex_step_mixed(Ref, seed):
    """Mixed mechanisms, including a reactive last species and species that appear
    on both sides of a reaction (nu_ki = 0 but [X] still enters R_i)."""
    rng = np.random.default_rng(seed)
    kinds = {k: int(rng.integers(0, 2)) for k in ALL_KINDS}
    kinds["elementary"] += 2
    mech = tiny(200 + seed, kinds, n_species=8, reactive_last=(seed % 2 == 0),
                rev_mix={"kc": 2, "explicit": 1, "irrev": 1}, allow_shared=(seed % 3 == 0))
    m = Ref(text=mech.to_text())
    phi, p = draw_states(seed, m.n_species, 10, T=(700.0, 2400.0), P_atm=(0.3, 80.0),
                         dirichlet=0.4)
    J = m.eval_jacobian(phi, p)
    Jcs = m.eval_jacobian_cs(phi, p)
    assert per_state_enorm(J, Jcs, m.n_species).max() < 1e-12


def test_jacobian_vs_richardson_fd(Ref):
    """Central differences in long double with 4-level Richardson extrapolation
    (an independent numerical derivative, no complex arithmetic)."""
    mech = tiny(31, {"elementary": 3, "thirdbody": 1, "falloff_troe": 1, "chemact_sri": 1,
                     "plog": 1, "cheb": 1}, rev_mix={"kc": 1.0})
    m = Ref(text=mech.to_text())
    N = m.n_species
    phi, p = draw_states(3, N, 4, T=(900.0, 2000.0), P_atm=(1.0, 20.0), dirichlet=1.0)
    J = m.eval_jacobian(phi, p)
    for s in range(phi.shape[1]):
        x0 = phi[:, s].astype(np.longdouble)
        Jfd = np.zeros((N, N))
        for j in range(N):
            base = (1e-3 * x0[0]) if j == 0 else 1e-3 * x0[j]
            hs = [base / 2 ** q for q in range(4)]
            cols = []
            for h in hs:
                plus = x0.copy(); plus[j] += h
                minus = x0.copy(); minus[j] -= h
                X = np.stack([plus, minus], axis=1)
                f = m.eval_rhs_ld(X, np.array([p[s], p[s]]))
                cols.append((f[:, 0] - f[:, 1]) / (2 * h))
            # Richardson table for an h^2 error expansion, step ratio 2
            T = [list(cols)]
            for lev in range(1, 4):
                fac = np.longdouble(4.0) ** lev
                T.append([(fac * T[lev - 1][q + 1] - T[lev - 1][q]) / (fac - 1)
                          for q in range(len(T[lev - 1]) - 1)])
            Jfd[:, j] = np.asarray(T[3][0], dtype=np.float64)
        Js = J[:, s].reshape(N, N)
        assert enorm(Js, Jfd) < 1e-8


def test_jacobian_invariants(Ref):
    """Element conservation carries over to the Jacobian: with an inert last species,
    sum_k a_ek/W_k * J[k+1, j] = 0 for every column; and the energy identity
    c_p J[0,j] + dc_p/dPhi_j f_0 + sum_k h_k J[k+1,j] + sum_k dh_k/dPhi_j f_k = 0."""
    mech = tiny(41, {"elementary": 4, "thirdbody": 1, "falloff_troe": 1, "falloff_sri": 1,
                     "chemact_lindemann": 1, "plog": 1, "cheb": 1})
    m = Ref(text=mech.to_text())
    N = m.n_species
    phi, p = draw_states(5, N, 6, T=(800.0, 2200.0), P_atm=(1.0, 50.0), dirichlet=0.5)
    J = m.eval_jacobian(phi, p)
    out = m.eval_rates(phi, p)
    a = mech.element_matrix()
    W = mech.molecular_weights()
    for s in range(phi.shape[1]):
        Js = J[:, s].reshape(N, N)
        scale = np.abs(Js[1:, :]).max() * np.abs(a / W).max()
        for e in range(a.shape[0]):
            col = (a[e, :N - 1] / W[: N - 1]) @ Js[1:, :]
            assert np.abs(col).max() < 1e-12 * scale * N
        # energy identity, mass units; h_k, c_p,k from the NASA values
        T = phi[0, s]
        cpR, hRT, _ = m.species_thermo(T)
        cpk = cpR * R / W
        hk = hRT * R * T / W
        Y = np.append(phi[1:, s], 1 - phi[1:, s].sum())
        cp = Y @ cpk
        f = out["dphi"][:, s]
        fN = W[N - 1] * out["wdot"][N - 1, s] / 1.0   # zero for the inert last species
        assert fN == 0.0
        fk = f[1:]
        # d c_p / dT: differentiate the NASA c_p numerically in mpmath (independent of oracle)
        def cp_mix(TT):
            cc = np.array([float(v) for v in m.species_thermo(TT)[0]]) * R / W
            return Y @ cc
        dcpdT = (cp_mix(T + 1e-3) - cp_mix(T - 1e-3)) / 2e-3
        dcp = np.concatenate([[dcpdT], cpk[: N - 1] - cpk[N - 1]])
        dh0 = cpk  # dh_k/dT
        for j in range(N):
            lhs = cp * Js[0, j] + dcp[j] * f[0] + hk[: N - 1] @ Js[1:, j]
            if j == 0:
                lhs += dh0[: N - 1] @ fk
            ref = abs(cp * Js[0, j]) + abs(dcp[j] * f[0]) + np.abs(hk[: N - 1] * Js[1:, j]).sum()
            assert abs(lhs) <= 1e-7 * ref + 1e-300


# -------------------------------------------------------------------- thermo
def test_nasa_thermo_derivative_relations(Ref):
    """d(H/R)/dT = C_p/R and d(S/R)/dT = C_p/(R T) for every species and both ranges
    (Sec. 2.2); also continuity of the generated fits at T_mid."""
    mech = tiny(51, {"elementary": 3})
    m = Ref(text=mech.to_text())
    for T in (350.0, 640.0, 999.0, 1001.0, 1700.0, 2900.0):
        d = 1e-4
        cp, _, _ = m.species_thermo(T)
        hp = m.species_thermo(T + d)[1] * (T + d)
        hm = m.species_thermo(T - d)[1] * (T - d)
        sp_, sm = m.species_thermo(T + d)[2], m.species_thermo(T - d)[2]
        np.testing.assert_allclose((hp - hm) / (2 * d), cp, rtol=1e-7)
        np.testing.assert_allclose((sp_ - sm) / (2 * d), cp / T, rtol=1e-7)
    lo = m.species_thermo(1000.0)
    hi = m.species_thermo(1000.0 + 1e-9)
    for a, b in zip(lo, hi):
        np.testing.assert_allclose(a, b, rtol=1e-8)


# -------------------------------------------------------- rate coefficients
def _single(kind, seed=61, **kw):
    return tiny(seed, {kind: 1}, **kw)


def test_arrhenius_cost_forms(Ref):
    """Eq. (kf_cost): exp(log A + beta log T - T_a/T) equals the plain form."""
    mech = tiny(62, {"elementary": 3})
    m = Ref(text=mech.to_text())
    y = np.full(m.n_species - 1, 1.0 / m.n_species)
    for T in (500.0, 1300.0, 2200.0):
        kf = m.reaction_terms(T, ATM, y)["kf"]
        for i, r in enumerate(mech.reactions):
            A, b, Ta = r.arr
            ref = mp.exp(mp.log(A) + b * mp.log(T) - mp.mpf(Ta) / T)
            assert abs(kf[i] - float(ref)) <= 1e-13 * float(ref)


def test_equilibrium_constant_two_paths(Ref):
    """K_c from Delta S - Delta H (oracle) equals the paper's B_k form, Sec. 2.3.1:
    K_c = (p_atm/R)^{sum nu} exp(sum nu_k B_k), evaluated here in mpmath."""
    mech = tiny(63, {"elementary": 4, "thirdbody": 1})
    m = Ref(text=mech.to_text())
    y = np.full(m.n_species - 1, 1.0 / m.n_species)
    nf, nr = mech.stoich()
    nu = nr - nf
    mp.mp.dps = 40
    for T in (600.0, 1000.0, 1500.0, 2400.0):
        Kc = m.reaction_terms(T, ATM, y)["Kc"]
        Tm = mp.mpf(T)
        for i in range(m.n_reactions):
            s = mp.mpf(0)
            for k in range(m.n_species):
                if nu[k, i] == 0:
                    continue
                sp = mech.species[k]
                a = [mp.mpf(v) for v in (sp.low if T <= sp.tmid else sp.high)]
                B = (a[6] - a[0] + (a[0] - 1) * mp.log(Tm)
                     + Tm * (a[1] / 2 + Tm * (a[2] / 6 + Tm * (a[3] / 12 + a[4] / 20 * Tm)))
                     - a[5] / Tm)
                s += nu[k, i] * B
            ref = (mp.mpf(PATM) / R) ** int(nu[:, i].sum()) * mp.exp(s)
            assert abs(Kc[i] - float(ref)) <= 1e-12 * abs(float(ref))


def test_constructed_equilibrium_zero_net_rates(Ref):
    """Pick T and element potentials lambda_e, set [X_k] = (p_atm/RT)
    exp(-G_k/RT + sum_e a_ek lambda_e).  Element balance makes every K_c-reversible
    reaction satisfy prod [X]^nu = K_c, so R_f = R_r and wdot = 0."""
    mech = tiny(64, {"elementary": 5, "thirdbody": 1, "falloff_troe": 1, "chemact_sri": 1,
                     "plog": 1, "cheb": 1})
    m = Ref(text=mech.to_text())
    a = mech.element_matrix()
    W = mech.molecular_weights()
    rng = np.random.default_rng(3)
    mp.mp.dps = 40
    for T in (900.0, 1500.0, 2100.0):
        lam = rng.uniform(-3, 3, size=a.shape[0])
        X = []
        for k, sp in enumerate(mech.species):
            c = [mp.mpf(v) for v in (sp.low if T <= sp.tmid else sp.high)]
            Tm = mp.mpf(T)
            H = Tm * (c[0] + Tm * (c[1] / 2 + Tm * (c[2] / 3 + Tm * (c[3] / 4 + c[4] / 5 * Tm)))) + c[5]
            S = c[0] * mp.log(Tm) + Tm * (c[1] + Tm * (c[2] / 2 + Tm * (c[3] / 3 + c[4] / 4 * Tm))) + c[6]
            g = H / Tm - S
            X.append(mp.mpf(PATM) / (R * Tm) * mp.exp(-g + sum(int(a[e, k]) * lam[e]
                                                                for e in range(a.shape[0]))))
        X = np.array([float(x) for x in X])
        rho = (X * W).sum()
        p = R * T * X.sum()
        Y = X * W / rho
        terms = m.reaction_terms(T, p, Y[:-1])
        Rf, Rr = terms["Rf"], terms["Rr"]
        assert np.all(np.abs(Rf - Rr) <= 1e-10 * np.maximum(Rf, Rr))
        phi = np.concatenate([[T], Y[:-1]])[:, None]
        out = m.eval_rates(phi, np.array([p]))
        nf, nr = mech.stoich()
        gross = np.abs(nr - nf) @ (np.abs(out["pres_mod"][:, 0]) * (Rf + Rr))
        assert np.all(np.abs(out["wdot"][:, 0]) <= 1e-10 * gross + 1e-300)


def test_conservation_of_elements_and_mass(Ref):
    mech = tiny(65, {"elementary": 5, "thirdbody": 2, "falloff_lindemann": 1, "falloff_troe": 1,
                     "chemact_troe": 1, "plog": 1, "cheb": 1})
    m = Ref(text=mech.to_text())
    phi, p = draw_states(9, m.n_species, 20, dirichlet=0.3)
    out = m.eval_rates(phi, p)
    a = mech.element_matrix()
    W = mech.molecular_weights()
    nf, nr = mech.stoich()
    gross = np.abs(nr - nf) @ (np.abs(out["pres_mod"]) * (out["rop_f"] + out["rop_r"]))
    wd = out["wdot"]
    for e in range(a.shape[0]):
        tot = a[e] @ wd
        ref = a[e] @ gross
        assert np.all(np.abs(tot) <= 1e-13 * ref + 1e-300)
    assert np.all(np.abs(W @ wd) <= 1e-13 * (W @ gross) + 1e-300)
    # RHS for species equals W_k wdot_k / rho and sums to -W_N wdot_N / rho = 0 (inert)
    assert np.all(np.abs(out["dphi"][1:].sum(axis=0)) <= 1e-13 * np.abs(out["dphi"][1:]).sum(axis=0))


def test_plog_grid_points_and_single_point(Ref):
    """PLOG (Sec. 2.3.4): at p = p_n the rate is that point's Arrhenius rate; a
    single-point PLOG is plain Arrhenius; between points log k is linear in log p;
    outside the grid the end point is used."""
    mech = tiny(66, {"plog": 2})
    m = Ref(text=mech.to_text())
    y = np.full(m.n_species - 1, 1.0 / m.n_species)
    T = 1234.5
    for i, r in enumerate(mech.reactions):
        pts = sorted(r.plog)
        arr = [A * T ** b * math.exp(-Ta / T) for _, A, b, Ta in pts]
        for (pn, *_), kn in zip(pts, arr):
            kf = m.reaction_terms(T, pn, y)["kf"][i]
            assert abs(kf - kn) <= 1e-12 * kn
        kf_lo = m.reaction_terms(T, pts[0][0] / 10, y)["kf"][i]
        kf_hi = m.reaction_terms(T, pts[-1][0] * 10, y)["kf"][i]
        assert abs(kf_lo - arr[0]) <= 1e-12 * arr[0]
        assert abs(kf_hi - arr[-1]) <= 1e-12 * arr[-1]
        if len(pts) > 1:
            pm = math.sqrt(pts[0][0] * pts[1][0])
            kf = m.reaction_terms(T, pm, y)["kf"][i]
            assert abs(math.log(kf) - 0.5 * (math.log(arr[0]) + math.log(arr[1]))) < 1e-11


def test_chebyshev_trig_identity(Ref):
    """Chebyshev (Sec. 2.3.4): with a single nonzero coefficient eta_{i1},
    log10 k = eta cos((i-1) theta) where T~ = cos(theta) -- the defining identity
    T_n(cos t) = cos(n t), evaluated with no polynomial code at all."""
    from synth.mechgen import Mechanism, Reaction
    base = tiny(67, {"cheb": 1})
    r = base.reactions[0]
    p = math.sqrt(r.cheb["Pmin"] * r.cheb["Pmax"])     # p~ = 0
    for deg in range(r.cheb["nT"]):
        coef = np.zeros((r.cheb["nT"], r.cheb["nP"]))
        coef[deg, 0] = 1.7
        r.cheb = dict(r.cheb, coef=coef)
        m = Ref(text=base.to_text())
        y = np.full(m.n_species - 1, 1.0 / m.n_species)
        for theta in (0.3, 1.1, 2.5):
            x = math.cos(theta)
            a, b = 1 / r.cheb["Tmin"], 1 / r.cheb["Tmax"]
            Tinv = (x * (b - a) + a + b) / 2
            kf = m.reaction_terms(1 / Tinv, p, y)["kf"][0]
            assert abs(math.log10(kf) - 1.7 * math.cos(deg * theta)) < 1e-12


def test_falloff_limits_and_special_points(Ref):
    """Falloff (Sec. 2.3.3): Troe F = F_cent exactly where A_Troe = 0; SRI at P_r = 1
    gives F = d T^e (a e^{-b/T} + e^{-T/c}); Lindemann c = P_r/(1+P_r) tends to
    k0[M]/kinf at low pressure; chemically activated q tends to k0 prod[X] as P_r -> 0."""
    T = 1400.0
    # Troe
    mech = tiny(68, {"falloff_troe": 1}, collider_probs=(1.0, 0.0))
    r = mech.reactions[0]
    m = Ref(text=mech.to_text())
    y = np.full(m.n_species - 1, 1.0 / m.n_species)
    a, T3, T1 = r.troe[:3]
    Fc = (1 - a) * math.exp(-T / T3) + a * math.exp(-T / T1)
    if len(r.troe) > 3:
        Fc += math.exp(-r.troe[3] / T)
    Pr_target = 10 ** (0.4 + 0.67 * math.log10(Fc))
    k0 = r.low[0] * T ** r.low[1] * math.exp(-r.low[2] / T)
    ki = r.high[0] * T ** r.high[1] * math.exp(-r.high[2] / T)
    p = Pr_target * R * T * ki / k0          # all-unity collider: [M] = p/RT
    t = m.reaction_terms(T, p, y)
    assert abs(t["Pr"][0] / Pr_target - 1) < 1e-12
    assert abs(t["F"][0] / Fc - 1) < 1e-12
    assert abs(t["c"][0] - Pr_target / (1 + Pr_target) * Fc) < 1e-12 * t["c"][0]
    # SRI at P_r = 1
    mech = tiny(69, {"falloff_sri": 1}, collider_probs=(1.0, 0.0))
    r = mech.reactions[0]
    m = Ref(text=mech.to_text())
    sa, sb, sc, sd, se = r.sri
    k0 = r.low[0] * T ** r.low[1] * math.exp(-r.low[2] / T)
    ki = r.high[0] * T ** r.high[1] * math.exp(-r.high[2] / T)
    p = R * T * ki / k0
    t = m.reaction_terms(T, p, y)
    Fref = sd * T ** se * (sa * math.exp(-sb / T) + math.exp(-T / sc))
    assert abs(t["Pr"][0] - 1) < 1e-12
    assert abs(t["F"][0] / Fref - 1) < 1e-12
    # Lindemann low-pressure limit and chemically-activated limit
    for kind, seed in (("falloff_lindemann", 70), ("chemact_lindemann", 71)):
        mech = tiny(seed, {kind: 1}, collider_probs=(1.0, 0.0))
        r = mech.reactions[0]
        m = Ref(text=mech.to_text())
        k0 = r.low[0] * T ** r.low[1] * math.exp(-r.low[2] / T)
        ki = r.high[0] * T ** r.high[1] * math.exp(-r.high[2] / T)
        p = 1e-9 * R * T * ki / k0              # P_r = 1e-9
        t = m.reaction_terms(T, p, y)
        M = p / (R * T)
        if kind.startswith("falloff"):
            # q -> k0 [M] prod[X]:  c * kf = Pr/(1+Pr) kinf -> k0 [M]
            assert abs(t["c"][0] * t["kf"][0] / (k0 * M) - 1) < 2e-9
        else:
            assert abs(t["c"][0] * t["kf"][0] / k0 - 1) < 2e-9
