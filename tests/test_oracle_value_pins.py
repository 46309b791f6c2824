"""Value pins of the oracle's rate expressions at points away from the trivial ones.

Every expected value here comes from the paper's definitions evaluated in
mpmath (40 digits) with the printed constants typed into this file, or from a
special point where the definition collapses to a closed form:
  * Troe (Sec. 2.3.3) where A = B and A = -B (then F = F_cent^(1/2)), and at
    generic P_r with and without the T** term;
  * SRI (Sec. 2.3.3) at P_r = 10 and 0.1 (then X = 1/2);
  * Chebyshev (Sec. 2.3.4) along the pressure axis: log10 k = eta cos(j theta)
    at p~ = cos(theta), and a mixed coefficient as a product of cosines;
  * the five cases of Eq. (kf_cost) (Sec. 2.3);
  * P_r -> infinity and P_r -> 0 limits of the blending (Sec. 2.3.3), and
    Lindemann as Troe with F_cent = 1;
  * an absent single-species collider (P_r = 0) gives finite rates and a
    Jacobian equal to the complex-step derivative of the RHS (Sec. 3.1).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from conftest import BLENDED, species_collider_mech, tiny, zero_collider_states
from synth import ATM, draw_states

R = 8314.462618
mp.mp.dps = 40

# Sec. 2.3.3, Troe: A = log10 P_r - 0.67 log10 F_cent - 0.4,
#                   B = 0.806 - 1.1762 log10 F_cent - 0.14 log10 P_r
TROE_A = (1.0, -0.67, -0.4)        # coefficients of (log10 P_r, log10 F_cent, 1)
TROE_B = (-0.14, -1.1762, 0.806)


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def _arr(a, T):
    A, b, Ta = (mp.mpf(v) for v in a)
    return A * mp.mpf(T) ** b * mp.exp(-Ta / mp.mpf(T))


def _fcent(troe, T):
    T = mp.mpf(T)
    a, T3, T1 = (mp.mpf(v) for v in troe[:3])
    Fc = (1 - a) * mp.exp(-T / T3) + a * mp.exp(-T / T1)
    if len(troe) > 3:
        Fc += mp.exp(-mp.mpf(troe[3]) / T)
    return Fc


def _troe_F(troe, T, lPr):
    Fc = _fcent(troe, T)
    lF = mp.log10(Fc)
    A = TROE_A[0] * lPr + TROE_A[1] * lF + TROE_A[2]
    B = TROE_B[0] * lPr + TROE_B[1] * lF + TROE_B[2]
    return Fc ** (1 / (1 + (A / B) ** 2))


def _sri_F(sri, T, lPr):
    a, b, c, d, e = (mp.mpf(v) for v in sri)
    T = mp.mpf(T)
    X = 1 / (1 + lPr ** 2)
    return d * T ** e * (a * mp.exp(-b / T) + mp.exp(-T / c)) ** X


def _p_for_Pr(r, T, Pr):
    """Pressure at which an all-unity collider ([M] = p/RT) gives this P_r."""
    return float(mp.mpf(Pr) * R * T * _arr(r.high, T) / _arr(r.low, T))


def _uniform_y(m):
    return np.full(m.n_species - 1, 1.0 / m.n_species)


# ------------------------------------------------------------------------ Troe
@pytest.mark.parametrize("seed", [81, 82, 83, 84])
@pytest.mark.parametrize("sign", [1, -1])
def test_troe_where_A_equals_plus_minus_B(Ref, seed, sign):
    mech = tiny(seed, {"falloff_troe": 1}, collider_probs=(1.0, 0.0))
    r = mech.reactions[0]
    m = Ref(text=mech.to_text())
    for T in (900.0, 1600.0, 2300.0):
        lF = mp.log10(_fcent(r.troe, T))
        # A = sign * B, solved for log10 P_r
        lPr = (sign * (TROE_B[1] * lF + TROE_B[2]) - (TROE_A[1] * lF + TROE_A[2])) / \
              (TROE_A[0] - sign * TROE_B[0])
        A = TROE_A[0] * lPr + TROE_A[1] * lF + TROE_A[2]
        assert abs(A) > 0.05                        # away from the A = 0 point
        t = m.reaction_terms(T, _p_for_Pr(r, T, mp.mpf(10) ** lPr), _uniform_y(m))
        assert abs(t["Pr"][0] / float(mp.mpf(10) ** lPr) - 1) < 1e-12
        Fref = mp.sqrt(_fcent(r.troe, T))
        assert abs(t["F"][0] / float(Fref) - 1) < 1e-12, (T, t["F"][0], Fref)


@pytest.mark.parametrize("seed", [85, 86, 87])
def test_troe_generic_points(Ref, seed):
    mech = tiny(seed, {"falloff_troe": 1}, collider_probs=(1.0, 0.0))
    r = mech.reactions[0]
    m = Ref(text=mech.to_text())
    for T in (1100.0, 1900.0):
        for lPr in (-2.5, -0.7, 0.4, 1.8, 3.3):
            Pr = mp.mpf(10) ** lPr
            t = m.reaction_terms(T, _p_for_Pr(r, T, Pr), _uniform_y(m))
            Fref = _troe_F(r.troe, T, mp.log10(mp.mpf(t["Pr"][0])))
            assert abs(t["F"][0] / float(Fref) - 1) < 1e-12
            assert abs(t["c"][0] / float(Pr / (1 + Pr) * Fref) - 1) < 1e-11


def test_troe_with_second_temperature_term(Ref):
    for seed in range(88, 120):
        mech = tiny(seed, {"falloff_troe": 1}, collider_probs=(1.0, 0.0))
        if len(mech.reactions[0].troe) == 4:
            break
    r = mech.reactions[0]
    assert len(r.troe) == 4
    m = Ref(text=mech.to_text())
    T = 1450.0
    for lPr in (-1.0, 0.5, 2.0):
        t = m.reaction_terms(T, _p_for_Pr(r, T, mp.mpf(10) ** lPr), _uniform_y(m))
        Fref = _troe_F(r.troe, T, mp.log10(mp.mpf(t["Pr"][0])))
        assert abs(t["F"][0] / float(Fref) - 1) < 1e-12


# ------------------------------------------------------------------------- SRI
@pytest.mark.parametrize("seed", [121, 122, 123])
def test_sri_where_X_is_one_half(Ref, seed):
    mech = tiny(seed, {"falloff_sri": 1}, collider_probs=(1.0, 0.0))
    r = mech.reactions[0]
    m = Ref(text=mech.to_text())
    a, b, c, d, e = (mp.mpf(v) for v in r.sri)
    for T in (950.0, 1750.0):
        Tm = mp.mpf(T)
        for Pr in (10.0, 0.1):                      # log10 P_r = +-1: X = 1/2
            t = m.reaction_terms(T, _p_for_Pr(r, T, Pr), _uniform_y(m))
            Fref = d * Tm ** e * mp.sqrt(a * mp.exp(-b / Tm) + mp.exp(-Tm / c))
            assert abs(t["F"][0] / float(Fref) - 1) < 1e-12
        for lPr in (-3.0, 2.2):
            t = m.reaction_terms(T, _p_for_Pr(r, T, mp.mpf(10) ** lPr), _uniform_y(m))
            Fref = _sri_F(r.sri, T, mp.log10(mp.mpf(t["Pr"][0])))
            assert abs(t["F"][0] / float(Fref) - 1) < 1e-12


# ------------------------------------------------------------------- Chebyshev
def _cheb_mech(coef_setter):
    base = tiny(67, {"cheb": 1})
    r = base.reactions[0]
    coef = np.zeros((r.cheb["nT"], r.cheb["nP"]))
    coef_setter(coef)
    r.cheb = dict(r.cheb, coef=coef)
    return base, r


def _T_for(r, x):
    a, b = 1 / r.cheb["Tmin"], 1 / r.cheb["Tmax"]
    return 2 / (x * (b - a) + a + b)


def _p_for(r, x):
    lo, hi = math.log10(r.cheb["Pmin"]), math.log10(r.cheb["Pmax"])
    return 10 ** ((x * (hi - lo) + lo + hi) / 2)


def test_chebyshev_pressure_axis(Ref):
    """Only eta_{1j} set: log10 k = eta T_{j-1}(p~) = eta cos((j-1) theta) at
    p~ = cos(theta), for every pressure degree j."""
    probe, _ = _cheb_mech(lambda c: None)
    nP = probe.reactions[0].cheb["nP"]
    for deg in range(nP):
        mech, r = _cheb_mech(lambda c: c.__setitem__((0, deg), 1.3))
        m = Ref(text=mech.to_text())
        y = _uniform_y(m)
        for theta in (0.2, 1.0, 2.0, 2.9):
            kf = m.reaction_terms(1234.0, _p_for(r, math.cos(theta)), y)["kf"][0]
            assert abs(math.log10(kf) - 1.3 * math.cos(deg * theta)) < 1e-12


def test_chebyshev_mixed_coefficient(Ref):
    """A single eta_{ij} with i, j >= 2 gives eta cos((i-1) t1) cos((j-1) t2) at
    (T~, p~) = (cos t1, cos t2)."""
    probe, _ = _cheb_mech(lambda c: None)
    nT, nP = probe.reactions[0].cheb["nT"], probe.reactions[0].cheb["nP"]
    for i in range(1, nT):
        for j in range(1, nP):
            mech, r = _cheb_mech(lambda c: c.__setitem__((i, j), -0.9))
            m = Ref(text=mech.to_text())
            y = _uniform_y(m)
            for t1, t2 in ((0.4, 2.2), (1.9, 0.7)):
                kf = m.reaction_terms(_T_for(r, math.cos(t1)), _p_for(r, math.cos(t2)), y)["kf"][0]
                ref = -0.9 * math.cos(i * t1) * math.cos(j * t2)
                assert abs(math.log10(kf) - ref) < 1e-12


# ------------------------------------------------------------- Eq. (kf_cost)
def test_arrhenius_cost_cases(Ref):
    """The five cases of Eq. (kf_cost) against the plain Arrhenius form."""
    mech = tiny(62, {"elementary": 5})
    cases = [(3.7e8, 0.0, 0.0), (3.7e8, 1.3, 0.0), (3.7e8, 1.3, 9000.0),
             (3.7e8, 0.0, 9000.0), (3.7e8, 2.0, 0.0)]
    for r, a in zip(mech.reactions, cases):
        r.arr = a
    m = Ref(text=mech.to_text())
    y = _uniform_y(m)
    for T in (600.0, 1500.0):
        kf = m.reaction_terms(T, ATM, y)["kf"]
        Tm = mp.mpf(T)
        A = mp.mpf(3.7e8)
        forms = [A,
                 mp.exp(mp.log(A) + mp.mpf(1.3) * mp.log(Tm)),
                 mp.exp(mp.log(A) + mp.mpf(1.3) * mp.log(Tm) - 9000 / Tm),
                 mp.exp(mp.log(A) - 9000 / Tm),
                 A * Tm * Tm]
        for i, ref in enumerate(forms):
            assert abs(kf[i] / float(ref) - 1) < 1e-13, (i, T)


# ------------------------------------------------------------ falloff limits
def test_high_pressure_limits(Ref):
    """P_r -> infinity: falloff c k_f -> k_inf (Lindemann); a chemically
    activated reaction's c k_f = k_0 / (1 + P_r) -> k_inf / [X]."""
    T = 1300.0
    for kind, seed in (("falloff_lindemann", 131), ("chemact_lindemann", 132)):
        mech = tiny(seed, {kind: 1}, collider_probs=(1.0, 0.0))
        r = mech.reactions[0]
        m = Ref(text=mech.to_text())
        p = _p_for_Pr(r, T, 1e10)
        t = m.reaction_terms(T, p, _uniform_y(m))
        kinf = float(_arr(r.high, T))
        if kind.startswith("falloff"):
            assert abs(t["c"][0] * t["kf"][0] / kinf - 1) < 2e-10
        else:
            M = p / (R * T)
            assert abs(t["c"][0] * t["kf"][0] * M / kinf - 1) < 2e-10


@pytest.mark.parametrize("kind", ["falloff", "chemact"])
def test_lindemann_is_troe_with_unit_fcent(Ref, kind):
    """Troe with T*** = T* = 1e300 and no T** has F_cent = 1 to rounding, so
    F = 1: rates and Jacobian equal those of the Lindemann form."""
    mech = tiny(140, {f"{kind}_troe": 2, "elementary": 2}, collider_probs=(0.3, 0.3))
    for r in mech.reactions:
        if r.troe is not None:
            r.troe = (0.37, 1e300, 1e300)
    m_troe = Ref(text=mech.to_text())
    for r in mech.reactions:
        if r.troe is not None:
            r.troe = None
            r.kind = f"{kind}_lindemann"
    m_lind = Ref(text=mech.to_text())
    phi, p = draw_states(5, mech.n_species, 8, dirichlet=0.5)
    a, b = m_troe.eval_rates(phi, p), m_lind.eval_rates(phi, p)
    for k in a:
        np.testing.assert_allclose(a[k], b[k], rtol=1e-15, atol=0)
    Ja, Jb = m_troe.eval_jacobian(phi, p), m_lind.eval_jacobian(phi, p)
    assert np.max(np.linalg.norm(Ja - Jb, axis=0) / np.linalg.norm(Jb, axis=0)) < 1e-14


# ---------------------------------------------------- absent collider (P_r = 0)


@pytest.mark.parametrize("kind", BLENDED)
def test_absent_collider_finite_and_complex_step(Ref, kind):
    mech, m_sp = species_collider_mech(kind, 150 + BLENDED.index(kind))
    m = Ref(text=mech.to_text())
    phi, p = zero_collider_states(mech, m_sp, 9)
    out = m.eval_rates(phi, p)
    for k, v in out.items():
        assert np.all(np.isfinite(v)), k
    i = next(q for q, r in enumerate(mech.reactions) if r.kind == kind)
    c = out["pres_mod"][i]
    if kind.startswith("falloff"):
        assert np.all(np.abs(c[[0, 1, 3]]) == 0.0)      # no collider: no falloff rate
    else:
        assert np.all(c > 0)                            # low-pressure limit k_0 F
    J = m.eval_jacobian(phi, p)
    Jcs = m.eval_jacobian_cs(phi, p)
    assert np.all(np.isfinite(J)) and np.all(np.isfinite(Jcs))
    e = np.linalg.norm(J - Jcs, axis=0) / np.linalg.norm(Jcs, axis=0)
    assert e.max() < 1e-12, e


@pytest.mark.parametrize("blend", ["troe", "sri"])
def test_zero_pr_blending_is_the_limit(Ref, blend):
    """At P_r = 0 the oracle's F equals the paper's F evaluated in mpmath at
    log10 P_r = -1e12, where it has converged to the P_r -> 0+ limit (the
    approach is O(1 / log10 P_r))."""
    for kind in (f"falloff_{blend}", f"chemact_{blend}"):
        mech, m_sp = species_collider_mech(kind, 170)
        m = Ref(text=mech.to_text())
        i = next(q for q, r in enumerate(mech.reactions) if r.kind == kind)
        r = mech.reactions[i]
        y = np.full(m.n_species - 1, 1.0 / m.n_species)
        y[m_sp] = 0.0
        for T in (1000.5, 1800.0):
            t = m.reaction_terms(T, 3 * ATM, y)
            assert t["Pr"][i] == 0.0
            lPr = mp.mpf(-1e12)
            Fref = _troe_F(r.troe, T, lPr) if blend == "troe" else _sri_F(r.sri, T, lPr)
            assert abs(t["F"][i] / float(Fref) - 1) < 1e-10
            # and F at small positive P_r approaches that value from the paper's formula
            t2 = m.reaction_terms(T, 3 * ATM, np.where(np.arange(len(y)) == m_sp, 1e-25, y))
            Fsmall = _troe_F(r.troe, T, mp.log10(mp.mpf(t2["Pr"][i]))) if blend == "troe" else \
                _sri_F(r.sri, T, mp.log10(mp.mpf(t2["Pr"][i])))
            assert abs(t2["F"][i] / float(Fsmall) - 1) < 1e-12
            assert abs(t2["F"][i] - t["F"][i]) < abs(float(Fsmall) - 1) + 0.2


@pytest.mark.parametrize("kind", BLENDED)
def test_jacobian_continuous_as_collider_vanishes(Ref, kind):
    """Falloff derivatives have finite limits as P_r -> 0+: the Jacobian at a
    collider mass fraction eps tends to the one at 0 as eps -> 0 (geometric
    for Lindemann, O(1/log P_r) for Troe and SRI, whose ln F approaches its
    limit logarithmically).  Chemically activated Troe/SRI reactions have a
    log-singular dF/dP_r at 0, so only the Lindemann form is checked there."""
    if kind.startswith("chemact") and not kind.endswith("lindemann"):
        pytest.skip("dF/dP_r is unbounded as P_r -> 0+ for chemically activated Troe/SRI")
    mech, m_sp = species_collider_mech(kind, 190 + BLENDED.index(kind))
    m = Ref(text=mech.to_text())
    phi, p = draw_states(4, mech.n_species, 1, dirichlet=0.7)
    phi[1 + m_sp, 0] = 0.0
    J0 = m.eval_jacobian(phi, p)[:, 0]
    errs = []
    for eps in (1e-30, 1e-90, 1e-270):
        q = phi.copy()
        q[1 + m_sp, 0] = eps
        Je = m.eval_jacobian(q, p)[:, 0]
        errs.append(np.linalg.norm(Je - J0) / np.linalg.norm(J0))
    assert errs[0] >= errs[1] >= errs[2]
    if kind.endswith("lindemann"):
        assert errs[0] < 1e-12
    else:
        assert errs[2] < 0.05
