"""GPU parity on the method's edge cases (Sec. 3.1, Sec. 5.1), through the C ABI
against the oracle:
  * mass fractions that are exactly zero, including the species that is a
    reaction's only collider (then P_r = 0, and the blending takes its
    P_r -> 0+ limit on both sides), and a collider driven slightly negative;
  * constructed chemical-equilibrium states (every K_c-reversible reaction has
    R_f = R_r, so q and the production rates are pure cancellation);
  * a reactive last species at the 53-species workload's size;
  * the finite-difference Jacobian against the oracle's forward-difference
    quotient with the same increments;
  * Newton solves at full batch size for the 111- and 360-species workloads,
    sampled states checked against the LAPACK + extended-precision reference;
  * served requests (mixed mechanisms, a 360-species request among them)
    against the oracle's Jacobian and Newton reference.
"""
import numpy as np
import pytest

from conftest import BLENDED, species_collider_mech, zero_collider_states
from equilibrium import equilibrium_states
from synth import (WORKLOADS, NEWTON_GAMMA, conditioned_steps, config_mechanism, config_states,
                   draw_newton_inputs, draw_states, make_mechanism)
from test_gpu_parity import JAC_TOL, check_jac, check_rates, gpu_jac, gpu_mech, gpu_rates

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
R = 8314.462618


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def _finite_parity(torch, Ref, mech, phi, p, label, ld=None):
    ref = Ref(text=mech.to_text())
    M = gpu_mech(mech)
    og, orf = gpu_rates(torch, M, phi, p, ld), ref.eval_rates(phi, p)
    for k in og:
        assert np.all(np.isfinite(og[k])), (label, k)
        assert np.all(np.isfinite(orf[k])), (label, k)
    check_rates(og, orf, mech, phi, p, label)
    return check_jac(gpu_jac(torch, M, phi, p, ld), ref.eval_jacobian(phi, p), label), og


# --------------------------------------------- absent single-species collider
@pytest.mark.parametrize("kind", BLENDED)
def test_absent_collider(torch, Ref, kind):
    """P_r = 0 (collider mass fraction 0) and P_r < 0 (-1e-14, as an integrator
    stage can produce): finite results equal to the oracle's."""
    mech, m_sp = species_collider_mech(kind, 150 + BLENDED.index(kind))
    phi, p = zero_collider_states(mech, m_sp, 9, values=(0.0, 0.0, -1e-14, 0.0, 1e-200, 1e-30))
    e, og = _finite_parity(torch, Ref, mech, phi, p, kind, ld=11)
    i = next(q for q, r in enumerate(mech.reactions) if r.kind == kind)
    c = og["pres_mod"][i]
    if kind.startswith("falloff"):
        assert np.all(c[[0, 1, 3]] == 0.0)               # no collider: no falloff rate
    else:
        assert np.all(c[[0, 1, 3]] > 0)                  # low-pressure limit k_0 F


# -------------------------------------------------- zero mass fractions (C1)
def test_zero_mass_fractions_full_mechanism(torch, Ref):
    """The 53-species mechanism with a third of the mass fractions set to 0 in
    each state (no division by [X] anywhere in Sec. 3.1), and states in which
    every single-species collider is absent."""
    mech = config_mechanism(1)
    N = mech.n_species
    phi, p = config_states(1, 400)
    rng = np.random.default_rng(21)
    zero = rng.random((N - 1, phi.shape[1])) < 0.33
    phi[1:][zero] = 0.0
    colliders = sorted({r.collider_species for r in mech.reactions
                        if r.collider == "species" and r.collider_species < N - 1})
    assert colliders, "the mechanism has single-species colliders"
    phi[1 + np.array(colliders), :50] = 0.0
    phi[1 + np.array(colliders), 50:60] = -1e-15
    e, _ = _finite_parity(torch, Ref, mech, phi, p, "zero Y")
    print(f"zero mass fractions: max E_norm {e.max():.2e}")


# ------------------------------------------------------- equilibrium states
@pytest.mark.parametrize("cfg,n", [(0, 12), (1, 6)])
def test_equilibrium_states(torch, Ref, cfg, n):
    """At constructed equilibrium R_f = R_r for every reaction; the GPU rates
    show the cancellation to rounding and match the oracle, and the Jacobian
    (nonzero at equilibrium) matches to E_norm <= 1e-10."""
    mech = config_mechanism(cfg)
    phi, p = equilibrium_states(mech, n, seed=40 + cfg)
    e, og = _finite_parity(torch, Ref, mech, phi, p, f"equilibrium C{cfg}")
    rel = np.abs(og["rop_f"] - og["rop_r"]) / np.maximum(og["rop_f"], 1e-300)
    assert rel.max() < 1e-9, rel.max()
    print(f"C{cfg} equilibrium: max |R_f - R_r|/R_f {rel.max():.2e}, max E_norm {e.max():.2e}")


# -------------------------------------------- reactive last species, C1 size
def test_reactive_last_species_full_size_mechanism(torch, Ref):
    """53 species / 325 reactions in the methane-shaped mix, but the last
    species (whose mass fraction is implied) takes part in reactions, so every
    placeholder-row term of Sec. 3.2 is exercised at full mechanism size."""
    c = WORKLOADS[1]
    mech = make_mechanism(1605 + 101, c["n_species"], c["n_reactions"], c["elements"], c["bounds"],
                          c["mix"], reactive_last=True, name="reactive_last_53")
    L = mech.n_species - 1
    assert any(L in dict(r.reac) or L in dict(r.prod) for r in mech.reactions)
    phi, p = draw_states(77, mech.n_species, 500, dirichlet=0.3)
    e, _ = _finite_parity(torch, Ref, mech, phi, p, "reactive last", ld=509)
    print(f"reactive last species: max E_norm {e.max():.2e}")


# ------------------------------------------------------- FD against the oracle
@pytest.mark.parametrize("cfg,n", [(0, 200), (1, 64)])
def test_fd_against_oracle_quotient(torch, Ref, cfg, n):
    """The GPU FD Jacobian equals the oracle's forward-difference quotient
    (f(phi + d_j e_j) - f(phi)) / d_j with the same increments
    d_j = fl(phi_j + 2^-26 max(|phi_j|, floor_j)) - phi_j.  The two RHS
    evaluations differ by their rounding, bounded by the rate gate
    (1e-12 of the gross magnitude per species element, 1e-11 of the
    temperature row's scale), so element (i, j) may differ by twice that
    bound over d_j."""
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, n)
    M = Mechanism(text=mech.to_text())
    Jf = M.eval_jacobian_fd(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    Jf = Jf.cpu().numpy().reshape(N, N, n)
    ref = Ref(text=mech.to_text())
    floor = np.full(N, 1e-10)
    floor[0] = 1.0
    nf, nr = mech.stoich()
    W = mech.molecular_weights()

    def rhs_and_scale(q):
        o = ref.eval_rates(q, p)
        gross = np.abs(nr - nf) @ (np.abs(o["pres_mod"]) * (np.abs(o["rop_f"]) + np.abs(o["rop_r"])))
        Y = np.vstack([q[1:], 1 - q[1:].sum(axis=0)])
        rho = p / (R * q[0] * (Y / W[:, None]).sum(axis=0))
        sc = np.empty((N, n))
        sc[1:] = W[:-1, None] * gross[:-1] / rho
        sc[0] = np.abs(o["dphi"][0]) + (W[:, None] * gross).sum(axis=0) * 1e4 / rho
        return o["dphi"], sc

    gate = np.full((N, 1), 1e-12)
    gate[0] = 1e-11
    f0, s0 = rhs_and_scale(phi)
    for j in range(N):
        q = phi.copy()
        q[j] = phi[j] + 2.0 ** -26 * np.maximum(np.abs(phi[j]), floor[j])
        d = q[j] - phi[j]
        fj, sj = rhs_and_scale(q)
        Jo = (fj - f0) / d
        tol = 2.0 * gate * np.maximum(s0, sj) / d
        bad = np.abs(Jf[:, j, :] - Jo) > tol
        assert not bad.any(), (j, np.max(np.abs(Jf[:, j, :] - Jo) / tol))


# ------------------------------------------------ Newton at full batch size
@pytest.mark.parametrize("cfg", [2, 3])
def test_newton_full_batch_sampled(torch, Ref, cfg):
    """The full batch (100,000 systems at 111 species; 20,000 at 360), both
    modes, conditioned steps.  The Jacobians are the oracle's, for 96 (C2) or
    24 (C3) distinct states tiled over the batch; each column has its own h and
    right-hand side, so every system is distinct.  Sampled systems are checked
    against the LAPACK + extended-precision reference (gate as in the Newton
    parity tests)."""
    from oracle.newton_ref import newton_reference
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED, Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    n = WORKLOADS[cfg]["n_states"]
    n_base = 96 if cfg == 2 else 24
    phi, p = config_states(cfg, n_base)
    Jb = Ref(text=mech.to_text()).eval_jacobian(phi, p)
    src = np.arange(n) % n_base
    rows = np.abs(Jb.reshape(N, N, n_base)).sum(axis=1)[:, src]
    h = conditioned_steps(80 + cfg, rows)
    _, b = draw_newton_inputs(81 + cfg, N, n)
    M = Mechanism(text=mech.to_text())
    dJ = torch.from_numpy(Jb).cuda()[:, torch.from_numpy(src).cuda()].contiguous()
    dh, db = torch.from_numpy(h).cuda(), torch.from_numpy(b).cuda()
    rng = np.random.default_rng(cfg)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)]))
    xr, kappa = newton_reference(Jb[:, src[idx]], h[idx], NEWTON_GAMMA, b[:, idx])
    well = kappa * U <= 1e-11
    out = {}
    for mode in (NEWTON_FP64, NEWTON_MIXED):
        x, info = M.newton_solve(dJ, dh, db, NEWTON_GAMMA, mode=mode, max_refine=10, rtol=1e-14)
        torch.cuda.synchronize()
        ti = torch.from_numpy(idx).cuda()
        out[mode] = (x[:, ti].cpu().numpy(), info[ti].cpu().numpy(), info[:n].cpu().numpy())
        del x, info
    del dJ
    torch.cuda.empty_cache()
    x0, i0, a0 = out[NEWTON_FP64]
    x1, i1, a1 = out[NEWTON_MIXED]
    assert np.all(a0 == 0)
    assert np.all((a1 >= 1) | (a1 == -2))
    e0 = np.max(np.abs(x0 - xr), axis=0) / np.max(np.abs(xr), axis=0)
    e1 = np.max(np.abs(x1 - xr), axis=0) / np.max(np.abs(xr), axis=0)
    b0 = np.where(well, 1e-10, 100 * kappa * U)
    b1 = np.where(well, 1e-10, 2 * np.maximum(e0, 100 * kappa * U))
    assert np.all(e0 <= b0), f"mode 0 worst {np.max(e0 / b0):.3g} x bar"
    assert np.all(e1 <= b1), f"mode 1 worst {np.max(e1 / b1):.3g} x bar"
    assert well.mean() > 0.3
    print(f"C{cfg} full batch n={n}: sampled {len(idx)}, err0 max {e0.max():.2e}, err1 max {e1.max():.2e}, "
          f"fallbacks {(a1 == -2).sum()}/{n}")


# --------------------------------------------------- served against the oracle
def test_served_results_against_oracle(torch, Ref):
    """Requests of the 13-, 53-, 111- and 360-species mechanisms served
    together (FP64 and mixed).  Each served x is compared with the Newton
    reference built on the oracle's Jacobian of the same states.  The served
    Jacobian is the GPU's, within E_norm 1e-10 of the oracle's, so the bar is
    kappa (1e-10 + 100 u) + 1e-10 (first-order perturbation of A = I - h gamma J
    by h gamma dJ, with h gamma ||J|| = c <= 30 here)."""
    from oracle.newton_ref import newton_reference
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED, Mechanism, Server
    rng = np.random.default_rng(5)
    plan = [(0, 40), (1, 33), (2, 9), (3, 3), (0, 7), (1, 5), (3, 2), (2, 4)]
    mechs = {c: config_mechanism(c) for c in (0, 1, 2, 3)}
    gm = {c: Mechanism(text=m.to_text()) for c, m in mechs.items()}
    refs = {c: Ref(text=m.to_text()) for c, m in mechs.items()}
    srv = Server(hbm_budget_bytes=2 << 30, max_batch_states=256, n_streams=2, max_refine=6, rtol=1e-14)
    reqs = []
    for q, (c, n) in enumerate(plan):
        N = mechs[c].n_species
        phi, p = draw_states(int(rng.integers(1 << 30)), N, n)
        Jr = refs[c].eval_jacobian(phi, p)
        h = conditioned_steps(300 + q, np.abs(Jr.reshape(N, N, n)).sum(axis=1), c_range=(1.0, 30.0))
        _, b = draw_newton_inputs(400 + q, N, n)
        mode = NEWTON_MIXED if q % 2 else NEWTON_FP64
        rid, x, info = srv.submit(gm[c], phi, p, h, b, NEWTON_GAMMA, mode=mode)
        reqs.append((c, Jr, h, b, mode, rid, x, info))
    for c, Jr, h, b, mode, rid, x, info in reqs:
        srv.wait(rid)
    srv.close()
    for c, Jr, h, b, mode, rid, x, info in reqs:
        xr, kappa = newton_reference(Jr, h, NEWTON_GAMMA, b)
        err = np.max(np.abs(x - xr), axis=0) / np.max(np.abs(xr), axis=0)
        bar = 1e-10 + kappa * (JAC_TOL + 100 * U)
        assert np.all(info == 0) if mode == NEWTON_FP64 else np.all((info >= 1) | (info == -2))
        assert np.all(err <= bar), (c, mode, float(np.max(err / bar)))
