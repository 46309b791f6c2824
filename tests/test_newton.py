"""Batched Newton solve (I - h gamma J) x = b: GPU modes vs the LAPACK +
extended-precision reference.

Bar (per state, infinity norms, u = 2^-53, kappa = kappa_inf(A)):
  well conditioned (kappa u <= 1e-11): ||x - x*|| / ||x*|| <= 1e-10 in both modes;
  otherwise mode 0 <= 100 kappa u (LU growth slack) and mode 1 <= 2 max(mode-0
  error, 100 kappa u).  Conditioning and FP64 fallbacks are reported.
J is the oracle's Jacobian (never the GPU's); the same J is uploaded as input.
"""
import numpy as np
import pytest

from synth import (NEWTON_GAMMA, conditioned_steps, config_mechanism, config_states,
                   draw_newton_inputs)

U = 2.0 ** -53


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def test_reference_backward_error(Ref):
    """The reference's refined solution has an extended-precision backward error
    at the level of a backward-stable FP64 solve, and its residual is tiny."""
    from oracle.newton_ref import newton_reference
    mech = config_mechanism(0)
    m = Ref(text=mech.to_text())
    phi, p = config_states(0, 12)
    J = m.eval_jacobian(phi, p)
    h, b = draw_newton_inputs(5, mech.n_species, 12)
    x, kappa = newton_reference(J, h, NEWTON_GAMMA, b)
    N = mech.n_species
    for s in range(12):
        A = (np.eye(N) - h[s] * NEWTON_GAMMA * J[:, s].reshape(N, N)).astype(np.longdouble)
        r = b[:, s].astype(np.longdouble) - A @ x[:, s].astype(np.longdouble)
        bw = np.max(np.abs(r)) / (np.max(np.abs(A)) * np.max(np.abs(x[:, s])) + np.max(np.abs(b[:, s])))
        assert float(bw) <= 4 * N * U
        assert kappa[s] >= 1.0


def _errs(x, xr):
    return np.max(np.abs(x - xr), axis=0) / np.max(np.abs(xr), axis=0)


@pytest.mark.gpu
@pytest.mark.parametrize("recipe", ["configured_h", "conditioned_h"])
@pytest.mark.parametrize("cfg,n", [(0, 300), (1, 199), (2, 37), (3, 6)])
def test_newton_modes_vs_reference(Ref, cfg, n, recipe):
    import torch
    from oracle.newton_ref import newton_reference
    from paper_1605_03262_amd import Mechanism, NEWTON_FP64, NEWTON_MIXED
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, n)
    J = Ref(text=mech.to_text()).eval_jacobian(phi, p)
    h, b = draw_newton_inputs(40 + cfg, N, n)
    if recipe == "conditioned_h":
        rows = np.abs(J.reshape(N, N, n)).sum(axis=1)
        h = conditioned_steps(60 + cfg, rows)
    xr, kappa = newton_reference(J, h, NEWTON_GAMMA, b)
    M = Mechanism(text=mech.to_text())
    ld = n + 5
    dJ = torch.zeros((N * N, ld), dtype=torch.float64, device="cuda")
    dJ[:, :n] = torch.from_numpy(J)
    dh = torch.ones(ld, dtype=torch.float64, device="cuda")
    dh[:n] = torch.from_numpy(h)
    db = torch.zeros((N, ld), dtype=torch.float64, device="cuda")
    db[:, :n] = torch.from_numpy(b)
    view = lambda t, rows: t.as_strided((rows, n), (ld, 1))  # noqa: E731
    x0, i0 = M.newton_solve(view(dJ, N * N), dh, view(db, N), NEWTON_GAMMA, mode=NEWTON_FP64)
    x1, i1 = M.newton_solve(view(dJ, N * N), dh, view(db, N), NEWTON_GAMMA, mode=NEWTON_MIXED,
                            max_refine=10, rtol=1e-14)
    torch.cuda.synchronize()
    x0 = x0[:, :n].cpu().numpy()
    x1 = x1[:, :n].cpu().numpy()
    i0 = i0[:n].cpu().numpy()
    i1 = i1[:n].cpu().numpy()
    assert np.all(i0 == 0), np.unique(i0)
    assert np.all((i1 >= 1) | (i1 == -2)), np.unique(i1)
    e0, e1 = _errs(x0, xr), _errs(x1, xr)
    well = kappa * U <= 1e-11
    b0 = np.where(well, 1e-10, 100 * kappa * U)
    b1 = np.where(well, 1e-10, 2 * np.maximum(e0, 100 * kappa * U))
    assert np.all(e0 <= b0), f"mode 0 worst {np.max(e0 / b0):.3g} x bar"
    assert np.all(e1 <= b1), f"mode 1 worst {np.max(e1 / b1):.3g} x bar"
    if recipe == "conditioned_h":
        # solvable systems: the strict bar must hold wherever conditioning allows it
        assert well.mean() > 0.3
    print(f"C{cfg} {recipe}: kappa median {np.median(kappa):.2e} max {kappa.max():.2e}; "
          f"well {well.mean():.0%}; err0 max {e0.max():.2e}, err1 max {e1.max():.2e}; "
          f"fallbacks {(i1 == -2).sum()}/{n}; sweeps {np.bincount(i1[i1 > 0]) if (i1 > 0).any() else []}")


@pytest.mark.gpu
def test_newton_singular_nonfinite_and_workspace():
    import torch
    from paper_1605_03262_amd import Mechanism, PyjacError, _lib
    mech = config_mechanism(0)
    N = mech.n_species
    M = Mechanism(text=mech.to_text())
    n = 4
    gamma = 0.5
    h = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    J = torch.zeros((N * N, n), dtype=torch.float64, device="cuda")
    eye = torch.eye(N, dtype=torch.float64, device="cuda").reshape(-1)
    J[:, 0] = eye                    # A = I - 2*0.5*I = 0: singular
    J[:, 1] = 0.1 * eye              # A = 0.9 I
    J[:, 2] = 0.1 * eye
    J[5, 2] = float("nan")           # non-finite
    J[:, 3] = 0.3 * eye
    b = torch.ones((N, n), dtype=torch.float64, device="cuda")
    for mode in (0, 1):
        x, info = M.newton_solve(J, h, b, gamma, mode=mode, max_refine=5, rtol=1e-14)
        torch.cuda.synchronize()
        info = info.cpu().numpy()
        assert info[0] == -1 and info[2] == -3, info
        assert info[1] >= 0 and info[3] >= 0
        xx = x.cpu().numpy()
        np.testing.assert_allclose(xx[:, 1], 1 / 0.9, rtol=1e-14)
        np.testing.assert_allclose(xx[:, 3], 1 / 0.7, rtol=1e-14)
    need = M.newton_workspace_bytes(n, 1)
    ws = torch.empty((need // 2,), dtype=torch.uint8, device="cuda")
    x = torch.empty((N, n), dtype=torch.float64, device="cuda")
    info = torch.empty((n,), dtype=torch.int32, device="cuda")
    with pytest.raises(PyjacError):
        _lib.pyjac_newton_factor_solve(M.handle, n, n, J.data_ptr(), h.data_ptr(), gamma, b.data_ptr(),
                                       x.data_ptr(), 1, 5, 1e-14, info.data_ptr(), ws.data_ptr(),
                                       ws.numel(), None)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [0, 1])
def test_newton_full_size_backward_error(mode):
    """The benchmark's full batch (100,000 states of the 53-species workload,
    conditioned steps): for sampled states, the returned x solves the system
    it was given, with an FP64 backward error at the level of a stable solve
    (||b - A x|| <= 4 N u (||A|| ||x|| + ||b||), infinity norms, A = I - h gamma J
    formed on the host from the same J)."""
    import torch
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(1)
    N = mech.n_species
    phi, p = config_states(1)
    n = phi.shape[1]
    M = Mechanism(text=mech.to_text())
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    J = M.eval_jacobian(d_phi, d_p)
    rows = torch.abs(J.view(N, N, n)).sum(dim=1).cpu().numpy()
    h = conditioned_steps(61, rows)
    _, b = draw_newton_inputs(41, N, n)
    x, info = M.newton_solve(J, torch.from_numpy(h).cuda(), torch.from_numpy(b).cuda(), NEWTON_GAMMA,
                             mode=mode, max_refine=4, rtol=1e-14)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert np.all((info == 0) if mode == 0 else ((info >= 1) | (info == -2))), np.unique(info)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 200, replace=False)]))
    Js = J[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    xs = x[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    for c, s in enumerate(idx):
        A = np.eye(N) - h[s] * NEWTON_GAMMA * Js[:, c].reshape(N, N)
        r = b[:, s].astype(np.longdouble) - A.astype(np.longdouble) @ xs[:, c].astype(np.longdouble)
        bound = 4 * N * U * (np.abs(A).sum(axis=1).max() * np.abs(xs[:, c]).max() + np.abs(b[:, s]).max())
        assert float(np.abs(r).max()) <= bound, (s, float(np.abs(r).max()), bound)


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,n", [(2, 64), (1, 64), (0, 37)])
def test_reused_factor_equals_fresh_solve(cfg, n):
    """Solves with PYJAC_NEWTON_REUSE_FACTOR after a PYJAC_NEWTON_KEEP_FACTOR
    solve of the same matrix equal fresh solves bitwise (blocked path and
    register-path FP64: the factor kept in the workspace; register-path
    mixed mode: the flags are accepted and the system factored)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_KEEP_FACTOR, NEWTON_MIXED, NEWTON_REUSE_FACTOR, Mechanism
    from synth import NEWTON_GAMMA, conditioned_steps, draw_newton_inputs
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, n)
    M = Mechanism(text=mech.to_text())
    J = M.eval_jacobian(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda())
    rows = torch.abs(J.view(N, N, n)).sum(dim=1).cpu().numpy()
    h = torch.from_numpy(conditioned_steps(7, rows)).cuda()
    b1 = torch.from_numpy(draw_newton_inputs(8, N, n)[1]).cuda()
    b2 = torch.from_numpy(draw_newton_inputs(9, N, n)[1]).cuda()
    for mode in (NEWTON_FP64, NEWTON_MIXED):
        ws = torch.empty((max(M.newton_workspace_bytes(n, mode | NEWTON_KEEP_FACTOR), 1),), dtype=torch.uint8,
                         device="cuda")
        xk, ik = M.newton_solve(J, h, b1, NEWTON_GAMMA, mode=mode | NEWTON_KEEP_FACTOR, workspace=ws)
        x1, i1 = M.newton_solve(J, h, b1, NEWTON_GAMMA, mode=mode)
        for b in (b2, b1, b2):             # several solves with one kept factor
            xr, ir = M.newton_solve(J, h, b, NEWTON_GAMMA, mode=mode | NEWTON_REUSE_FACTOR, workspace=ws)
            xf, i_f = M.newton_solve(J, h, b, NEWTON_GAMMA, mode=mode)
            torch.cuda.synchronize()
            assert torch.equal(xr, xf), mode
            assert torch.equal(ir[:n], i_f[:n]), mode
        assert torch.equal(xk, x1) and torch.equal(ik[:n], i1[:n]), mode
