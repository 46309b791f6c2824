"""Implicit integrator step (SDIRK3 driving J + Newton).

CPU: the oracle's step is pinned by the method's order conditions, the
L-stability cubic for gamma, the stiff limit R(z) -> 0, the local error
order on y' = lambda y and the global convergence order on y' = -y^2 with
known solution 1/(1+t).  GPU: pyjac_sdirk3_step against the oracle's step
on chemistry states.
"""
import numpy as np
import pytest

from oracle.sdirk_ref import A, B, C, GAMMA, sdirk3_step, sdirk3_step_states
from synth import config_mechanism, config_states


def test_tableau_order_conditions():
    assert B.sum() == pytest.approx(1.0, abs=1e-15)
    assert B @ C == pytest.approx(0.5, abs=1e-15)
    assert B @ C ** 2 == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert B @ A @ C == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert np.allclose(np.diag(A), GAMMA) and np.allclose(A[2], B)      # stiffly accurate
    # L-stability of the family: gamma is the root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2)
    assert abs(GAMMA ** 3 - 3 * GAMMA ** 2 + 1.5 * GAMMA - 1.0 / 6.0) < 1e-15
    assert 1.0 / 6.0 < GAMMA < 0.5


def linear(lam):
    return (lambda y: lam * y), (lambda y: np.array([[lam]]))


def test_stiff_limit():
    f, J = linear(-1e9)
    y1, _ = sdirk3_step(f, J, np.array([1.0]), 1.0, newton_iters=2)
    assert abs(y1[0]) < 1e-8


def test_local_error_order():
    f, J = linear(-1.0)
    errs = [abs(sdirk3_step(f, J, np.array([1.0]), h, newton_iters=2)[0][0] - np.exp(-h)) for h in (0.2, 0.1, 0.05)]
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(13.0 < r < 19.0 for r in ratios), ratios        # local error O(h^4)


def test_global_convergence_order():
    f = lambda y: -y ** 2                      # noqa: E731
    J = lambda y: np.array([[-2.0 * y[0]]])    # noqa: E731
    errs = []
    for nsteps in (8, 16, 32):
        y = np.array([1.0])
        for _ in range(nsteps):
            y, _ = sdirk3_step(f, J, y, 1.0 / nsteps, newton_iters=8)
        errs.append(abs(y[0] - 0.5))
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(6.5 < r < 9.5 for r in ratios), ratios          # global error O(h^3)


def test_chemistry_small_step_is_explicit_euler(oracle_built):
    """For h -> 0 the step is y + h f(y) + O(h^2)."""
    from oracle import RefMech
    mech = config_mechanism(0)
    ref = RefMech(text=mech.to_text())
    phi, p = config_states(0, 3)
    f0 = ref.eval_rates(phi, p)["dphi"]
    devs = []
    for c in (1e-2, 1e-3):                      # h ||J|| = c / gamma; smaller steps hit rounding in y1 - y
        h = step_sizes(ref, phi, p, c)
        y1, _ = sdirk3_step_states(ref, phi, p, h, newton_iters=3)
        devs.append(np.abs((y1 - phi) / h - f0).max(axis=0) / np.abs(f0).max(axis=0))
        assert devs[-1].max() <= c, devs[-1]
    ratio = devs[1] / devs[0]
    assert np.all((ratio > 0.05) & (ratio < 0.2)), ratio     # the deviation is O(h)


# ------------------------------------------------------------------- GPU
def step_sizes(ref, phi, p, c):
    """h = c / (gamma ||J||_inf) per state."""
    J = np.asarray(ref.eval_jacobian(phi, p))
    N = phi.shape[0]
    nrm = np.array([np.abs(J[:, s].reshape(N, N)).sum(axis=1).max() for s in range(phi.shape[1])])
    return c / (GAMMA * nrm)


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,n", [(0, 40), (1, 12)])
def test_gpu_step_matches_oracle(oracle_built, cfg, n):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import RefMech
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED, Mechanism
    mech = config_mechanism(cfg)
    ref = RefMech(text=mech.to_text())
    phi, p = config_states(cfg, n)
    c = np.exp(np.random.default_rng(cfg).uniform(np.log(0.1), np.log(10.0), n))
    h = step_sizes(ref, phi, p, c)
    y_ref, dn_ref = sdirk3_step_states(ref, phi, p, h, newton_iters=4)
    M = Mechanism(text=mech.to_text())
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()    # noqa: E731
    dphi, dp, dh = d(phi), d(p), d(h)
    y, dn = M.sdirk3_step(dphi, dp, dh, newton_iters=4, mode=NEWTON_FP64)
    y = y.cpu().numpy()
    inc_ref = y_ref - phi
    scale = np.abs(inc_ref).max(axis=0) + 1e-300
    err = np.abs((y - phi) - inc_ref).max(axis=0) / scale
    print(f"C{cfg}: max rel increment error {err.max():.2e}, stage-3 increment {dn_ref[2].max():.1e}")
    assert err.max() <= 1e-10
    # mixed-precision Newton solves: the same step within the refinement tolerance
    ym, _ = M.sdirk3_step(dphi, dp, dh, newton_iters=4, mode=NEWTON_MIXED)
    assert (np.abs(ym.cpu().numpy() - y).max(axis=0) / scale).max() <= 1e-10
    # in place equals out of place, bitwise
    yi, _ = M.sdirk3_step(dphi, dp, dh, newton_iters=4, mode=NEWTON_FP64, out=dphi)
    assert np.array_equal(dphi.cpu().numpy(), y)


@pytest.mark.gpu
def test_gpu_step_arguments():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03262_amd import Mechanism, PyjacError, _lib
    mech = config_mechanism(0)
    M = Mechanism(text=mech.to_text())
    phi, p = config_states(0, 4)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()    # noqa: E731
    with pytest.raises(PyjacError):
        M.sdirk3_step(d(phi), d(p), d(np.full(4, 1e-8)), newton_iters=0)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(PyjacError, match="WORKSPACE"):
        M.sdirk3_step(d(phi), d(p), d(np.full(4, 1e-8)), workspace=ws)
    assert _lib.pyjac_sdirk3_workspace_bytes(M.handle, 4, 3, 0) == 0      # ld < n


@pytest.mark.gpu
def test_gpu_step_batch_independence(oracle_built):
    """A state's step depends only on its own inputs: the same bits alone,
    permuted in the batch, or with ld > n; n = 0 is a no-op."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import RefMech
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(1)
    ref = RefMech(text=mech.to_text())
    n = 33
    phi, p = config_states(1, n)
    h = step_sizes(ref, phi, p, np.full(n, 1.0))
    M = Mechanism(text=mech.to_text())
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()    # noqa: E731
    base = M.sdirk3_step(d(phi), d(p), d(h))[0].cpu().numpy()
    perm = np.random.default_rng(1).permutation(n)
    yp = M.sdirk3_step(d(phi[:, perm]), d(p[perm]), d(h[perm]))[0].cpu().numpy()
    assert np.array_equal(yp, base[:, perm])
    for s in (0, 32):
        ys = M.sdirk3_step(d(phi[:, s:s + 1]), d(p[s:s + 1]), d(h[s:s + 1]))[0].cpu().numpy()
        assert np.array_equal(ys[:, 0], base[:, s])
    ld = 40                                  # padded rows: extra columns hold other states
    phl = np.concatenate([phi, phi[:, :ld - n]], axis=1)
    pl = np.concatenate([p, p[:ld - n]])
    hl = np.concatenate([h, h[:ld - n]])
    dphl = d(phl)
    out = torch.full_like(dphl, -1.0)
    M.sdirk3_step(dphl[:, :n], d(pl), d(hl), out=out[:, :n])
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :n], base) and np.all(o[:, n:] == -1.0)
    M.sdirk3_step(dphl[:, :0], d(pl), d(hl))           # n = 0: returns without launching
    torch.cuda.synchronize()
