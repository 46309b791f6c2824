"""The no-allocation Newton entry point (static device scratch) against the
workspace entry point it shares its kernels with: bitwise equal x and info,
on two calls in a row with the second smaller, for the register path
(53 species) and the blocked path (111 species), both modes; sizes beyond the
static array are refused before anything is enqueued."""
import numpy as np
import pytest

from synth import NEWTON_GAMMA, conditioned_steps, config_mechanism, config_states, draw_newton_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _inputs(torch, M, cfg, n, seed):
    N = M.n_species
    phi, p = config_states(cfg, n)
    J = M.eval_jacobian(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda())
    rows = torch.abs(J.view(N, N, n)).sum(dim=1).cpu().numpy()
    h = torch.from_numpy(conditioned_steps(seed, rows)).cuda()
    b = torch.from_numpy(draw_newton_inputs(seed + 1, N, n)[1]).cuda()
    return J, h, b


def _noalloc(torch, M, J, h, b, mode):
    from paper_1605_03262_amd import _lib
    N, n = M.n_species, b.shape[1]
    x = torch.full((N, n), float("nan"), dtype=torch.float64, device="cuda")
    info = torch.full((n,), 12345, dtype=torch.int32, device="cuda")
    _lib.pyjac_newton_factor_solve_noalloc(M.handle, n, n, J.data_ptr(), h.data_ptr(), NEWTON_GAMMA,
                                           b.data_ptr(), x.data_ptr(), mode, 6, 1e-14, info.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
    return x, info


@pytest.mark.parametrize("cfg,sizes", [(1, (3000, 700)), (0, (500, 31)), (2, (300, 97))])
@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_equals_workspace_entry_point(torch, cfg, sizes, mode):
    from paper_1605_03262_amd import Mechanism
    M = Mechanism(text=config_mechanism(cfg).to_text())
    for k, n in enumerate(sizes):
        J, h, b = _inputs(torch, M, cfg, n, 50 + 3 * k + cfg)
        xs, is_ = _noalloc(torch, M, J, h, b, mode)
        xw, iw = M.newton_solve(J, h, b, NEWTON_GAMMA, mode=mode, max_refine=6, rtol=1e-14)
        torch.cuda.synchronize()
        assert torch.equal(is_, iw[:n]), (cfg, n, mode)
        assert torch.equal(xs, xw[:, :n]), (cfg, n, mode)
        assert bool(torch.isfinite(xs).all())


def test_noalloc_rejects_oversize(torch):
    from paper_1605_03262_amd import Mechanism, PyjacError, _lib
    M = Mechanism(text=config_mechanism(2).to_text())
    N = M.n_species
    n = 2000                                        # 111 species: ~148 KB per state in mode 1
    assert M.newton_workspace_bytes(n, 1) > 64 << 20
    J = torch.zeros((N * N, n), dtype=torch.float64, device="cuda")
    h = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones((N, n), dtype=torch.float64, device="cuda")
    x = torch.empty((N, n), dtype=torch.float64, device="cuda")
    info = torch.empty((n,), dtype=torch.int32, device="cuda")
    with pytest.raises(PyjacError, match="static scratch"):
        _lib.pyjac_newton_factor_solve_noalloc(M.handle, n, n, J.data_ptr(), h.data_ptr(), 0.5, b.data_ptr(),
                                               x.data_ptr(), 1, 4, 1e-14, info.data_ptr(), None)
    with pytest.raises(PyjacError):
        _lib.pyjac_newton_factor_solve_noalloc(M.handle, n, n, J.data_ptr(), h.data_ptr(), 0.5, b.data_ptr(),
                                               x.data_ptr(), 1 | 32, 4, 1e-14, info.data_ptr(), None)
