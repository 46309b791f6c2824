"""The hot path under HIP graph capture.

After one eager call per launch shape (which builds the shape's device
tables), the Jacobian and the Newton solve enqueue only kernels on the
caller's stream: no allocation, no host synchronization and no memset node
(counters are cleared by a kernel).  A graph captured once is replayed on new
inputs, with eager work and synchronizations between the replays, and every
replay must equal the eager result bitwise.
"""
import numpy as np
import pytest

from synth import NEWTON_GAMMA, config_mechanism, config_states, conditioned_steps, draw_newton_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.mark.parametrize("cfg,n,mode", [(1, 700, 1), (1, 700, 0), (2, 96, 1)])
def test_captured_step_replays_match_eager(torch, cfg, n, mode):
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    M = Mechanism(text=mech.to_text())
    inputs = []
    for k in range(4):
        phi, p = config_states(cfg, n) if k == 0 else config_states(cfg, n + 37 * k)
        phi, p = phi[:, -n:], p[-n:]                      # different states each time
        jac0 = M.eval_jacobian(torch.from_numpy(np.ascontiguousarray(phi)).cuda(),
                               torch.from_numpy(np.ascontiguousarray(p)).cuda())
        rows = torch.abs(jac0.view(N, N, n)).sum(dim=1).cpu().numpy()
        h = conditioned_steps(100 + k, rows)
        b = draw_newton_inputs(200 + k, N, n)[1]
        inputs.append(tuple(np.ascontiguousarray(a) for a in (phi, p, h, b)))
    d_phi, d_p, d_h, d_b = (torch.from_numpy(a.copy()).cuda() for a in inputs[0])
    jac = torch.empty((N * N, n), dtype=torch.float64, device="cuda")
    ws = torch.empty((max(M.newton_workspace_bytes(n, mode), 1),), dtype=torch.uint8, device="cuda")

    def step():
        M.eval_jacobian(d_phi, d_p, out=jac)
        return M.newton_solve(jac, d_h, d_b, NEWTON_GAMMA, mode=mode, workspace=ws)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                            # warm-up: launch tables built here
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        x_g, info_g = step()
    for k in (1, 2, 3, 1):
        for dst, src in zip((d_phi, d_p, d_h, d_b), inputs[k]):
            dst.copy_(torch.from_numpy(src))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        J_r, x_r, i_r = jac.cpu().numpy(), x_g.cpu().numpy(), info_g.cpu().numpy()
        # eager reference on the same inputs, in fresh buffers
        e_phi, e_p, e_h, e_b = (torch.from_numpy(a.copy()).cuda() for a in inputs[k])
        J_e = M.eval_jacobian(e_phi, e_p)
        x_e, i_e = M.newton_solve(J_e, e_h, e_b, NEWTON_GAMMA, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(J_r, J_e.cpu().numpy()), k
        assert np.array_equal(x_r, x_e.cpu().numpy()), k
        assert np.array_equal(i_r[:n], i_e.cpu().numpy()[:n]), k
