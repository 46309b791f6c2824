"""Finite-difference Jacobian on the GPU (the paper's comparison method,
Sec. 5): forward differences of the GPU RHS, checked against the oracle's
analytical Jacobian and for independence of the chunking."""
import numpy as np
import pytest

from synth import config_mechanism, config_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def _enorm(Jg, Jr, N):
    # per-state relative Frobenius error on row-scaled matrices (as in the
    # analytical parity tests), so that no norm overflows
    n = Jg.shape[1]
    A = Jg.reshape(N, N, n)
    B = Jr.reshape(N, N, n)
    sc = np.max(np.abs(B), axis=1, keepdims=True)
    sc[sc == 0] = 1.0
    A, B = A / sc, B / sc
    return np.sqrt(((A - B) ** 2).sum(axis=(0, 1)) / (B ** 2).sum(axis=(0, 1)))


@pytest.mark.parametrize("cfg,n", [(0, 300), (1, 120)])
def test_fd_matches_host_differences_of_the_gpu_rhs(cfg, n):
    """The FD Jacobian is exactly the forward-difference quotient of the GPU
    RHS (itself pinned to the oracle by the parity tests): perturbed states
    built on the host with the documented increments, evaluated by
    eval_rates and differenced on the host, agree bit for bit.  (2^-26 is a
    power of two, so the increment arithmetic is exact on both sides.)"""
    import torch
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, n)
    M = Mechanism(text=mech.to_text())
    Jf = M.eval_jacobian_fd(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()).cpu().numpy()
    floor = np.full(N, 1e-10)
    floor[0] = 1.0
    cols = [phi]
    incs = np.empty((N, n))
    for j in range(N):
        q = phi.copy()
        vp = phi[j] + 2.0 ** -26 * np.maximum(np.abs(phi[j]), floor[j])
        incs[j] = vp - phi[j]
        q[j] = vp
        cols.append(q)
    big = np.ascontiguousarray(np.concatenate(cols, axis=1))
    pp = np.tile(p, N + 1)
    f = M.eval_rates(torch.from_numpy(big).cuda(), torch.from_numpy(pp).cuda(), rop_f=False, rop_r=False,
                     pres_mod=False, wdot=False)["dphi"].cpu().numpy()
    f0 = f[:, :n]
    J = np.empty((N, N, n))
    for j in range(N):
        J[:, j, :] = (f[:, (j + 1) * n:(j + 2) * n] - f0) / incs[j]
    assert np.array_equal(J.reshape(N * N, n), Jf)


@pytest.mark.parametrize("cfg,n", [(0, 300), (1, 120)])
def test_fd_error_against_analytical(Ref, cfg, n):
    """Diagnostic, as in the paper's accuracy comparison: the FD Jacobian's
    distance from the exact one (row-scaled relative Frobenius error).  Only
    finiteness is asserted: forward differences lose accuracy wherever a mass
    fraction is far below the increment floor, which is the method's own
    error, not the implementation's."""
    import torch
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg, n)
    Jr = Ref(text=mech.to_text()).eval_jacobian(phi, p)
    M = Mechanism(text=mech.to_text())
    Jf = M.eval_jacobian_fd(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    e = _enorm(Jf.cpu().numpy(), Jr, N)
    assert np.all(np.isfinite(e))
    print(f"C{cfg} FD vs analytical E_norm: median {np.median(e):.2e} p90 {np.percentile(e, 90):.2e} "
          f"max {e.max():.2e}")


def test_fd_chunking_does_not_change_results():
    import torch
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(1)
    phi, p = config_states(1, 50)
    M = Mechanism(text=mech.to_text())
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    J1 = M.eval_jacobian_fd(d_phi, d_p, chunk_states=50).cpu().numpy()
    J2 = M.eval_jacobian_fd(d_phi, d_p, chunk_states=7).cpu().numpy()
    assert np.array_equal(J1, J2)


def test_fd_workspace_too_small():
    import torch
    from paper_1605_03262_amd import Mechanism, PyjacError, _lib
    mech = config_mechanism(0)
    N = mech.n_species
    phi, p = config_states(0, 4)
    M = Mechanism(text=mech.to_text())
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    J = torch.empty((N * N, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty((64,), dtype=torch.uint8, device="cuda")
    with pytest.raises(PyjacError):
        _lib.pyjac_eval_jacobian_fd(M.handle, 4, 4, d_phi.data_ptr(), d_p.data_ptr(), J.data_ptr(),
                                    ws.data_ptr(), 64, None)
