"""GPU complex-step Jacobian (Sec. 5.1's accuracy references; the paper names
complex-step derivatives as an option it did not explore) against the oracle:
the analytical Jacobian (E_norm <= 1e-10, the Jacobian gate) and the oracle's
own complex-step Jacobian of the same RHS."""
import numpy as np
import pytest

from conftest import ALL_KINDS, BLENDED, species_collider_mech, tiny, zero_collider_states
from synth import config_mechanism, config_states, draw_states
from test_gpu_parity import JAC_TOL, enorm_per_state

pytestmark = pytest.mark.gpu


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


def gpu_cs(torch, mech, phi, p, ld=None):
    from paper_1605_03262_amd import Mechanism
    M = Mechanism(text=mech.to_text())
    n = phi.shape[1]
    ld = ld or n
    a = np.zeros((phi.shape[0], ld))
    a[:, :n] = phi
    a[0, n:] = 1500.0
    a[1:, n:] = 1.0 / phi.shape[0]
    b = np.full(ld, 101325.0)
    b[:n] = p
    d = torch.from_numpy(a).cuda()
    view = d.as_strided((phi.shape[0], n), (ld, 1))
    J = M.eval_jacobian_cs(view, torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    return J[:, :n].cpu().numpy()


def check(torch, Ref, mech, phi, p, label, ld=None):
    Jg = gpu_cs(torch, mech, phi, p, ld)
    assert np.all(np.isfinite(Jg)), label
    ref = Ref(text=mech.to_text())
    e = enorm_per_state(Jg, ref.eval_jacobian(phi, p))
    assert e.max() <= JAC_TOL, f"{label}: vs analytical {e.max():.3e}"
    ec = enorm_per_state(Jg, ref.eval_jacobian_cs(phi, p))
    assert ec.max() <= 1e-12, f"{label}: vs oracle complex step {ec.max():.3e}"
    return e


CASES = [(k, {k: 2, "elementary": 1}) for k in ALL_KINDS] + [(f"mixed{s}", None) for s in range(4)]


@pytest.mark.parametrize("name,kinds", CASES, ids=[c[0] for c in CASES])
def test_cs_tiny(torch, Ref, name, kinds):
    if kinds is None:
        s = int(name[5:])
        rng = np.random.default_rng(900 + s)
        kinds = {k: int(rng.integers(0, 2)) for k in ALL_KINDS}
        kinds["elementary"] += 2
        mech = tiny(700 + s, kinds, n_species=8, reactive_last=(s % 2 == 0),
                    rev_mix={"kc": 2, "explicit": 1, "irrev": 1})
    else:
        mech = tiny(500 + ALL_KINDS.index(name), kinds, rev_mix={"kc": 1.0})
    phi, p = draw_states(11, mech.n_species, 77, T=(700.0, 2400.0), P_atm=(0.3, 80.0), dirichlet=0.5)
    check(torch, Ref, mech, phi, p, name, ld=83)


@pytest.mark.parametrize("kind", BLENDED)
def test_cs_absent_collider(torch, Ref, kind):
    mech, m_sp = species_collider_mech(kind, 150 + BLENDED.index(kind))
    phi, p = zero_collider_states(mech, m_sp, 9)
    check(torch, Ref, mech, phi, p, kind)


@pytest.mark.parametrize("cfg,n", [(0, 500), (1, 300), (2, 40)])
def test_cs_configs(torch, Ref, cfg, n):
    mech = config_mechanism(cfg)
    phi, p = config_states(cfg, n)
    e = check(torch, Ref, mech, phi, p, f"C{cfg}")
    print(f"C{cfg} complex step vs analytical: max E_norm {e.max():.2e}")


def test_cs_arguments(torch):
    from paper_1605_03262_amd import Mechanism, PyjacError, _lib
    mech = config_mechanism(0)
    M = Mechanism(text=mech.to_text())
    N = mech.n_species
    phi, p = config_states(0, 4)
    d, dp = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    J = torch.empty((N * N, 4), dtype=torch.float64, device="cuda")
    for step in (0.0, -1e-30, 1e-3):
        with pytest.raises(PyjacError):
            _lib.pyjac_eval_jacobian_cs(M.handle, 4, 4, d.data_ptr(), dp.data_ptr(), step, J.data_ptr(), None)
    _lib.pyjac_eval_jacobian_cs(M.handle, 0, 4, d.data_ptr(), dp.data_ptr(), 1e-30, J.data_ptr(), None)
