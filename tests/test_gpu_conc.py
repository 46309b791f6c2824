"""GPU parity of the concentration-based, constant-volume Jacobian (Sec. 3.3's
sparse formulation) against the oracle's dense Jacobian of the same RHS.

The GPU writes, per state, the temperature column and row, the dense row
parts u_k and the values of the sparse part S in a fixed compressed-column
pattern; the test rebuilds the dense (N+1) x (N+1) matrix (J_kj = u_k + S_kj)
and gates it at E_norm <= 1e-10 per state.  The pattern itself is compared with
one derived here from the mechanism's reactions.
"""
import numpy as np
import pytest

from conftest import ALL_KINDS, BLENDED, species_collider_mech, tiny, zero_collider_states
from synth import WORKLOADS, config_mechanism, config_states, draw_states
from test_gpu_parity import JAC_TOL, enorm_per_state
from test_oracle_conc_pins import conc_states

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


def expected_pattern(mech):
    """Rows of S per column from the reaction definitions: row k with nu_k != 0,
    column l a reactant, a product of a reversible reaction, a non-unit
    efficiency species or the single collider species."""
    N = mech.n_species
    S = np.zeros((N, N), bool)
    for r in mech.reactions:
        net = {}
        for k, n in r.reac:
            net[k] = net.get(k, 0) - n
        for k, n in r.prod:
            net[k] = net.get(k, 0) + n
        rows = [k for k, v in net.items() if v]
        cols = {k for k, _ in r.reac}
        if r.rev != "irrev":
            cols |= {k for k, _ in r.prod}
        if r.collider == "mix":
            cols |= {l for l, a in r.eff.items() if a != 1.0}
        elif r.collider == "species":
            cols.add(r.collider_species)
        for k in rows:
            for j in cols:
                S[k, j] = True
    return S


def densify(out, colptr, rowidx, N):
    """GPU output [3N+1+nnz, n] -> dense [(N+1)^2, n] row-major."""
    n = out.shape[1]
    J = np.zeros((N + 1, N + 1, n))
    J[0, 0] = out[0]
    J[1:, 0] = out[1:N + 1]
    J[0, 1:] = out[N + 1:2 * N + 1]
    J[1:, 1:] = out[2 * N + 1:3 * N + 1][:, None, :]
    vals = out[3 * N + 1:]
    for j in range(N):
        for q in range(colptr[j], colptr[j + 1]):
            J[1 + rowidx[q], 1 + j] += vals[q]
    return J.reshape((N + 1) ** 2, n)


def gpu_conc(torch, M, c, ld=None):
    n = c.shape[1]
    ld = ld or n
    buf = np.zeros((c.shape[0], ld))
    buf[:, :n] = c
    buf[0, n:] = 1500.0
    buf[1:, n:] = 1e-3
    d = torch.from_numpy(buf).cuda()
    view = d.as_strided((c.shape[0], n), (ld, 1))
    out = M.eval_jacobian_conc(view)
    torch.cuda.synchronize()
    return out[:, :n].cpu().numpy()


def check(torch, Ref, mech, c, label, ld=None):
    from paper_1605_03262_amd import Mechanism
    M = Mechanism(text=mech.to_text())
    colptr, rowidx = M.conc_pattern()
    N = mech.n_species
    S = np.zeros((N, N), bool)
    for j in range(N):
        S[rowidx[colptr[j]:colptr[j + 1]], j] = True
        assert np.all(np.diff(rowidx[colptr[j]:colptr[j + 1]]) > 0)
    assert np.array_equal(S, expected_pattern(mech)), label
    out = gpu_conc(torch, M, c, ld)
    assert np.all(np.isfinite(out)), label
    Jg = densify(out, colptr, rowidx, N)
    Jr = Ref(text=mech.to_text()).eval_jacobian_conc(c)
    e = enorm_per_state(Jg, Jr)
    assert e.max() <= JAC_TOL, f"{label}: max E_norm {e.max():.3e}"
    return M, out, e


CASES = [(k, {k: 2, "elementary": 1}) for k in ALL_KINDS] + [(f"mixed{s}", None) for s in range(4)]


@pytest.mark.parametrize("name,kinds", CASES, ids=[c[0] for c in CASES])
def test_conc_tiny(torch, Ref, name, kinds):
    if kinds is None:
        s = int(name[5:])
        rng = np.random.default_rng(910 + s)
        kinds = {k: int(rng.integers(0, 2)) for k in ALL_KINDS}
        kinds["elementary"] += 2
        mech = tiny(720 + s, kinds, n_species=8, reactive_last=(s % 2 == 0),
                    rev_mix={"kc": 2, "explicit": 1, "irrev": 1})
    else:
        mech = tiny(540 + ALL_KINDS.index(name), kinds, rev_mix={"kc": 1.0})
    phi, p = draw_states(21, mech.n_species, 77, T=(700.0, 2400.0), P_atm=(0.3, 80.0), dirichlet=0.5)
    check(torch, Ref, mech, conc_states(mech, phi, p), name, ld=83)


@pytest.mark.parametrize("kind", BLENDED)
def test_conc_absent_collider(torch, Ref, kind):
    mech, m_sp = species_collider_mech(kind, 150 + BLENDED.index(kind))
    phi, p = zero_collider_states(mech, m_sp, 9)
    c = conc_states(mech, phi, p)
    c[1 + m_sp] = np.where(phi[1 + m_sp] == 0, 0.0, c[1 + m_sp])
    check(torch, Ref, mech, c, kind)


@pytest.mark.parametrize("cfg,n", [(0, 1000), (1, 1000), (2, 200), (3, 24)])
def test_conc_configs(torch, Ref, cfg, n):
    mech = config_mechanism(cfg)
    phi, p = config_states(cfg, n)
    _, out, e = check(torch, Ref, mech, conc_states(mech, phi, p), f"C{cfg}")
    print(f"C{cfg}: rows per state {out.shape[0]} (dense {(mech.n_species + 1) ** 2}); max E_norm {e.max():.2e}")


def test_conc_shapes_and_batch_independence(torch):
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(1)
    phi, p = config_states(1, 300)
    c = conc_states(mech, phi, p)
    M = Mechanism(text=mech.to_text())
    base = gpu_conc(torch, M, c)
    assert np.array_equal(base, gpu_conc(torch, M, c, ld=311))
    assert np.array_equal(base[:, 17:18], gpu_conc(torch, M, c[:, 17:18]))
    tried = 0
    for ts, nt in ((16, 1024), (8, 512), (8, 1024), (4, 512), (4, 1024), (2, 512), (8, 256), (4, 256)):
        try:
            M.set_variant(2, ts, nt)
        except Exception:
            continue
        tried += 1
        assert np.array_equal(base, gpu_conc(torch, M, c)), (ts, nt)
    assert tried >= 3


@pytest.mark.parametrize("cfg,n_sample", [(1, 64), (2, 32), (3, 8)])
def test_conc_full_size_sampled(torch, Ref, cfg, n_sample):
    """The full batch, autotuned as the benchmark times it; sampled states
    against the oracle."""
    from paper_1605_03262_amd import Mechanism
    mech = config_mechanism(cfg)
    N = mech.n_species
    phi, p = config_states(cfg)
    c = conc_states(mech, phi, p)
    n = c.shape[1]
    M = Mechanism(text=mech.to_text())
    dc = torch.from_numpy(c).cuda()
    out = torch.empty((3 * N + 1 + len(M.conc_pattern()[1]), n), dtype=torch.float64, device="cuda")
    M.autotune(2, dc, None, out=out, reps=1)
    M.eval_jacobian_conc(dc, out=out)
    rng = np.random.default_rng(cfg)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, n_sample, replace=False)]))
    o = out[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    colptr, rowidx = M.conc_pattern()
    e = enorm_per_state(densify(o, colptr, rowidx, N), Ref(text=mech.to_text()).eval_jacobian_conc(c[:, idx]))
    assert e.max() <= JAC_TOL, e.max()
    print(f"C{cfg} conc full n={n}: shape {M.get_variant(2)[:2]}, max E_norm {e.max():.2e}")
