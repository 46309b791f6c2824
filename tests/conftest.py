import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_built():
    from oracle import build_oracle
    return build_oracle(force=False)


# Reaction classes for the tiny pin mechanisms.
ALL_KINDS = ("elementary", "thirdbody", "falloff_lindemann", "falloff_troe", "falloff_sri",
             "chemact_lindemann", "chemact_troe", "chemact_sri", "plog", "cheb")


def tiny(seed, kinds, n_species=7, reactive_last=False, rev_mix=None, allow_shared=False,
         collider_probs=(0.25, 0.25)):
    from synth import tiny_mechanism
    return tiny_mechanism(seed, kinds, n_species=n_species, reactive_last=reactive_last,
                          rev_mix=rev_mix or {"kc": 1.0}, elements=("H", "O"),
                          bounds={"H": 3, "O": 3}, allow_shared=allow_shared,
                          collider_probs=collider_probs)


def split_form_mech(seed, reactive_last=False):
    """40 species, one reaction of every class plus elementary ones: most
    (row, column) pairs of the Jacobian have no terms, and the species span two
    32-row blocks."""
    from synth import tiny_mechanism
    kinds = {k: 1 for k in ALL_KINDS}
    kinds["elementary"] += 3
    return tiny_mechanism(seed, kinds, n_species=40, reactive_last=reactive_last,
                          rev_mix={"kc": 2, "explicit": 1, "irrev": 1},
                          elements=("C", "H", "O", "N"), bounds={"C": 2, "H": 5, "O": 3, "N": 1})


# Falloff and chemically activated classes with a blending function.
BLENDED = [f"{a}_{b}" for a in ("falloff", "chemact") for b in ("lindemann", "troe", "sri")]


def species_collider_mech(kind, seed):
    """One reaction of the class with a single-species collider m, plus two
    elementary reactions; m is not the implied last species."""
    for attempt in range(40):
        mech = tiny(seed + 1000 * attempt, {kind: 1, "elementary": 2}, collider_probs=(0.0, 1.0))
        r = next(x for x in mech.reactions if x.kind == kind)
        if r.collider_species != mech.n_species - 1:
            return mech, r.collider_species
    raise RuntimeError("no mechanism with a non-last collider species")


def zero_collider_states(mech, m, seed, values=(0.0, 0.0, -1e-14, 0.0)):
    phi, p = _draw_states(seed, mech.n_species, len(values), dirichlet=0.7)
    for s, v in enumerate(values):
        phi[1 + m, s] = v
    if len(values) > 3:
        phi[1:, 3] = np.where(np.arange(mech.n_species - 1) == m, 0.0, phi[1:, 3])
        phi[1 + (m + 1) % (mech.n_species - 1), 3] = 0.0     # a second zero species
    return phi, p


def _draw_states(*a, **k):
    from synth import draw_states
    return draw_states(*a, **k)
