import os
import sys

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
