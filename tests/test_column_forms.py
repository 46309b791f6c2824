"""Which form of Jacobian column stream each test mechanism gets.

The library streams every row of a column unless most (row, column) pairs of
the Jacobian's species block have no mass-action or third-body terms; then it
streams only the rows with terms and writes the others from the dense part.
Both forms must be exercised by the GPU parity tests: this pins which
mechanisms take which form (the rule restated from the term structure of the
species-block derivatives, Sec. 3.1).
"""
import numpy as np

from conftest import ALL_KINDS, split_form_mech, tiny
from synth import config_mechanism


def empty_pair_fraction(mech):
    """Fraction of (row k, column j) pairs, j < N-1, with no column terms:
    a term exists where species k changes in a reaction whose rate depends on
    the concentration of species j (a reactant, a product of a reversible
    reaction, or a third body with efficiency other than 1)."""
    N = mech.n_species
    has = np.zeros((N, N - 1), dtype=bool)
    for r in mech.reactions:
        net = {}
        for s, nu in r.reac:
            net[s] = net.get(s, 0) - nu
        for s, nu in r.prod:
            net[s] = net.get(s, 0) + nu
        cols = [l for l, _ in r.reac]
        if r.rev != "irrev":
            cols += [l for l, _ in r.prod]
        if r.collider == "mix":
            cols += [l for l, a in r.eff.items() if a != 1.0]
        elif r.collider == "species":
            cols.append(r.collider_species)
        for k, nk in net.items():
            if nk:
                for l in cols:
                    if l != N - 1:
                        has[k, l] = True
    return 1.0 - has.mean()


def test_config_forms():
    frac = {c: empty_pair_fraction(config_mechanism(c)) for c in range(4)}
    for c in (0, 1, 2):
        assert frac[c] < 0.5, (c, frac[c])        # every row streamed
    assert frac[3] > 0.5, frac[3]                 # present rows only


def test_tiny_mechanisms_forms():
    # third-body efficiencies fill most pairs of a 7-species mechanism; the
    # purely elementary one is left sparse
    forms = {name: empty_pair_fraction(tiny(500 + ALL_KINDS.index(name), {name: 2, "elementary": 1},
                                            rev_mix={"kc": 1.0})) > 0.5 for name in ALL_KINDS}
    assert forms["elementary"] and not forms["thirdbody"], forms


def test_split_form_mechanisms():
    for seed, last in ((11, False), (12, True)):
        mech = split_form_mech(seed, reactive_last=last)
        assert mech.n_species > 32
        assert len({r.kind for r in mech.reactions}) == len(ALL_KINDS)
        assert empty_pair_fraction(mech) > 0.5
