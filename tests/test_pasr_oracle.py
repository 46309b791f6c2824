"""Pins of the oracle's PaSR mixing step (App. C): the pairwise relaxation
conserves each pair's enthalpy and mass, w = 0 is the identity, w = 1/2 gives
both particles the pair mean, and the temperature recovered from an enthalpy
reproduces the temperature it came from."""
import numpy as np
import pytest

from synth import config_mechanism, config_states, pasr_fresh


@pytest.fixture(scope="module")
def setup(oracle_built):
    from oracle import RefMech
    mech = config_mechanism(1)
    return mech, RefMech(text=mech.to_text()), mech.molecular_weights()


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.permutation(n)
    partner = np.empty(n, dtype=np.int32)
    partner[idx[0::2]] = idx[1::2]
    partner[idx[1::2]] = idx[0::2]
    return partner


def _full(phi):
    return np.vstack([phi[1:], 1 - phi[1:].sum(axis=0)])


def test_pair_conservation(setup):
    from oracle.pasr_ref import mix_pairs, mixture_enthalpy
    mech, ref, W = setup
    phi, _ = config_states(1, 20)
    partner = _pairs(20, 1)
    out = mix_pairs(ref, W, phi, partner, 0.3)
    Y0, Y1 = _full(phi), _full(out)
    for s in range(20):
        q = partner[s]
        if s > q:
            continue
        h0 = mixture_enthalpy(ref, W, phi[0, s], Y0[:, s])[0] + mixture_enthalpy(ref, W, phi[0, q], Y0[:, q])[0]
        h1 = mixture_enthalpy(ref, W, out[0, s], Y1[:, s])[0] + mixture_enthalpy(ref, W, out[0, q], Y1[:, q])[0]
        scale = abs(mixture_enthalpy(ref, W, phi[0, s], Y0[:, s])[0]) + abs(
            mixture_enthalpy(ref, W, phi[0, q], Y0[:, q])[0])
        assert abs(h1 - h0) <= 1e-12 * scale
        np.testing.assert_allclose(Y1[:, s] + Y1[:, q], Y0[:, s] + Y0[:, q], rtol=0, atol=1e-15)


def test_identity_and_mean(setup):
    from oracle.pasr_ref import mix_pairs
    mech, ref, W = setup
    phi, _ = config_states(1, 10)
    partner = _pairs(10, 2)
    np.testing.assert_allclose(mix_pairs(ref, W, phi, partner, 0.0), phi, rtol=1e-14)
    out = mix_pairs(ref, W, phi, partner, 0.5)
    for s in range(10):
        q = partner[s]
        np.testing.assert_allclose(out[:, s], out[:, q], rtol=1e-12)


def test_temperature_round_trip(setup):
    from oracle.pasr_ref import mixture_enthalpy, temperature_from_enthalpy
    mech, ref, W = setup
    comp = pasr_fresh(mech, 600.0, 3)
    Y = np.append(comp[1:], 1 - comp[1:].sum())
    for T in (350.0, 999.0, 1000.0, 1001.0, 2400.0):
        h, _ = mixture_enthalpy(ref, W, T, Y)
        assert abs(temperature_from_enthalpy(ref, W, h, Y, 1500.0) - T) <= 1e-11 * T
