"""Chemkin-format reader (pyjac_chemkin_to_text / pyjac_mech_load_chemkin).

CPU tests convert Chemkin text written from the synthetic mechanisms (and a
hand-made snippet of format variants with made-up numbers) and check the
result with the oracle against the same mechanism in the library's own
format: the Chemkin layout keeps 9 significant digits of the NASA
coefficients, so the reference is the mechanism with its coefficients
rounded the same way; unit conversions (cm-mol-s and cal/mol to SI-kmol and
T_a, atm to Pa) leave differences of a few ulp.  The GPU test loads a file
through the C ABI and checks it against the oracle.
"""
import ctypes

import numpy as np
import pytest

from conftest import ALL_KINDS, split_form_mech, tiny
from synth import config_mechanism, config_states, draw_states
from synth.chemkin import rounded_like_chemkin, to_chemkin

TOL = 1e-13


@pytest.fixture(scope="module")
def convert():
    from paper_1605_03262_amd import _lib, chemkin_to_text
    _lib.load_library()          # raises if the library is not built
    return chemkin_to_text


@pytest.fixture(scope="module")
def Ref(oracle_built):
    from oracle import RefMech
    return RefMech


def enorm(Ja, Jb):
    Ja, Jb = np.asarray(Ja), np.asarray(Jb)
    n = Ja.shape[-1]
    d = np.sqrt(((Ja - Jb) ** 2).reshape(-1, n).sum(0))
    return d / np.sqrt((Jb ** 2).reshape(-1, n).sum(0))


def compare(Ref, mech, tok, phi, p):
    """Converted text vs the rounded mechanism: Jacobian, production rates,
    per-reaction net rates q = c (R_f - R_r).  R_f, R_r and c agree one by
    one except for third-body reactions with a single collider species,
    which Chemkin writes with that species on both sides (c moves into R)."""
    a, b = Ref(text=tok), Ref(text=rounded_like_chemkin(mech).to_text())
    assert enorm(a.eval_jacobian(phi, p), b.eval_jacobian(phi, p)).max() <= TOL
    ra, rb = a.eval_rates(phi, p), b.eval_rates(phi, p)
    gross = rb["pres_mod"] * (np.abs(rb["rop_f"]) + np.abs(rb["rop_r"]))
    qa = ra["pres_mod"] * (ra["rop_f"] - ra["rop_r"])
    qb = rb["pres_mod"] * (rb["rop_f"] - rb["rop_r"])
    assert np.all(np.abs(qa - qb) <= TOL * gross + 1e-300)
    wg = np.abs(mech.stoich()[1] - mech.stoich()[0]) @ gross
    assert np.all(np.abs(ra["wdot"] - rb["wdot"]) <= TOL * wg + 1e-300)
    for i, r in enumerate(mech.reactions):
        if r.kind == "thirdbody" and r.collider == "species":
            continue
        for k in ("rop_f", "rop_r", "pres_mod"):
            assert np.all(np.abs(ra[k][i] - rb[k][i]) <= TOL * np.abs(rb[k][i]) + 1e-300), (i, k)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_config_mechanisms_round_trip(convert, Ref, cfg):
    mech = config_mechanism(cfg)
    phi, p = config_states(cfg, 9)
    compare(Ref, mech, convert(to_chemkin(mech)), phi, p)


@pytest.mark.parametrize("name", list(ALL_KINDS))
def test_every_reaction_class_round_trip(convert, Ref, name):
    mech = tiny(500 + ALL_KINDS.index(name), {name: 2, "elementary": 1},
                rev_mix={"kc": 1.0, "explicit": 1.0, "irrev": 1.0})
    phi, p = draw_states(3, mech.n_species, 11, T=(700.0, 2400.0), P_atm=(0.3, 80.0), dirichlet=0.5)
    compare(Ref, mech, convert(to_chemkin(mech)), phi, p)


def test_sparse_mechanism_round_trip(convert, Ref):
    mech = split_form_mech(12, reactive_last=True)
    phi, p = draw_states(5, mech.n_species, 11, T=(700.0, 2400.0), P_atm=(0.3, 80.0), dirichlet=0.5)
    compare(Ref, mech, convert(to_chemkin(mech)), phi, p)


@pytest.mark.parametrize("energy", ["KCAL/MOLE", "JOULES/MOLE", "KJOULES/MOLE", "KELVINS"])
def test_energy_units(convert, Ref, energy):
    mech = config_mechanism(0)
    phi, p = config_states(0, 9)
    compare(Ref, mech, convert(to_chemkin(mech, energy=energy)), phi, p)


def test_separate_thermo_and_standard_weights(convert):
    mech = config_mechanism(1)
    inline = convert(to_chemkin(mech))
    text, thermo = to_chemkin(mech, separate_thermo=True)
    assert convert(text, thermo) == inline
    # the synthetic mechanisms use the IUPAC abridged weights the reader knows
    assert convert(to_chemkin(mech, explicit_weights=False)) == inline


SNIPPET = """! format variants; all numbers made up
elem
  h o ar /39.95/
end
spec
  H  O2 HO2 OH H2O2 CH2(S)
  AR
end
reactions  kcal/mole
H + O2 (+AR) <=> HO2 (+AR)        1.0E+12  0.5  1.0
   LOW / 1.0D+18 -1.0 0.0 /
2OH(+M) = H2O2 (+M)               2.0e13   0.0  2.0
   low/ 3.0e17 -0.5 0.0/  TROE / 0.5 100.0 2000.0 /
   H2O2/5.0/ O2/0.5/
H + HO2 => 2 OH                   7.0E13  0.0  0.3
H + HO2 => 2OH                    1.0E13  0.0  0.0
   DUPLICATE
HO2 + M <=> H + O2 + M            3.0E15  -1.0  40.0
   REV / 1.0E16 -1.0 0.0 /
END
"""


def thermo_record(name, comp, a_high, a_low, tmid=1000.0):
    cf = "".join(f"{e:<2s}{c:3d}" for e, c in comp) + " " * (5 * (4 - len(comp)))
    l1 = f"{name:<18s}{'':6s}{cf}G{300.0:10.3f}{5000.0:10.3f}{tmid:8.2f}{'':6s}1"
    a = list(a_high) + list(a_low)
    return [l1, "".join(f"{v:15.8E}" for v in a[:5]) + "    2",
            "".join(f"{v:15.8E}" for v in a[5:10]) + "    3",
            "".join(f"{v:15.8E}" for v in a[10:]) + " " * 19 + "4"]


def snippet_thermo():
    comps = {"H": [("H", 1)], "O2": [("O", 2)], "HO2": [("H", 1), ("O", 2)], "OH": [("O", 1), ("H", 1)],
             "H2O2": [("H", 2), ("O", 2)], "CH2(S)": [("H", 2)], "AR": [("AR", 1)]}
    lines = ["THERMO"]
    for q, (n, c) in enumerate(comps.items()):
        base = [3.0 + 0.1 * q, 1.0e-3, -2.0e-7, 3.0e-11, -1.0e-15, -1.0e3 * (q + 1), 4.0 + q]
        lines += thermo_record(n, c, base, [b * 1.01 for b in base])
    return "\n".join(lines + ["END"]) + "\n"


def test_format_variants(convert, Ref):
    tok = convert(SNIPPET.replace("  AR\nend", "  AR\nend\n" + snippet_thermo().replace("THERMO\n", "thermo\n"), 1))
    blocks = tok.split("  reaction ")[1:]
    assert len(blocks) == 5
    kinds = [b.split("\n")[0] for b in blocks]
    assert kinds == ["falloff kc", "falloff kc", "elementary irrev", "elementary irrev", "thirdbody explicit"]
    assert "collider species AR" in blocks[0] and "lindemann" in blocks[0]
    assert "collider mix 2 H2O2 5 O2 0.5" in blocks[1] and "troe 3 0.5 100 2000" in blocks[1]
    assert "reactants 1 OH 2" in blocks[1] and "products 1 OH 2" in blocks[2]
    # units: k_inf bimolecular, k0 termolecular; E in kcal/mol -> T_a = E * 4184 / R
    def nums(block, key):
        line = [ln for ln in block.split("\n") if ln.strip().startswith(key)][0]
        return [float(v) for v in line.split()[1:]]
    hi, lo = nums(blocks[0], "high"), nums(blocks[0], "low")
    assert hi[0] == pytest.approx(1.0e12 * 1e-3, rel=1e-15) and lo[0] == pytest.approx(1.0e18 * 1e-6, rel=1e-15)
    assert hi[2] == pytest.approx(1.0 * 4184.0 / 8.314462618, rel=1e-15)
    rev = nums(blocks[4], "reverse")
    assert rev[0] == pytest.approx(1.0e16 * 1e-6, rel=1e-15)         # H + O2 + M: third order
    m = Ref(text=tok)
    phi, p = draw_states(1, 7, 4, dirichlet=0.5)
    assert np.all(np.isfinite(m.eval_jacobian(phi, p)))


def raw_status(text, thermo=None):
    from paper_1605_03262_amd import _lib
    lib = _lib.load_library()
    n = ctypes.c_size_t()
    st = lib.pyjac_chemkin_to_text(text.encode(), None if thermo is None else thermo.encode(), None, 0,
                                   ctypes.byref(n))
    return st, lib.pyjac_last_error().decode() if st else ""


@pytest.mark.parametrize("edit,status,needle", [
    (("H + HO2 => 2 OH", "H + HO2 => 2 OX"), -2, "line 15"),                  # unknown species
    (("reactions  kcal/mole", "reactions MOLECULES"), -3, "MOLECULES"),
    (("   DUPLICATE", "   FORD / H 1.0 /"), -3, "FORD"),
    (("   LOW / 1.0D+18 -1.0 0.0 /", "   LOW / 1.0D+18 -1.0 0.0 / HIGH / 1 0 0 /"), -2, "exactly one of LOW"),
    (("low/ 3.0e17 -0.5 0.0/", "low/ 3.0e17 -0.5 0.0"), -2, "unterminated"),
    (("2OH(+M) = H2O2 (+M)", "2OH(+M) = H2O2"), -2, "both sides"),
])
def test_errors(convert, edit, status, needle):
    text = SNIPPET.replace(*edit)
    st, msg = raw_status(text, snippet_thermo())
    assert st == status and needle in msg, (st, msg)


def test_missing_thermo_and_small_buffer(convert):
    st, msg = raw_status(SNIPPET)
    assert st == -2 and "no thermo data" in msg
    from paper_1605_03262_amd import _lib
    lib = _lib.load_library()
    n = ctypes.c_size_t()
    th = snippet_thermo().encode()
    assert lib.pyjac_chemkin_to_text(SNIPPET.encode(), th, None, 0, ctypes.byref(n)) == 0
    buf = ctypes.create_string_buffer(n.value - 1)
    assert lib.pyjac_chemkin_to_text(SNIPPET.encode(), th, buf, n.value - 1, ctypes.byref(n)) == -1


@pytest.mark.gpu
def test_load_chemkin_file_on_gpu(tmp_path, Ref):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_03262_amd import Mechanism, chemkin_to_text
    mech = config_mechanism(1)
    text, thermo = to_chemkin(mech, separate_thermo=True)
    (tmp_path / "mech.ck").write_text(text)
    (tmp_path / "therm.dat").write_text(thermo)
    M = Mechanism.from_chemkin(str(tmp_path / "mech.ck"), str(tmp_path / "therm.dat"))
    assert (M.n_species, M.n_reactions) == (mech.n_species, mech.n_reactions)
    phi, p = config_states(1, 64)
    J = M.eval_jacobian(torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()).cpu().numpy()
    Jr = Ref(text=chemkin_to_text(text, thermo)).eval_jacobian(phi, p)
    assert enorm(J, np.asarray(Jr).reshape(J.shape)).max() <= 1e-10
