"""Chemkin-II text for a synthetic mechanism (test input for the library's
Chemkin reader).

Writes the usual cm-mol-s / cal-mol units: A in (cm^3/mol)^(order-1)/s with
order the molecularity of that rate coefficient ([M] counted for third-body
and falloff low-pressure-limit coefficients; the high-pressure limit of a
chemically activated reaction has one order less), activation energies in the chosen
energy unit, pressures in atm, NASA-7 records in the fixed 80-column layout
with 15-column E15.8 coefficients (9 significant digits, as the format
allows).  `rounded_like_chemkin` returns the mechanism with its NASA
coefficients rounded the same way, the exact counterpart of what a reader of
this text sees.
"""
from __future__ import annotations

import copy

from .mechgen import ATM, Mechanism

R_J_PER_MOL_K = 8.314462618
ENERGY_PER_K = {  # energy unit per kelvin of activation temperature
    "CAL/MOLE": R_J_PER_MOL_K / 4.184,
    "KCAL/MOLE": R_J_PER_MOL_K / 4184.0,
    "JOULES/MOLE": R_J_PER_MOL_K,
    "KJOULES/MOLE": R_J_PER_MOL_K / 1000.0,
    "KELVINS": 1.0,
}


def _e15(v: float) -> str:
    return f"{v:15.8E}"


def rounded_like_chemkin(mech: Mechanism) -> Mechanism:
    m = copy.deepcopy(mech)
    for sp in m.species:
        sp.low = [float(_e15(a)) for a in sp.low]
        sp.high = [float(_e15(a)) for a in sp.high]
    return m


def _thermo_records(mech: Mechanism) -> list:
    out = []
    for sp in mech.species:
        comp = [(e, c) for e, c in sp.comp.items() if c]
        if len(comp) > 4:
            raise ValueError(f"{sp.name}: more than 4 elements")
        tm = f"{sp.tmid:8.2f}"
        if float(tm) != sp.tmid:
            raise ValueError(f"{sp.name}: T_mid {sp.tmid!r} is not exact in 8.2f")
        cfields = "".join(f"{e.upper():<2s}{c:3d}" for e, c in comp) + " " * (5 * (4 - len(comp)))
        l1 = f"{sp.name:<18s}{'':6s}{cfields}G{200.0:10.3f}{6000.0:10.3f}{tm}{'':6s}1"
        a = list(sp.high) + list(sp.low)
        l2 = "".join(_e15(v) for v in a[0:5]) + "    2"
        l3 = "".join(_e15(v) for v in a[5:10]) + "    3"
        l4 = "".join(_e15(v) for v in a[10:14]) + " " * 19 + "4"
        out += [l1, l2, l3, l4]
    return out


def to_chemkin(mech: Mechanism, energy: str = "CAL/MOLE", separate_thermo: bool = False,
               explicit_weights: bool = True):
    """Chemkin text of `mech`; with separate_thermo, returns (mech_text,
    thermo_text) and the mechanism text has no THERMO block."""
    from .mechgen import ATOMIC_WEIGHTS
    e_per_k = ENERGY_PER_K[energy]
    names = [s.name for s in mech.species]
    lines = ["! synthetic mechanism " + mech.name, "ELEMENTS"]
    lines.append(" ".join(f"{e} /{ATOMIC_WEIGHTS[e]!r}/" if explicit_weights else e for e in mech.elements))
    lines += ["END", "SPECIES"]
    for k in range(0, len(names), 6):
        lines.append("  ".join(names[k:k + 6]))
    lines.append("END")
    thermo = ["THERMO ALL", f"{300.0:10.3f}{1000.0:10.3f}{5000.0:10.3f}"] + _thermo_records(mech) + ["END"]
    if not separate_thermo:
        lines += thermo
    lines.append("REACTIONS" + ("" if energy == "CAL/MOLE" else f" {energy}") + " MOLES")

    def arr(A, b, Ta, order):
        return f"{A * 1e3 ** (order - 1)!r} {b!r} {Ta * e_per_k!r}"

    def side(terms):
        return " + ".join((f"{n}{names[k]}" if n > 1 else names[k]) for k, n in terms)

    for r in mech.reactions:
        nf = sum(n for _, n in r.reac)
        nr = sum(n for _, n in r.prod)
        tb = ""
        reac, prod = list(r.reac), list(r.prod)
        if r.kind == "thirdbody" and r.collider == "species":
            # no "+M" form for a single collider species: it appears on both
            # sides of an elementary reaction (the same rate expression)
            x = r.collider_species
            reac = [(k, n + (k == x)) for k, n in reac] + ([(x, 1)] if x not in dict(reac) else [])
            prod = [(k, n + (k == x)) for k, n in prod] + ([(x, 1)] if x not in dict(prod) else [])
        elif r.kind == "thirdbody":
            tb = " + M"
        elif r.low is not None:
            tb = " (+M)" if r.collider == "mix" else f" (+{names[r.collider_species]})"
        arrow = " => " if r.rev == "irrev" else " <=> "
        eq = side(reac) + tb + arrow + side(prod) + tb
        aux = []
        if r.kind in ("elementary",):
            main = arr(*r.arr, nf)
        elif r.kind == "thirdbody":
            main = arr(*r.arr, nf + 1)
        elif r.low is not None:
            if r.kind.startswith("falloff"):
                main = arr(*r.high, nf)
                aux.append(f"LOW / {arr(*r.low, nf + 1)} /")
            else:   # chemically activated: k0 has the rate's order, k_inf one less
                main = arr(*r.low, nf)
                aux.append(f"HIGH / {arr(*r.high, nf - 1)} /")
            if r.troe is not None:
                aux.append("TROE / " + " ".join(repr(float(v)) for v in r.troe) + " /")
            elif r.sri is not None:
                aux.append("SRI / " + " ".join(repr(float(v)) for v in r.sri) + " /")
        elif r.kind == "plog":
            main = "1.0 0.0 0.0"
            for p, A, b, Ta in r.plog:
                aux.append(f"PLOG / {p / ATM!r} {arr(A, b, Ta, nf)} /")
        elif r.kind == "cheb":
            c = r.cheb
            main = "1.0 0.0 0.0"
            coef = [float(v) for row in c["coef"] for v in row]
            coef[0] += 3.0 * (nf - 1)
            aux.append(f"TCHEB / {c['Tmin']!r} {c['Tmax']!r} /  PCHEB / {c['Pmin'] / ATM!r} {c['Pmax'] / ATM!r} /")
            aux.append(f"CHEB / {c['nT']} {c['nP']} /")
            for q in range(0, len(coef), 4):
                aux.append("CHEB / " + " ".join(repr(v) for v in coef[q:q + 4]) + " /")
        else:
            raise ValueError(r.kind)
        if r.collider == "mix" and r.eff:
            aux.append(" ".join(f"{names[k]}/{float(a)!r}/" for k, a in sorted(r.eff.items())))
        if r.reverse is not None:
            aux.append(f"REV / {arr(*r.reverse, nr + (1 if r.kind == 'thirdbody' else 0))} /")
        lines.append(f"{eq}   {main}")
        lines += ["    " + a for a in aux]
    lines.append("END")
    text = "\n".join(lines) + "\n"
    if separate_thermo:
        return text, "\n".join(thermo) + "\n"
    return text
