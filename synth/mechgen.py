"""Seeded synthetic kinetic mechanisms shaped like the paper's benchmark models.

This module only *builds inputs*: element-balanced reactions, NASA-7 thermo fits
and Arrhenius/falloff/PLOG/Chebyshev parameters. It evaluates no reaction rate,
no equilibrium constant and no derivative, so that both the CPU oracle and the
GPU library can consume its output without sharing any of the method's
arithmetic.

Units written to the mechanism file (SI-kmol throughout):
  W [kg/kmol], Arrhenius A in (m^3/kmol)^(order-1)/s, activation temperature
  Ta [K], pressures [Pa], Chebyshev coefficients for log10 k in SI units.
Random draws follow the paper-shaped recipe: A log-uniform over [1e5, 1e15] in
cm-mol-s units (converted by 1e-3^(order-1)), beta ~ U[-2, 3],
Ea ~ U[0, 50] kcal/mol (converted to Ta = Ea * 4184 / 8.314462618 K).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ATOMIC_WEIGHTS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "Ar": 39.95}
KCAL_PER_MOL_TO_K = 4184.0 / 8.314462618  # Ea [kcal/mol] -> Ta [K]
ATM = 101325.0
CGS_TO_SI_PER_ORDER = 1.0e-3  # (cm^3/mol) -> (m^3/kmol)

REACTION_TYPES = (
    "elementary", "thirdbody",
    "falloff_lindemann", "falloff_troe", "falloff_sri",
    "chemact_lindemann", "chemact_troe", "chemact_sri",
    "plog", "cheb",
)


@dataclasses.dataclass
class Species:
    name: str
    comp: Dict[str, int]
    W: float
    tmid: float
    low: List[float]     # a0..a6 valid for T <= tmid
    high: List[float]    # a0..a6 valid for T > tmid
    inert: bool = False


@dataclasses.dataclass
class Reaction:
    kind: str                       # one of REACTION_TYPES
    rev: str                        # "kc" | "explicit" | "irrev"
    reac: List[Tuple[int, int]]     # (species index, nu')
    prod: List[Tuple[int, int]]     # (species index, nu'')
    arr: Optional[Tuple[float, float, float]] = None   # elementary / thirdbody
    low: Optional[Tuple[float, float, float]] = None   # falloff / chemact k0
    high: Optional[Tuple[float, float, float]] = None  # falloff / chemact kinf
    troe: Optional[Tuple[float, ...]] = None           # (a, T3, T1[, T2])
    sri: Optional[Tuple[float, ...]] = None            # (a, b, c, d, e)
    collider: Optional[str] = None                      # "mix" | "species"
    eff: Dict[int, float] = dataclasses.field(default_factory=dict)
    collider_species: Optional[int] = None
    plog: Optional[List[Tuple[float, float, float, float]]] = None  # (p, A, b, Ta)
    cheb: Optional[dict] = None     # {nT, nP, Tmin, Tmax, Pmin, Pmax, coef (nT x nP)}
    reverse: Optional[Tuple[float, float, float]] = None

    @property
    def order_fwd(self) -> int:
        return sum(n for _, n in self.reac)


@dataclasses.dataclass
class Mechanism:
    elements: List[str]
    species: List[Species]
    reactions: List[Reaction]
    name: str = "synthetic"

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_reactions(self) -> int:
        return len(self.reactions)

    # ---------------------------------------------------------------- writer
    def to_text(self) -> str:
        out = []
        w = out.append
        w("pyjac-mech 1")
        w(f"# {self.name}: {self.n_species} species, {self.n_reactions} reactions")
        w(f"elements {len(self.elements)}")
        for e in self.elements:
            w(f"  {e} {ATOMIC_WEIGHTS[e]!r}")
        w(f"species {self.n_species}")
        for sp in self.species:
            comp = [(e, c) for e, c in sp.comp.items() if c]
            ctext = " ".join(f"{e} {c}" for e, c in comp)
            w(f"  {sp.name} {sp.W!r} {sp.tmid!r} {len(comp)} {ctext}")
            w("    " + " ".join(repr(float(a)) for a in sp.low))
            w("    " + " ".join(repr(float(a)) for a in sp.high))
        w(f"reactions {self.n_reactions}")
        names = [s.name for s in self.species]
        kind_token = {
            "elementary": "elementary", "thirdbody": "thirdbody",
            "falloff_lindemann": "falloff", "falloff_troe": "falloff",
            "falloff_sri": "falloff", "chemact_lindemann": "chemact",
            "chemact_troe": "chemact", "chemact_sri": "chemact",
            "plog": "plog", "cheb": "cheb",
        }
        for r in self.reactions:
            toks = [f"reaction {kind_token[r.kind]} {r.rev}"]
            toks.append(f"reactants {len(r.reac)} " +
                        " ".join(f"{names[k]} {n}" for k, n in r.reac))
            toks.append(f"products {len(r.prod)} " +
                        " ".join(f"{names[k]} {n}" for k, n in r.prod))
            if r.arr is not None:
                toks.append("arrhenius " + " ".join(repr(float(v)) for v in r.arr))
            if r.low is not None:
                toks.append("low " + " ".join(repr(float(v)) for v in r.low))
                toks.append("high " + " ".join(repr(float(v)) for v in r.high))
                if r.troe is not None:
                    toks.append(f"troe {len(r.troe)} " +
                                " ".join(repr(float(v)) for v in r.troe))
                elif r.sri is not None:
                    toks.append(f"sri {len(r.sri)} " +
                                " ".join(repr(float(v)) for v in r.sri))
                else:
                    toks.append("lindemann")
            if r.collider == "mix":
                toks.append(f"collider mix {len(r.eff)} " +
                            " ".join(f"{names[k]} {float(a)!r}"
                                     for k, a in sorted(r.eff.items())))
            elif r.collider == "species":
                toks.append(f"collider species {names[r.collider_species]}")
            if r.plog is not None:
                toks.append(f"plog {len(r.plog)} " + " ".join(
                    " ".join(repr(float(v)) for v in pt) for pt in r.plog))
            if r.cheb is not None:
                c = r.cheb
                coef = np.asarray(c["coef"], dtype=float)
                toks.append(f"cheb {c['nT']} {c['nP']} {c['Tmin']!r} {c['Tmax']!r} "
                            f"{c['Pmin']!r} {c['Pmax']!r} " +
                            " ".join(repr(float(v)) for v in coef.ravel()))
            if r.reverse is not None:
                toks.append("reverse " + " ".join(repr(float(v)) for v in r.reverse))
            w("  " + "\n    ".join(toks))
        w("end")
        return "\n".join(out) + "\n"

    def write(self, path: str) -> str:
        with open(path, "w") as fh:
            fh.write(self.to_text())
        return path

    # ------------------------------------------------------- array helpers
    def stoich(self) -> Tuple[np.ndarray, np.ndarray]:
        """Integer reactant/product coefficient matrices, shape (N, N_R)."""
        nu_f = np.zeros((self.n_species, self.n_reactions), dtype=np.int64)
        nu_r = np.zeros_like(nu_f)
        for i, r in enumerate(self.reactions):
            for k, n in r.reac:
                nu_f[k, i] += n
            for k, n in r.prod:
                nu_r[k, i] += n
        return nu_f, nu_r

    def element_matrix(self) -> np.ndarray:
        """a[e, k]: atoms of element e in species k."""
        a = np.zeros((len(self.elements), self.n_species), dtype=np.int64)
        for k, sp in enumerate(self.species):
            for e, c in sp.comp.items():
                a[self.elements.index(e), k] = c
        return a

    def molecular_weights(self) -> np.ndarray:
        return np.array([s.W for s in self.species])


# ------------------------------------------------------------------- thermo
def _fit_nasa(rng: np.random.Generator, n_atoms: int, tmid: float = 1000.0):
    """Least-squares NASA-7 fit of a smooth random cp(T)/R.

    cp/R = c_inf - (c_inf - c_0) exp(-T/theta); the two ranges share cp at tmid,
    and the integration constants make H and S continuous there.
    """
    if n_atoms == 1:
        c0 = 2.5
        cinf = 2.5 + rng.uniform(0.0, 0.15)
    else:
        c0 = rng.uniform(2.5, 3.5 + n_atoms)
        hi = max(1.5 * (3 * n_atoms - 1.5), c0 + 1.0)
        cinf = rng.uniform(c0 + 0.5, hi)
    theta = rng.uniform(400.0, 1500.0)
    cp = lambda T: cinf - (cinf - c0) * np.exp(-T / theta)   # noqa: E731

    P = np.polynomial.Polynomial
    u_lo = np.linspace(0.3, tmid / 1000.0, 60)
    p_lo = P.fit(u_lo, cp(u_lo * 1000.0), 4).convert()
    u_m = tmid / 1000.0
    u_hi = np.linspace(u_m, 5.0, 80)
    c_m = p_lo(u_m)
    # cp_hi(u) = c_m + (u - u_m) q(u), q cubic -> continuity of cp at tmid
    A = np.stack([(u_hi - u_m) * u_hi ** n for n in range(4)], axis=1)
    q, *_ = np.linalg.lstsq(A, cp(u_hi * 1000.0) - c_m, rcond=None)
    p_hi = P([c_m]) + P([-u_m, 1.0]) * P(q)

    def coeffs(poly):
        c = np.zeros(5)
        cc = poly.coef
        c[: len(cc)] = cc
        return [c[n] / 1000.0 ** n for n in range(5)]

    lo = coeffs(p_lo)
    hi = coeffs(p_hi)
    # Enthalpy/R and entropy/R as integrals of the fitted cp/R polynomial.
    def h_int(a, T):
        return sum(a[n] * T ** (n + 1) / (n + 1) for n in range(5))

    def s_int(a, T):
        return a[0] * np.log(T) + sum(a[n] * T ** n / n for n in range(1, 5))

    Tref = 298.15
    hf = rng.uniform(-3.0e4, 3.0e4)
    s298 = rng.uniform(20.0, 40.0)
    a5_lo = hf - h_int(lo, Tref)
    a6_lo = s298 - s_int(lo, Tref)
    a5_hi = (h_int(lo, tmid) + a5_lo) - h_int(hi, tmid)
    a6_hi = (s_int(lo, tmid) + a6_lo) - s_int(hi, tmid)
    return lo + [a5_lo, a6_lo], hi + [a5_hi, a6_hi]


# ----------------------------------------------------------------- species
def _species_name(comp: Dict[str, int], taken: set) -> str:
    base = "".join(f"{e}{c if c > 1 else ''}" for e, c in comp.items() if c) or "X"
    name = base
    n = 1
    while name in taken:
        n += 1
        name = f"{base}-{n}"
    taken.add(name)
    return name


def _make_species(rng, elements, bounds, n_species, inert_last="N2",
                  reactive_last=False):
    reactive_elems = [e for e in elements if e != "Ar"]
    comps: List[Dict[str, int]] = []
    seen = set()

    def add(comp):
        key = tuple(comp.get(e, 0) for e in elements)
        if key in seen or sum(key) == 0:
            return False
        seen.add(key)
        comps.append({e: comp.get(e, 0) for e in elements})
        return True

    n_reactive = n_species
    if not reactive_last:
        n_reactive -= 1                              # inert last species
        if "Ar" in elements and "N" in elements:
            n_reactive -= 1                          # an extra inert Ar
    # atoms first, then a few diatomics, then random compositions in the box
    for e in reactive_elems:
        if bounds.get(e, 0) >= 1 and len(comps) < n_reactive:
            add({e: 1})
    for e in reactive_elems:
        if bounds.get(e, 0) >= 2 and e != "N" and len(comps) < n_reactive:
            add({e: 2})
    guard = 0
    while len(comps) < n_reactive:
        guard += 1
        if guard > 100000:
            raise RuntimeError("composition box too small for requested species count")
        comp = {e: int(rng.integers(0, bounds.get(e, 0) + 1)) for e in reactive_elems}
        add(comp)
    taken: set = set()
    species = []
    for comp in comps:
        n_atoms = sum(comp.values())
        lo, hi = _fit_nasa(rng, n_atoms)
        W = sum(ATOMIC_WEIGHTS[e] * c for e, c in comp.items())
        species.append(Species(_species_name(comp, taken), comp, W, 1000.0, lo, hi))
    if not reactive_last:
        if "Ar" in elements:
            comp = {e: (1 if e == "Ar" else 0) for e in elements}
            lo, hi = _fit_nasa(rng, 1)
            species.append(Species(_species_name(comp, taken), comp,
                                   ATOMIC_WEIGHTS["Ar"], 1000.0, lo, hi, inert=True))
        if "N" not in elements:       # Ar (appended above) is the inert last species
            return species
        comp = {e: 0 for e in elements}
        comp["N"] = 2
        lo, hi = _fit_nasa(rng, 2)
        name = "N2" if "N2" not in taken else _species_name(comp, taken)
        taken.add(name)
        species.append(Species(name, comp, 2 * ATOMIC_WEIGHTS["N"], 1000.0, lo, hi,
                               inert=True))
    return species


# ---------------------------------------------------------------- reactions
def _arrhenius(rng, order: int) -> Tuple[float, float, float]:
    A_cgs = 10.0 ** rng.uniform(5.0, 15.0)
    A = A_cgs * CGS_TO_SI_PER_ORDER ** (order - 1)
    beta = rng.uniform(-2.0, 3.0)
    Ta = rng.uniform(0.0, 50.0) * KCAL_PER_MOL_TO_K
    return (float(A), float(beta), float(Ta))


class _Balancer:
    def __init__(self, species: Sequence[Species], elements: Sequence[str]):
        self.reactive = [k for k, s in enumerate(species) if not s.inert]
        self.comp = np.array([[s.comp.get(e, 0) for e in elements] for s in species],
                             dtype=np.int64)
        self.by_comp: Dict[tuple, List[int]] = {}
        for k in self.reactive:
            self.by_comp.setdefault(tuple(self.comp[k]), []).append(k)

    def sides(self, total: np.ndarray, max_molecules: int = 3):
        """All multisets of reactive species (nu in {1,2}, <= 2 distinct species,
        <= max_molecules molecules) whose compositions sum to `total`."""
        out = []
        for k in self.by_comp.get(tuple(total), []):
            out.append(((k, 1),))
        if max_molecules < 2:
            return out
        if np.all(total % 2 == 0):
            for k in self.by_comp.get(tuple(total // 2), []):
                out.append(((k, 2),))
        R = np.asarray(self.reactive)
        rest = total[None, :] - self.comp[R]
        ok = np.all(rest >= 0, axis=1) & np.any(rest > 0, axis=1)
        for b, rr in zip(R[ok], rest[ok]):
            for c in self.by_comp.get(tuple(rr), []):
                if c > b:
                    out.append(((int(b), 1), (c, 1)))
        if max_molecules >= 3:
            rest2 = total[None, :] - 2 * self.comp[R]
            ok2 = np.all(rest2 >= 0, axis=1) & np.any(rest2 > 0, axis=1)
            for b, rr in zip(R[ok2], rest2[ok2]):
                for c in self.by_comp.get(tuple(rr), []):
                    if c != b:
                        out.append(((int(b), 2), (c, 1)))
        return out


def _canon(side):
    return tuple(sorted(side))


def _draw_reaction_sides(rng, bal: _Balancer, kind: str, used: set,
                         must_include: Optional[int] = None, allow_shared=False,
                         tries: int = 400):
    """Draw an element-balanced, non-duplicate (reactants, products) pair."""
    assoc = kind in ("thirdbody",) or kind.startswith("falloff")
    bimol = kind.startswith("chemact")
    R = bal.reactive
    for _ in range(tries):
        if must_include is not None and rng.random() < 0.8:
            a = must_include
        else:
            a = int(rng.choice(R))
        shape = rng.random()
        if assoc or bimol:
            # two reactant molecules
            if shape < 0.25:
                reac = ((a, 2),)
            else:
                b = int(rng.choice(R))
                if b == a:
                    reac = ((a, 2),)
                else:
                    reac = tuple(sorted(((a, 1), (b, 1))))
        else:
            if shape < 0.12:
                reac = ((a, 1),)
            elif shape < 0.22:
                reac = ((a, 2),)
            else:
                b = int(rng.choice(R))
                reac = ((a, 2),) if b == a else tuple(sorted(((a, 1), (b, 1))))
        total = sum(n * bal.comp[k] for k, n in reac)
        maxm = 1 if assoc else 3
        opts = bal.sides(total, max_molecules=maxm)
        if assoc:
            opts = [o for o in opts if len(o) == 1 and o[0][1] == 1]
        rs = {k for k, _ in reac}
        if not allow_shared:
            opts = [o for o in opts if not ({k for k, _ in o} & rs)]
        else:
            opts = [o for o in opts if _canon(o) != _canon(reac)]
        opts = [o for o in opts if (_canon(reac), _canon(o)) not in used
                and (_canon(o), _canon(reac)) not in used]
        if not opts:
            continue
        prod = opts[int(rng.integers(len(opts)))]
        if assoc and rng.random() < 0.5:
            reac, prod = tuple(prod), tuple(reac)      # dissociation direction
        used.add((_canon(reac), _canon(prod)))
        return [tuple(x) for x in reac], [tuple(x) for x in prod]
    return None


def _fill_reaction(rng, kind: str, rev: str, reac, prod, n_species: int,
                   eff_pool: Sequence[int], plog_points=(4, 6), cheb_shape=(7, 3),
                   collider_probs=(0.15, 0.10)) -> Reaction:
    order = sum(n for _, n in reac)
    r = Reaction(kind=kind, rev=rev, reac=list(reac), prod=list(prod))
    if kind == "elementary":
        r.arr = _arrhenius(rng, order)
    elif kind == "thirdbody":
        r.arr = _arrhenius(rng, order + 1)
    elif kind.startswith("falloff"):
        r.low = _arrhenius(rng, order + 1)
        r.high = _arrhenius(rng, order)
    elif kind.startswith("chemact"):
        r.low = _arrhenius(rng, order)
        r.high = _arrhenius(rng, order - 1)
    if kind.endswith("_troe"):
        a = rng.uniform(0.1, 0.9)
        T3 = 10.0 ** rng.uniform(np.log10(30.0), np.log10(3000.0))
        T1 = 10.0 ** rng.uniform(np.log10(300.0), 4.0)
        if rng.random() < 0.5:
            T2 = 10.0 ** rng.uniform(3.0, 4.0)
            r.troe = (a, T3, T1, T2)
        else:
            r.troe = (a, T3, T1)
    elif kind.endswith("_sri"):
        r.sri = (rng.uniform(0.1, 2.0), rng.uniform(100.0, 2000.0),
                 rng.uniform(200.0, 3000.0), rng.uniform(0.5, 2.0),
                 rng.uniform(-0.5, 0.5))
    if kind == "thirdbody" or kind.startswith("falloff") or kind.startswith("chemact"):
        u = rng.random()
        p_unity, p_species = collider_probs
        if u < p_unity:
            r.collider = "mix"
            r.eff = {}
        elif u < p_unity + p_species:
            r.collider = "species"
            r.collider_species = int(rng.choice(eff_pool))
        else:
            r.collider = "mix"
            n_eff = int(rng.integers(3, 9))
            n_eff = min(n_eff, len(eff_pool))
            ks = rng.choice(eff_pool, size=n_eff, replace=False)
            r.eff = {int(k): float(rng.uniform(0.5, 12.0)) for k in ks}
    if kind == "plog":
        npt = int(rng.integers(plog_points[0], plog_points[1] + 1))
        ps = np.logspace(np.log10(0.01), np.log10(100.0), npt) * ATM
        r.plog = [(float(p),) + _arrhenius(rng, order) for p in ps]
    if kind == "cheb":
        nT, nP = cheb_shape
        coef = np.zeros((nT, nP))
        for i in range(nT):
            for j in range(nP):
                coef[i, j] = rng.normal() * 0.3 ** (i + j)
        coef[0, 0] = rng.uniform(8.0, 14.0) + 3.0 * (1 - order)   # log10, cgs -> SI
        r.cheb = dict(nT=nT, nP=nP, Tmin=300.0, Tmax=2500.0,
                      Pmin=0.01 * ATM, Pmax=100.0 * ATM, coef=coef)
    if rev == "explicit":
        r.reverse = _arrhenius(rng, sum(n for _, n in prod) + (1 if kind == "thirdbody" else 0))
    return r


def make_mechanism(seed: int, n_species: int, n_reactions: int,
                   elements: Sequence[str], bounds: Dict[str, int],
                   mix: Dict[str, int], rev_mix: Optional[Dict[str, float]] = None,
                   reactive_last: bool = False, allow_shared: bool = False,
                   plog_points=(4, 6), cheb_shape=(7, 3), name="synthetic",
                   collider_probs=(0.15, 0.10)) -> Mechanism:
    """Build a random element-balanced mechanism with the given reaction mix."""
    assert sum(mix.values()) == n_reactions, (mix, n_reactions)
    rng = np.random.default_rng(seed)
    elements = list(elements)
    if not reactive_last and "N" not in elements and "Ar" not in elements:
        elements.append("Ar")
    species = _make_species(rng, list(elements), bounds, n_species,
                            reactive_last=reactive_last)
    bal = _Balancer(species, list(elements))
    kinds: List[str] = []
    for k in REACTION_TYPES:
        kinds += [k] * int(mix.get(k, 0))
    rng.shuffle(kinds)
    rev_mix = rev_mix or {"kc": 1.0}
    rev_keys = list(rev_mix)
    rev_p = np.array([rev_mix[k] for k in rev_keys], dtype=float)
    rev_p /= rev_p.sum()
    used: set = set()
    uncovered = list(bal.reactive)
    rng.shuffle(uncovered)
    eff_pool = list(range(len(species)))
    reactions = []
    for kind in kinds:
        target = uncovered[0] if uncovered else None
        sides = _draw_reaction_sides(rng, bal, kind, used, must_include=target,
                                     allow_shared=allow_shared)
        if sides is None:
            sides = _draw_reaction_sides(rng, bal, kind, used, allow_shared=allow_shared,
                                         tries=4000)
        if sides is None:
            raise RuntimeError(f"could not draw a balanced {kind} reaction")
        reac, prod = sides
        for k, _ in reac + prod:
            if k in uncovered:
                uncovered.remove(k)
        rev = rev_keys[int(rng.choice(len(rev_keys), p=rev_p))]
        reactions.append(_fill_reaction(rng, kind, rev, reac, prod, len(species),
                                        eff_pool, plog_points, cheb_shape,
                                        collider_probs))
    # reactions that could not cover a species: swap in covering reactions
    for k in list(uncovered):
        for idx, r in enumerate(reactions):
            if r.kind != "elementary":
                continue
            sides = _draw_reaction_sides(rng, bal, "elementary", used, must_include=k,
                                         allow_shared=allow_shared, tries=4000)
            if sides is not None and k in {s for s, _ in sides[0] + sides[1]}:
                reactions[idx] = _fill_reaction(rng, "elementary", r.rev, sides[0],
                                                sides[1], len(species), eff_pool)
                uncovered.remove(k)
                break
    return Mechanism(list(elements), species, reactions, name=name)


# ------------------------------------------------------------ paper shapes
def _c1_mix(n_total: int) -> Dict[str, int]:
    """Methane-shaped proportions: 70% elementary, 10% third body,
    15% Lindemann/Troe falloff (1/3, 2/3), 5% chemically activated / SRI."""
    n_el = round(0.70 * n_total)
    n_tb = round(0.10 * n_total)
    n_fo = round(0.15 * n_total)
    n_sp = n_total - n_el - n_tb - n_fo
    n_lind = round(n_fo / 3)
    n_sri = n_sp // 2
    n_ca = n_sp - n_sri
    ca_l = n_ca // 3
    ca_t = (n_ca - ca_l) // 2
    ca_s = n_ca - ca_l - ca_t
    return {"elementary": n_el, "thirdbody": n_tb, "falloff_lindemann": n_lind,
            "falloff_troe": n_fo - n_lind, "falloff_sri": n_sri,
            "chemact_lindemann": ca_l, "chemact_troe": ca_t, "chemact_sri": ca_s}


WORKLOADS = {
    0: dict(name="h2_shaped_13sp_27rxn", n_species=13, n_reactions=27,
            elements=["H", "O", "N", "Ar"], bounds={"H": 2, "O": 2, "N": 1},
            mix={"elementary": 20, "thirdbody": 5, "falloff_troe": 2},
            n_states=1000, T=(1000.0, 2000.0), P_atm=(1.0, 20.0), dirichlet=0.5),
    1: dict(name="ch4_shaped_53sp_325rxn", n_species=53, n_reactions=325,
            elements=["C", "H", "O", "N", "Ar"], bounds={"C": 2, "H": 4, "O": 3, "N": 1},
            mix={"elementary": 228, "thirdbody": 32, "falloff_lindemann": 16,
                 "falloff_troe": 33, "falloff_sri": 8, "chemact_lindemann": 3,
                 "chemact_troe": 3, "chemact_sri": 2},
            n_states=100_000, T=(800.0, 2200.0), P_atm=(1.0, 50.0), dirichlet=0.3),
    2: dict(name="c2h4_shaped_111sp_784rxn", n_species=111, n_reactions=784,
            elements=["C", "H", "O", "N", "Ar"], bounds={"C": 2, "H": 6, "O": 3, "N": 1},
            mix=dict(_c1_mix(744), plog=30, cheb=10),
            n_states=100_000, T=(800.0, 2200.0), P_atm=(1.0, 50.0), dirichlet=0.3),
    3: dict(name="ic5h11oh_shaped_360sp_2172rxn", n_species=360, n_reactions=2172,
            elements=["C", "H", "O", "N", "Ar"], bounds={"C": 5, "H": 12, "O": 3, "N": 1},
            mix=dict(_c1_mix(2129), plog=43),
            n_states=20_000, T=(800.0, 2200.0), P_atm=(1.0, 50.0), dirichlet=0.3),
}

MECH_SEED_BASE = 1605
STATE_SEED_BASE = 3262


def config_mechanism(cfg_id: int) -> Mechanism:
    c = WORKLOADS[cfg_id]
    return make_mechanism(MECH_SEED_BASE + cfg_id, c["n_species"], c["n_reactions"],
                          c["elements"], c["bounds"], c["mix"], name=c["name"])


def tiny_mechanism(seed: int, kinds: Dict[str, int], n_species: int = 6,
                   reactive_last: bool = False, rev_mix=None,
                   elements=("H", "O", "N", "Ar"), bounds=None,
                   allow_shared: bool = False, collider_probs=(0.25, 0.25),
                   plog_points=(1, 4), cheb_shape=(3, 2)) -> Mechanism:
    """Small mechanism for oracle pins: every reaction class can be requested."""
    bounds = bounds or {"H": 2, "O": 2, "N": 1}
    n_r = sum(kinds.values())
    last_err = None
    for attempt in range(50):      # deterministic reseeding if a class cannot be drawn
        try:
            return make_mechanism(seed + 7919 * attempt, n_species, n_r, list(elements),
                                  bounds, kinds, rev_mix=rev_mix,
                                  reactive_last=reactive_last, allow_shared=allow_shared,
                                  plog_points=plog_points, cheb_shape=cheb_shape,
                                  name=f"tiny_{seed}", collider_probs=collider_probs)
        except RuntimeError as err:
            last_err = err
    raise last_err
