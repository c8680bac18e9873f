"""Seeded synthetic reaction mechanisms (input generator only).

The paper integrates a detailed methane/ammonia mechanism (59 species, 356
reactions; Sec. 2.5) and names the GRI-3.0 size (53 species) in its
mechanism comparison (Table 2).  Neither file is available, so every
workload here is a *synthetic* mechanism of the same size and structure:

* species built from the elements {H,O,N} or {C,H,O,N}, molar masses from
  IUPAC conventional atomic weights;
* elementally balanced reversible reactions with 2-3 species per side
  (integer stoichiometric coefficients 1 or 2), a given number of them
  third-body and Troe fall-off;
* modified-Arrhenius parameters: log10 A uniform in [8,16] (cgs), b uniform
  in [-2,2], Ea uniform in [0,250] kJ/mol;
* single-range (200-6000 K) smooth NASA-7 thermochemistry with a monotone
  heat capacity, from which reverse rates follow through equilibrium
  constants.

Large mechanisms get the structure real ones have: a small radical pool
(about 15% of the species) that may appear anywhere, and a "skeleton" of
larger species of which each reaction carries at most one per side.

This module evaluates no rate law, no reactor equation and no integrator: it
only writes the mechanism text that both the oracle and the device library
parse on their own.  The text format is described in ``to_text``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# IUPAC conventional atomic weights, g/mol
ATOMIC_WEIGHT = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999}
R_GAS = 8.314462618  # J/(mol K)
P_REF = 101325.0  # Pa, standard-state pressure of the equilibrium constants
T_LO, T_HI = 200.0, 6000.0
T_298 = 298.15


@dataclass
class Species:
    name: str
    comp: dict
    role: str  # ref | product | radical | fuel | skeleton
    W: float = 0.0  # kg/mol
    nasa: tuple = ()  # a1..a7
    h298: float = 0.0  # J/mol
    s298: float = 0.0  # J/(mol K)


@dataclass
class Reaction:
    kind: str  # plain | third | troe
    reac: list  # [(species index, nu)]
    prod: list
    log10A: float
    b: float
    Ea: float  # J/mol
    eff: dict = field(default_factory=dict)  # species index -> efficiency
    troe: tuple = ()  # (log10A0, b0, Ea0, a, T3, T1, T2)


@dataclass
class Mechanism:
    elements: list
    species: list
    reactions: list
    name: str = "synthetic"

    @property
    def n_species(self):
        return len(self.species)

    @property
    def n_reactions(self):
        return len(self.reactions)

    def index(self, name):
        for i, s in enumerate(self.species):
            if s.name == name:
                return i
        raise KeyError(name)

    def element_matrix(self):
        """a[e, k] = atoms of element e in species k."""
        a = np.zeros((len(self.elements), self.n_species))
        for k, s in enumerate(self.species):
            for e, el in enumerate(self.elements):
                a[e, k] = s.comp.get(el, 0)
        return a

    def molar_masses(self):
        return np.array([s.W for s in self.species])

    def stoich(self):
        """nu[k, j] = net stoichiometric coefficient (products minus reactants)."""
        nu = np.zeros((self.n_species, self.n_reactions))
        for j, r in enumerate(self.reactions):
            for k, v in r.reac:
                nu[k, j] -= v
            for k, v in r.prod:
                nu[k, j] += v
        return nu

    def nasa_array(self):
        return np.array([s.nasa for s in self.species], dtype=np.float64)

    def to_text(self) -> str:
        """Serialise to the line-based ``.mech`` text format.

        Layout (whitespace separated, ``#`` starts a comment)::

            STIFFCHEM-MECH 1
            NAME <name>
            GAS_CONSTANT <R J/mol/K>
            REF_PRESSURE <p0 Pa>
            ELEMENTS <E> <sym> ...
            SPECIES <N>
            SP <name> <W kg/mol> <count per element, ELEMENTS order>
            NASA7 <name> <a1> ... <a7>        (one per species, same order)
            REACTIONS <R>
            RX <kind> <log10A cgs> <b> <Ea J/mol> <nr> (<name> <nu>)*nr <np> (<name> <nu>)*np
            EFF <n> (<name> <alpha>)*n        (optional, after a third/troe RX)
            TROE <log10A0> <b0> <Ea0> <a> <T3> <T1> <T2>   (after each troe RX)
            END

        ``kind`` is ``plain``, ``third`` or ``troe``.  Floats are written with
        17 significant digits so every reader recovers the same doubles.
        """
        f = lambda x: repr(float(x))
        out = ["STIFFCHEM-MECH 1", f"NAME {self.name}", f"GAS_CONSTANT {f(R_GAS)}",
               f"REF_PRESSURE {f(P_REF)}",
               f"ELEMENTS {len(self.elements)} " + " ".join(self.elements),
               f"SPECIES {self.n_species}"]
        for s in self.species:
            counts = " ".join(str(int(s.comp.get(e, 0))) for e in self.elements)
            out.append(f"SP {s.name} {f(s.W)} {counts}")
        for s in self.species:
            out.append(f"NASA7 {s.name} " + " ".join(f(a) for a in s.nasa))
        out.append(f"REACTIONS {self.n_reactions}")
        for r in self.reactions:
            side = lambda lst: f"{len(lst)} " + " ".join(
                f"{self.species[k].name} {v}" for k, v in lst)
            out.append(f"RX {r.kind} {f(r.log10A)} {f(r.b)} {f(r.Ea)} {side(r.reac)} {side(r.prod)}")
            if r.eff:
                out.append(f"EFF {len(r.eff)} " + " ".join(
                    f"{self.species[k].name} {f(a)}" for k, a in sorted(r.eff.items())))
            if r.kind == "troe":
                out.append("TROE " + " ".join(f(x) for x in r.troe))
        out.append("END")
        return "\n".join(out) + "\n"


# ----------------------------------------------------------------------------
# species
# ----------------------------------------------------------------------------

def _formula(comp, elements):
    s = ""
    for e in elements:
        c = comp.get(e, 0)
        if c:
            s += e + (str(c) if c > 1 else "")
    return s


_CORE = {
    # (composition, role); order = preference for the radical pool
    "H": ({"H": 1}, "radical"), "O": ({"O": 1}, "radical"), "OH": ({"O": 1, "H": 1}, "radical"),
    "HO2": ({"H": 1, "O": 2}, "radical"), "H2": ({"H": 2}, "ref"), "O2": ({"O": 2}, "ref"),
    "H2O": ({"H": 2, "O": 1}, "product"), "NO": ({"N": 1, "O": 1}, "product"),
    "N": ({"N": 1}, "radical"), "NH": ({"N": 1, "H": 1}, "radical"),
    "NH2": ({"N": 1, "H": 2}, "radical"), "CH3": ({"C": 1, "H": 3}, "radical"),
    "HCO": ({"C": 1, "H": 1, "O": 1}, "radical"), "CO": ({"C": 1, "O": 1}, "product"),
    "N2O": ({"N": 2, "O": 1}, "product"), "NO2": ({"N": 1, "O": 2}, "product"),
    "N2": ({"N": 2}, "ref"), "CH4": ({"C": 1, "H": 4}, "fuel"), "CO2": ({"C": 1, "O": 2}, "product"),
    "NH3": ({"N": 1, "H": 3}, "fuel"), "H2O2": ({"H": 2, "O": 2}, "product"),
}
_POOL_ORDER = ["H", "O", "OH", "HO2", "H2", "O2", "H2O", "NO", "N", "NH", "NH2", "CH3",
               "HCO", "CO", "N2O", "NO2"]
# species every mechanism of the element set carries (roles used by the cell generator)
_REQUIRED = {"HON": ["H", "O", "OH", "H2", "O2", "H2O", "NO", "N2"],
             "CHON": ["H", "O", "OH", "HO2", "H2", "O2", "H2O", "NO", "N2", "CH4", "CO",
                      "CO2", "NH3"]}


def _random_comp(rng, elements):
    while True:
        if "C" in elements:
            comp = {"C": int(rng.integers(0, 4)), "H": int(rng.integers(0, 9)),
                    "O": int(rng.integers(0, 4)), "N": int(rng.integers(0, 3))}
        else:
            comp = {"H": int(rng.integers(0, 5)), "O": int(rng.integers(0, 4)),
                    "N": int(rng.integers(0, 3))}
        comp = {e: c for e, c in comp.items() if c}
        nat = sum(comp.values())
        if 2 <= nat <= 9:
            return comp


def _nasa7(rng, comp, h298, s298):
    """Single-range NASA-7 with a monotone-increasing cp/R on [200, 6000] K.

    cp/R = lo + (hi-lo) P(tau), tau = (T-200)/5800, P a convex mix of
    tau, 1-(1-tau)^2 and 1-(1-tau)^4 (each monotone from 0 to 1), expanded
    to the power basis a1..a5.  a6, a7 pin h(298.15) and s(298.15).
    """
    nat = sum(comp.values())
    if nat == 1:
        lo, hi = 2.5, 2.5 + rng.uniform(0.0, 0.3)
    elif nat == 2:
        lo, hi = 3.5 + rng.uniform(-0.1, 0.1), 4.5 + rng.uniform(-0.2, 0.2)
    else:
        lo, hi = 4.0 + rng.uniform(-0.2, 0.4), 3 * nat - 2 + rng.uniform(-0.5, 0.0)
    w = rng.dirichlet(np.ones(3))
    P = np.polynomial.Polynomial
    tau = P([-T_LO / (T_HI - T_LO), 1.0 / (T_HI - T_LO)])
    one = P([1.0])
    poly = w[0] * tau + w[1] * (one - (one - tau) ** 2) + w[2] * (one - (one - tau) ** 4)
    cp = lo * one + (hi - lo) * poly
    a = np.zeros(7)
    c = cp.coef
    a[: len(c)] = c
    T = T_298
    h_rt_noa6 = a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5
    a[5] = h298 / R_GAS - T * h_rt_noa6
    s_noa7 = a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4
    a[6] = s298 / R_GAS - s_noa7
    return tuple(float(x) for x in a)


def _h298(rng, role):
    if role == "ref":
        return 0.0
    if role == "product":
        return rng.uniform(-300e3, -50e3)
    if role == "radical":
        return rng.uniform(30e3, 250e3)
    if role == "fuel":
        return rng.uniform(-80e3, 20e3)
    return rng.uniform(-200e3, 200e3)


def _make_species(rng, elements, n_species, n_pool):
    key = "CHON" if "C" in elements else "HON"
    allowed = lambda comp: set(comp) <= set(elements)
    names, comps, roles = [], [], []

    def add(name, comp, role):
        names.append(name)
        comps.append(comp)
        roles.append(role)

    required = _REQUIRED[key]
    if n_pool >= n_species:  # small mechanism: every species is a pool species
        pool_names = list(required)
    else:
        pool_names = [n for n in _POOL_ORDER if allowed(_CORE[n][0])][:n_pool]
    for n in pool_names:
        add(n, *_CORE[n])
    for n in required:
        if n not in names:
            add(n, *_CORE[n])
    seen = {_formula(c, elements) for c in comps}
    extras = [n for n in _CORE if n not in names and allowed(_CORE[n][0])]
    rng.shuffle(extras)
    while len(names) < n_species:
        if extras and rng.uniform() < 0.5:
            n = extras.pop()
            comp, role = _CORE[n]
        else:
            comp, role = _random_comp(rng, elements), "skeleton"
            n = _formula(comp, elements)
        f = _formula(comp, elements)
        if f in seen:
            continue
        seen.add(f)
        add(n, comp, role)
    n_pool_eff = n_species if n_pool >= n_species else len(pool_names)
    out = []
    for n, c, r in zip(names, comps, roles):
        nat = sum(c.values())
        h = _h298(rng, r)
        s = R_GAS * (13.0 + 3.0 * nat + rng.uniform(-2.0, 2.0))
        sp = Species(name=n, comp=dict(c), role=r, h298=h, s298=s)
        sp.W = sum(ATOMIC_WEIGHT[e] * v for e, v in c.items()) / 1000.0
        sp.nasa = _nasa7(rng, c, h, s)
        out.append(sp)
    return out, n_pool_eff


# ----------------------------------------------------------------------------
# reactions
# ----------------------------------------------------------------------------

def _sides(species, elements, n_pool, pool_only):
    """All 2- and 3-multisets with at most one non-pool species (all species
    count as pool when ``pool_only``).  Returns {element vector: [multiset]}."""
    N = len(species)
    vec = [tuple(s.comp.get(e, 0) for e in elements) for s in species]
    pool = list(range(N)) if pool_only else list(range(n_pool))
    skel = [] if pool_only else list(range(n_pool, N))
    msets = []
    for size in (2, 3):
        msets += list(itertools.combinations_with_replacement(pool, size))
        for x in skel:
            for rest in itertools.combinations_with_replacement(pool, size - 1):
                msets.append(tuple(sorted((x,) + rest)))
    buckets = {}
    for m in msets:
        v = tuple(sum(vec[k][e] for k in m) for e in range(len(elements)))
        buckets.setdefault(v, []).append(m)
    return buckets


def _counts(m):
    d = {}
    for k in m:
        d[k] = d.get(k, 0) + 1
    return sorted(d.items())


def _make_reactions(rng, species, elements, n_pool, n_reactions, pool_only, dh_max=400e3):
    buckets = _sides(species, elements, n_pool, pool_only)
    h = np.array([s.h298 for s in species])
    cands = []
    for ms in buckets.values():
        for a, b in itertools.combinations(ms, 2):
            if set(a) & set(b):
                continue
            dh = sum(h[k] for k in b) - sum(h[k] for k in a)
            if abs(dh) > dh_max:
                continue
            cands.append((a, b))
    if len(cands) < n_reactions:
        return None  # too few balanced reactions for this species set: caller retries
    order = rng.permutation(len(cands))
    chosen, used = [], set()
    covered = np.zeros(len(species), bool)
    # first make sure every species takes part in some reaction
    by_species = {}
    for ci, (a, b) in enumerate(cands):
        for k in set(a) | set(b):
            by_species.setdefault(k, []).append(ci)
    for k in rng.permutation(len(species)):
        if covered[k]:
            continue
        lst = by_species.get(int(k))
        if not lst:
            return None  # species cannot be balanced: caller retries
        ci = lst[int(rng.integers(len(lst)))]
        if ci in used:
            continue
        used.add(ci)
        chosen.append(ci)
        for s in set(cands[ci][0]) | set(cands[ci][1]):
            covered[s] = True
    for ci in order:
        if len(chosen) >= n_reactions:
            break
        if int(ci) in used:
            continue
        used.add(int(ci))
        chosen.append(int(ci))
    if len(chosen) > n_reactions or not covered.all():
        return None
    out = []
    for ci in chosen:
        a, b = cands[ci]
        # write every reaction in its exothermic direction: the sampled
        # Arrhenius parameters belong to that direction, so the reverse rate
        # kf/Kc carries the activation energy Ea + |dH| >= 0
        if sum(h[k] for k in b) - sum(h[k] for k in a) > 0.0:
            a, b = b, a
        out.append((_counts(a), _counts(b)))
    return out


def _arrhenius(rng):
    return rng.uniform(8.0, 16.0), rng.uniform(-2.0, 2.0), rng.uniform(0.0, 250e3)


def make_mechanism(n_species, n_reactions, n_third, n_troe, elements, seed,
                   pool_frac=0.15, name=None) -> Mechanism:
    """Seeded synthetic mechanism of the given size (see module docstring)."""
    rng = np.random.default_rng(seed)
    pool_only = n_species < 20
    n_pool = n_species if pool_only else max(4, int(round(pool_frac * n_species)))
    for _attempt in range(50):
        species, n_pool_eff = _make_species(rng, elements, n_species, n_pool)
        rx = _make_reactions(rng, species, elements, n_pool_eff, n_reactions, pool_only)
        if rx is not None:
            break
    else:
        raise RuntimeError("could not build a covering reaction set")
    kinds = ["plain"] * n_reactions
    idx = rng.permutation(n_reactions)
    for j in idx[:n_third]:
        kinds[j] = "third"
    for j in idx[n_third:n_third + n_troe]:
        kinds[j] = "troe"
    reactions = []
    for j, (reac, prod) in enumerate(rx):
        lgA, b, Ea = _arrhenius(rng)
        r = Reaction(kind=kinds[j], reac=reac, prod=prod, log10A=lgA, b=b, Ea=Ea)
        if kinds[j] != "plain":
            n_eff = int(rng.integers(0, 4))
            for k in rng.choice(len(species), size=n_eff, replace=False):
                r.eff[int(k)] = float(rng.uniform(0.0, 5.0))
        if kinds[j] == "troe":
            r.troe = (lgA + 5.0 + rng.uniform(-3.0, 3.0), b, rng.uniform(0.0, 1.0) * Ea,
                      rng.uniform(0.1, 0.9), 10 ** rng.uniform(1, 3), 10 ** rng.uniform(2.5, 4),
                      10 ** rng.uniform(3, 4))
        reactions.append(r)
    mech = Mechanism(elements=list(elements), species=species, reactions=reactions,
                     name=name or f"syn{n_species}x{n_reactions}s{seed}")
    return mech


# ----------------------------------------------------------------------------
# the workloads' mechanisms and small hand-built ones for closed-form checks
# ----------------------------------------------------------------------------

MECH_SPECS = {
    # 9 species {H,O,N}, 24 reactions, 3 third-body
    "h2_9": dict(n_species=9, n_reactions=24, n_third=3, n_troe=0, elements=["H", "O", "N"],
                 seed=101),
    # GRI-3.0-size C/H/O/N: 53 species, 325 reactions, 30 third-body, 15 Troe
    "chon_53": dict(n_species=53, n_reactions=325, n_third=30, n_troe=15,
                    elements=["C", "H", "O", "N"], seed=102),
    # 110 species, 700 reactions, third-body/Troe in the same proportions
    "chon_110": dict(n_species=110, n_reactions=700, n_third=65, n_troe=32,
                     elements=["C", "H", "O", "N"], seed=103),
}

_CACHE = {}


def standard_mechanism(key) -> Mechanism:
    if key not in _CACHE:
        _CACHE[key] = make_mechanism(name=key, **MECH_SPECS[key])
    return _CACHE[key]


def isomer_mechanism(log10A=10.0, b=0.0, Ea=40e3, ds_R=0.7, comp=None) -> Mechanism:
    """Two isomers A, B (same composition, so equal molar mass) with identical
    a1..a6 (equal enthalpy, so an adiabatic reactor stays isothermal) and
    a7 differing by ``ds_R`` (so K = exp(ds_R)), and the single reaction
    A <=> B.  The mass fraction of A then relaxes exponentially."""
    comp = comp or {"H": 1, "O": 1, "N": 1}
    rng = np.random.default_rng(7)
    base = _nasa7(rng, comp, 10e3, 200.0)
    W = sum(ATOMIC_WEIGHT[e] * v for e, v in comp.items()) / 1000.0
    spA = Species("A", dict(comp), "skeleton", W, base, 10e3, 200.0)
    nb = list(base)
    nb[6] += ds_R
    spB = Species("B", dict(comp), "skeleton", W, tuple(nb), 10e3, 200.0 + ds_R * R_GAS)
    rx = Reaction("plain", [(0, 1)], [(1, 1)], log10A, b, Ea)
    return Mechanism(elements=["H", "O", "N"], species=[spA, spB], reactions=[rx],
                     name="isomer")


def single_reaction_mechanism(kind, seed=5, troe=None, eff=None, log10A=12.0, b=0.5,
                              Ea=30e3) -> Mechanism:
    """Species H, O, OH, N2 and one reaction H + O (+M) <=> OH (+M) of the given
    kind ('plain', 'third' or 'troe').  A plain H + O <=> OH is allowed here:
    only the 2-3-species-per-side rule of the random workloads is dropped."""
    rng = np.random.default_rng(seed)
    sp = []
    for n in ("H", "O", "OH", "N2"):
        comp, role = _CORE[n]
        h = _h298(rng, role)
        s = R_GAS * (13.0 + 3.0 * sum(comp.values()))
        x = Species(n, dict(comp), role, sum(ATOMIC_WEIGHT[e] * v for e, v in comp.items()) / 1000.0,
                    (), h, s)
        x.nasa = _nasa7(rng, comp, h, s)
        sp.append(x)
    r = Reaction(kind, [(0, 1), (1, 1)], [(2, 1)], log10A, b, Ea)
    if kind != "plain":
        r.eff = dict(eff or {})
    if kind == "troe":
        r.troe = tuple(troe or (log10A + 4.0, b, 0.5 * Ea, 0.6, 100.0, 3000.0, 5000.0))
    return Mechanism(elements=["H", "O", "N"], species=sp, reactions=[r], name=f"single_{kind}")
