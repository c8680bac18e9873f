"""Pins of the CPU reference of zonal reference-cell mapping
(oracle/mapping.py): the mixture fraction against closed forms that a wrong
weight or sign would break, the zone and reference choice against a brute
force search, and the mapped integration against its special cases."""
import math

import numpy as np
import pytest

from oracle import mapping as om


def _mech_text():
    from synth.mechgen import standard_mechanism
    return standard_mechanism("chon_53").to_text()


@pytest.fixture(scope="module")
def chon():
    from synth.mechgen import standard_mechanism
    m = standard_mechanism("chon_53")
    return m, m.to_text()


def _mass(m, moles):
    W = m.molar_masses()
    x = np.zeros(m.n_species)
    for k, v in moles.items():
        x[m.index(k)] = v
    y = x * W
    return y / y.sum()


def test_stoichiometric_methane_air(chon):
    """Bilger's coupling function vanishes at stoichiometry: for pure CH4
    against air (O2 0.233, N2 0.767 by mass) the stoichiometric mixture
    fraction is 1 / (1 + s / Y_O2) with s = 2 W_O2 / W_CH4 the mass of
    oxygen per mass of fuel, about 0.055; the mixture of that fraction has
    Z equal to it, the stoichiometric products (CO2 + 2 H2O + the air's N2)
    too, and both have beta = 0.  A wrong element weight moves the zero."""
    m, text = chon
    W = dict(zip([s.name for s in m.species], m.molar_masses()))
    fuel = _mass(m, {"CH4": 1.0})
    air = np.zeros(m.n_species)
    air[m.index("O2")], air[m.index("N2")] = 0.233, 0.767
    s = 2 * W["O2"] / W["CH4"]
    z_st = 1.0 / (1.0 + s / 0.233)
    assert abs(z_st - 0.055) < 1e-3
    w = om.bilger_weights(text)
    mix = z_st * fuel + (1 - z_st) * air
    assert abs(w @ mix) < 1e-12 * np.abs(w) @ mix
    assert abs(om.mixture_fraction(w, mix, fuel, air)[0] - z_st) < 1e-13
    # complete combustion of that mixture: per kg, CH4 -> CO2 + 2 H2O
    nf = z_st / W["CH4"]
    prod = np.zeros(m.n_species)
    prod[m.index("CO2")] = nf * W["CO2"]
    prod[m.index("H2O")] = 2 * nf * W["H2O"]
    prod[m.index("N2")] = (1 - z_st) * 0.767
    assert abs(prod.sum() - 1.0) < 1e-12
    assert abs(om.mixture_fraction(w, prod, fuel, air)[0] - z_st) < 1e-12


def test_mixture_fraction_streams_and_linearity(chon):
    """Z = 1 in the fuel, 0 in the oxidiser, a in the mass mixture a fuel +
    (1 - a) oxidiser, and unchanged by any reaction of the mechanism (each
    conserves the elements)."""
    m, text = chon
    rng = np.random.default_rng(3)
    w = om.bilger_weights(text)
    fuel = _mass(m, {"CH4": 0.2, "NH3": 0.05, "O2": 0.157, "N2": 0.593})
    air = _mass(m, {"O2": 0.21, "N2": 0.79})
    Z = om.mixture_fraction(w, np.stack([fuel, air]), fuel, air)
    assert abs(Z[0] - 1.0) < 1e-14 and abs(Z[1]) < 1e-14
    for a in rng.uniform(0, 1, 5):
        assert abs(om.mixture_fraction(w, a * fuel + (1 - a) * air, fuel, air)[0] - a) < 1e-13
    # a reaction's net change of mass fractions: dY_k = nu_k W_k (per mol)
    W = m.molar_masses()
    for r in m.reactions[:40]:
        d = np.zeros(m.n_species)
        for k, v in r.reac:
            d[k] -= v * W[k]
        for k, v in r.prod:
            d[k] += v * W[k]
        assert abs(w @ d) < 1e-12 * (np.abs(w) @ np.abs(d))


def _brute_refs(T, p, Y, dt, w, fuel, ox, z_tol, dT, dlnp):
    """O(n^2) search: a mappable cell's reference is the lowest-index
    mappable cell with the same temperature band and pressure band."""
    n = len(T)
    Z = [(w @ Y[c] - w @ ox) / (w @ fuel - w @ ox) for c in range(n)]

    def band(c):
        if not (Z[c] < z_tol and dt[c] > 0 and T[c] > 0 and p[c] > 0):
            return None
        iT = math.floor(T[c] / dT)
        if iT >= math.ceil(om.T_MAX / dT):
            return None
        ip = 0
        if dlnp > 0:
            ip = math.floor(math.log(p[c]) / dlnp)
            if not 0 <= ip < math.ceil(math.log(om.P_MAX) / dlnp):
                return None
        return iT, ip

    bands = [band(c) for c in range(n)]
    ref = np.arange(n)
    for c in range(n):
        if bands[c] is not None:
            ref[c] = min(d for d in range(n) if bands[d] == bands[c])
    return ref


@pytest.mark.parametrize("dlnp", [0.0, 0.3])
def test_references_brute_force(chon, dlnp):
    m, text = chon
    rng = np.random.default_rng(11)
    w = om.bilger_weights(text)
    fuel = _mass(m, {"CH4": 1.0})
    air = _mass(m, {"O2": 0.21, "N2": 0.79})
    n = 60
    a = np.where(rng.uniform(size=n) < 0.6, rng.uniform(0, 2e-3, n), rng.uniform(0, 1, n))
    Y = a[:, None] * fuel + (1 - a[:, None]) * air
    T = rng.choice([300.0, 301.5, 305.0, 900.0, 12000.0], n)
    p = 101325.0 * rng.choice([1.0, 1.2, 3.0], n)
    dt = np.where(rng.uniform(size=n) < 0.1, 0.0, 1e-5)
    got = om.references(om.zones(T, p, Y, dt, w, fuel, air, 1e-3, 2.0, dlnp))
    ref = _brute_refs(T, p, Y, dt, w, fuel, air, 1e-3, 2.0, dlnp)
    assert np.array_equal(got, ref)
    assert np.any(got != np.arange(n)) and np.any(got == np.arange(n))
    # every reference is its own reference, and no cell maps to a later one
    assert np.array_equal(got[got], got) and np.all(got <= np.arange(n))


def test_mapped_integration_special_cases(chon):
    """A z_tol below every cell's Z maps nothing: the result is the
    oracle's integration of every cell.  Copies of one state with one dt map exactly onto their
    reference (to the rounding of y0 + (y1 - y0)); a copy with twice the
    step takes twice the reference's change."""
    from oracle.oracle import Oracle
    from synth.cells import make_cells
    m, text = chon
    o = Oracle(text)
    c = make_cells("C2", n=24)
    fuel = _mass(m, {"CH4": 1.0})
    air = _mass(m, {"O2": 0.21, "N2": 0.79})
    T, p, Y, dt = c["T"], c["p"], c["Y"], c["dt"]
    plain = o.integrate(T, p, Y, dt, rtol=1e-8, atol=1e-14)
    r = om.integrate_mapped(o, text, T, p, Y, dt, fuel, air, -1e300, 5.0, rtol=1e-8, atol=1e-14)
    assert np.array_equal(r["ref"], np.arange(T.size))
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert np.array_equal(r[k], plain[k])
    # a warm air-side state, copied: all copies share the first as reference
    y0 = 0.999 * air + 0.001 * fuel
    n = 4
    Tc, pc = np.full(n, 1400.0), np.full(n, 101325.0)
    Yc = np.tile(y0, (n, 1))
    dtc = np.array([1e-5, 1e-5, 1e-5, 2e-5])
    r = om.integrate_mapped(o, text, Tc, pc, Yc, dtc, fuel, air, 2e-3, 5.0, rtol=1e-8, atol=1e-14)
    assert np.array_equal(r["ref"], [0, 0, 0, 0])
    assert np.array_equal(r["n_acc"][1:], [0, 0, 0]) and r["n_acc"][0] > 0
    d = r["Y"][0] - Yc[0]
    assert np.max(np.abs(r["Y"][1] - r["Y"][0])) <= 1e-16
    assert np.max(np.abs((r["Y"][3] - Yc[3]) - 2 * d)) <= 1e-16
    assert abs((r["T"][3] - Tc[3]) - 2 * (r["T"][0] - Tc[0])) <= 1e-12 * Tc[0]
    assert abs(r["Y"][3].sum() - 1.0) < 1e-14
