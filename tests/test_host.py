"""CPU-only tests of the host side: the C ABI's symbols and host-only calls
(mechanism parsing, validation, compile-time counts), the Rosenbrock tableau
and the seeded input generators.  No device computation is made here."""
import os
import re

import numpy as np
import pytest

import paper_2311_14941_amd as sc
from paper_2311_14941_amd import tableau
from synth.cells import make_cells
from synth.mechgen import (MECH_SPECS, isomer_mechanism, make_mechanism, single_reaction_mechanism,
                           standard_mechanism)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    sc.ensure_built()


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "stiffchem.h")).read()
    names = set(re.findall(r"\b(sc_[a-z_]+)\s*\(", hdr))
    assert {"sc_mech_load", "sc_plan_create", "sc_integrate", "sc_rhs", "sc_jacobian"} <= names
    L = sc.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def test_mechanism_info_and_counts():
    m = sc.Mechanism(standard_mechanism("chon_53").to_text())
    i = m.info
    assert (i["n_species"], i["n_reactions"], i["n_third_body"], i["n_troe"]) == (53, 325, 30, 15)
    assert i["n_state"] == 54 and i["n_padded"] == 56
    n = 54
    assert i["flops_lu"] == sum((n - k - 1) + 2 * (n - k - 1) ** 2 for k in range(n))
    assert i["flops_solve"] == 2 * n * (n - 1) + n
    assert 0 < i["nnz_jac"] <= n * n
    assert m.species_index("NO") >= 0
    with pytest.raises(sc.StiffchemError):
        m.species_index("XYZ")


def test_parse_errors_are_reported():
    good = standard_mechanism("h2_9").to_text()
    cases = {
        "no header": good.replace("STIFFCHEM-MECH 1", "HELLO 1"),
        "unknown species": good.replace("RX plain", "RX plain", 1).replace(" H2O 1", " XQ 1", 1),
        "bad number": good.replace("GAS_CONSTANT 8.314462618", "GAS_CONSTANT abc"),
        "bad kind": good.replace("RX plain", "RX weird", 1),
        "truncated": good[: len(good) // 2],
    }
    for what, text in cases.items():
        with pytest.raises(sc.StiffchemError) as e:
            sc.Mechanism(text)
        assert e.value.code in (sc.SC_EPARSE, sc.SC_EINVAL), what
        assert sc.last_error(), what
    # element imbalance is caught
    lines = good.splitlines()
    for k, l in enumerate(lines):
        if l.startswith("RX "):
            t = l.split()
            t[7] = str(int(t[7]) + 1)  # first reactant coefficient
            lines[k] = " ".join(t)
            break
    with pytest.raises(sc.StiffchemError) as e:
        sc.Mechanism("\n".join(lines))
    assert "balance" in str(e.value) or e.value.code == sc.SC_EPARSE


def test_merged_coefficients_and_duplicate_efficiencies_are_rejected():
    """A side written as 'O 2 O 2' merges to nu = 4, which the kernels' integer
    powers (1..3) cannot take: SC_EUNSUPPORTED, not a silently wrong rate.
    Two efficiencies for one species of one reaction are ambiguous: SC_EPARSE."""
    from synth.mechgen import single_reaction_mechanism
    good = single_reaction_mechanism("third", eff={3: 2.0}).to_text()
    sc.Mechanism(good)  # the unmodified text loads
    lines = good.splitlines()
    k = next(i for i, l in enumerate(lines) if l.startswith("RX "))
    t = lines[k].split()
    # H 2 + H 2 + O <=> OH + 3 H: balanced, but H merges to nu = 4 on the left
    t = t[:5] + ["3", "H", "2", "H", "2", "O", "1", "2", "OH", "1", "H", "3"]
    merged = "\n".join(lines[:k] + [" ".join(t)] + lines[k + 1:])
    with pytest.raises(sc.StiffchemError) as e:
        sc.Mechanism(merged)
    assert e.value.code == sc.SC_EUNSUPPORTED and "merged" in str(e.value)
    dup = good.replace("EFF 1 N2 2.0", "EFF 2 N2 2.0 N2 3.0")
    assert dup != good
    with pytest.raises(sc.StiffchemError) as e:
        sc.Mechanism(dup)
    assert e.value.code == sc.SC_EPARSE and "duplicate efficiency" in str(e.value)


def test_oversized_mechanism_is_unsupported():
    """Up to 127 species load (the sparse kernels hold two state components
    per lane); 130 do not."""
    import copy
    from synth.mechgen import Mechanism
    base = standard_mechanism("chon_110")
    sc.Mechanism(base.to_text())
    extra = []
    for i in range(20):
        s = copy.deepcopy(base.species[i])
        s.name = f"{s.name}_X{i}"
        extra.append(s)
    big = Mechanism(elements=base.elements, species=base.species + extra, reactions=base.reactions, name="big")
    with pytest.raises(sc.StiffchemError) as e:
        sc.Mechanism(big.to_text())
    assert e.value.code == sc.SC_EUNSUPPORTED and "127" in str(e.value)


def test_null_arguments_rejected_before_any_device_call():
    L = sc.lib()
    assert L.sc_integrate(None, 4, None, None, None, 4, None, None, None, None, None, None, None, None,
                          None) == sc.SC_EINVAL
    assert L.sc_rhs(None, 1, None, None, None, 1, None, None, None, None) == sc.SC_EINVAL
    assert "NULL" in sc.last_error()


# ------------------------------------------------------------------ tableau

def test_tableau_order_conditions_and_stability():
    r = tableau.check()
    assert r["R_inf"] < 1e-10
    assert r["max_R_imag_axis"] <= 1.0 + 1e-12
    sol = tableau.derive()
    assert len(sol) == 1


def test_tableau_convergence_order():
    """Observed orders 3 (main) and 2 (embedded) on a nonlinear oscillator."""
    from scipy.integrate import solve_ivp
    t = tableau.tableau()
    a = np.array(t["a"], float)
    c = np.array(t["c"], float)
    m = np.array(t["m"], float)
    mh = np.array(t["mhat"], float)
    g = float(t["gamma"])
    f = lambda y: np.array([y[1], -y[0] - 0.5 * y[0] ** 3])
    J = lambda y: np.array([[0.0, 1.0], [-1.0 - 1.5 * y[0] ** 2, 0.0]])

    def step(y, h, w):
        M = np.eye(2) / (h * g) - J(y)
        U = []
        for i in range(4):
            Yi = y + sum(a[i, j] * U[j] for j in range(i))
            U.append(np.linalg.solve(M, f(Yi) + sum(c[i, j] / h * U[j] for j in range(i))))
        return y + sum(w[i] * U[i] for i in range(4))

    y0 = np.array([1.0, 0.0])
    ref = solve_ivp(lambda _, y: f(y), (0, 2.0), y0, method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    for w, order in ((m, 3), (mh, 2)):
        errs = []
        for n in (40, 80, 160):
            y = y0.copy()
            for _ in range(n):
                y = step(y, 2.0 / n, w)
            errs.append(np.abs(y - ref).max())
        obs = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
        assert all(abs(o - order) < 0.15 for o in obs), (order, obs)


def test_order4_tableau_conditions_and_order():
    """The device method: order-4 conditions hold, the embedded method has
    order 3 (not 4), L-stability, and observed orders 4 and 3."""
    from scipy.integrate import solve_ivp
    r4, r3 = tableau.ros4_residuals()
    assert np.abs(r4).max() < 1e-14
    assert np.abs(r3[:4]).max() < 1e-14 and np.abs(r3[4:]).max() > 1e-3
    t = tableau.ros4()
    assert abs(tableau.stability(1e12, t)[0]) < 1e-9
    assert np.abs(tableau.stability(1j * np.logspace(-3, 4, 300), t)).max() <= 1 + 1e-12
    # stage 4 is evaluated where stage 3 is
    assert np.array_equal(t["alpha"][3], t["alpha"][2]) and np.array_equal(t["a"][3], t["a"][2])
    f = lambda y: np.array([y[1], -y[0] - 0.5 * y[0] ** 3])
    J = lambda y: np.array([[0.0, 1.0], [-1.0 - 1.5 * y[0] ** 2, 0.0]])

    def run(w, n):
        y = np.array([1.0, 0.0])
        h = 2.0 / n
        for _ in range(n):
            M = np.eye(2) / (h * t["gamma"]) - J(y)
            U = []
            for i in range(4):
                Yi = y + sum(t["a"][i, j] * U[j] for j in range(i))
                U.append(np.linalg.solve(M, f(Yi) + sum(t["c"][i, j] / h * U[j] for j in range(i))))
            y = y + sum(w[i] * U[i] for i in range(4))
        return y

    ref = solve_ivp(lambda _, y: f(y), (0, 2.0), [1.0, 0.0], method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    for w, order in ((t["m"], 4), (t["mhat"], 3)):
        e = [np.abs(run(w, n) - ref).max() for n in (20, 40, 80)]
        obs = np.log2(e[0] / e[1]), np.log2(e[1] / e[2])
        assert all(abs(o - order) < 0.15 for o in obs), (order, obs)


def test_device_tableau_matches_derivation():
    """The constants compiled into the kernels equal the derived order-4 tableau."""
    src = open(os.path.join(ROOT, "paper_2311_14941_amd", "csrc", "core.hpp")).read()
    t = tableau.ros4()
    num = lambda s: [float(x) for x in re.findall(r"-?[0-9]+\.[0-9]+(?:e-?[0-9]+)?", s)]
    TA = num(re.search(r"TA\[NS\]\[NS\] = \{(.*?)\};", src, re.S).group(1))
    TC = num(re.search(r"TC\[NS\]\[NS\] = \{(.*?)\};", src, re.S).group(1))
    TM = num(re.search(r"TM\[NS\] = \{(.*?)\};", src, re.S).group(1))
    TE = num(re.search(r"TE\[NS\] = \{(.*?)\};", src, re.S).group(1))
    GAM = float(re.search(r"constexpr double GAM = ([0-9.e-]+);", src).group(1))
    assert GAM == t["gamma"]
    assert np.array_equal(TA, t["a"].ravel())
    assert np.array_equal(TC, t["c"].ravel())
    assert np.array_equal(TM, t["m"])
    assert np.array_equal(TE, t["m"] - t["mhat"])
    reuse = [int(x) for x in re.search(r"TREUSE\[NS\] = \{(.*?)\};", src).group(1).split(",")]
    assert reuse == t["reuse"]


# ------------------------------------------------------------------ generator

@pytest.mark.parametrize("key", list(MECH_SPECS))
def test_generator_balance_counts_and_determinism(key):
    m = standard_mechanism(key)
    spec = MECH_SPECS[key]
    assert m.n_species == spec["n_species"] and m.n_reactions == spec["n_reactions"]
    assert sum(r.kind == "third" for r in m.reactions) == spec["n_third"]
    assert sum(r.kind == "troe" for r in m.reactions) == spec["n_troe"]
    assert np.abs(m.element_matrix() @ m.stoich()).max() == 0
    m2 = make_mechanism(**spec)
    assert m2.to_text().replace(m2.name, m.name) == m.to_text()
    # every species takes part in some reaction; sides have 2-3 species
    assert np.all(np.abs(m.stoich()).sum(1) > 0)
    for r in m.reactions:
        assert 2 <= sum(v for _, v in r.reac) <= 3 and 2 <= sum(v for _, v in r.prod) <= 3
    # NASA-7 heat capacity positive and increasing on [200, 6000] K
    T = np.linspace(200, 6000, 200)
    a = m.nasa_array()
    cp = a[:, 0:1] + a[:, 1:2] * T + a[:, 2:3] * T**2 + a[:, 3:4] * T**3 + a[:, 4:5] * T**4
    assert np.all(cp > 0) and np.all(np.diff(cp, axis=1) >= -1e-9)
    # the NO analogue exists
    assert m.species[m.index("NO")].comp == {"N": 1, "O": 1}


def test_cell_classes():
    c = make_cells("C2", n=3000)
    assert set(np.unique(c["cls"])) == {0, 1, 2}
    assert np.allclose(c["Y"].sum(1), 1.0, atol=1e-14)
    assert np.all(c["Y"] >= 0)
    assert c["T"].min() >= 300 and c["T"].max() <= 2400
    mech = c["mech"]
    rad = [mech.index(x) for x in ("H", "O", "OH", "HO2")]
    assert np.all(c["Y"][c["cls"] == 0][:, rad] == 0)
    m = c["Y"][c["cls"] == 1][:, rad].sum(1)
    assert m.min() >= 1e-4 * 0.99 and m.max() <= 1e-2 * 1.01
    c3 = make_cells("C3", n=4000)
    assert c3["dt"].min() >= 1e-7 and c3["dt"].max() <= 1e-3


def test_small_builders():
    iso = isomer_mechanism()
    assert iso.species[0].W == iso.species[1].W
    assert iso.species[0].nasa[:6] == iso.species[1].nasa[:6]
    for k in ("plain", "third", "troe"):
        single_reaction_mechanism(k)


def test_bench_calls_match_package_signatures():
    """Every keyword that bench.py passes to Plan, autotune.tune, SplitDriver
    and the package's functions exists in their signatures (the benchmark
    itself only runs on a GPU)."""
    import ast
    import inspect

    import paper_2311_14941_amd as sc
    from paper_2311_14941_amd import autotune, driver
    targets = {"Plan": sc.Plan.__init__, "tune": autotune.tune, "SplitDriver": driver.SplitDriver.__init__,
               "chem_integrate": sc.chem_integrate, "Chain": sc.Chain.__init__, "transport2d": sc.transport2d}
    src = open(os.path.join(ROOT, "bench.py")).read()
    seen = set()
    for node in ast.walk(ast.parse(src)):
        if isinstance(node, ast.Call):
            f = node.func
            name = f.attr if isinstance(f, ast.Attribute) else getattr(f, "id", None)
            if name in targets:
                params = inspect.signature(targets[name]).parameters
                for kw in node.keywords:
                    if kw.arg is not None:
                        assert kw.arg in params, (name, kw.arg)
                seen.add(name)
    assert {"Plan", "tune", "SplitDriver"} <= seen
