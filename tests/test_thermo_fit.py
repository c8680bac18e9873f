"""CPU tests of the interpolated thermodynamics' tables (sc_mech_thermo_fit,
host only).  Each reaction's -dG/RT and dH/RT are recomputed here in NumPy
from the mechanism's NASA-7 coefficients and net stoichiometry (not from
the library), at random temperatures over the whole range, and compared
with the tables' polynomials: the error stays within the requested
tolerance.  The chosen degree has the smallest table among the degrees
that reach the tolerance, and bad arguments are refused."""
import numpy as np
import pytest

import paper_2311_14941_amd as sc
from synth.mechgen import standard_mechanism


@pytest.fixture(scope="module", autouse=True)
def built():
    sc.ensure_built()


def exact(m, T):
    """-dG/RT and dH/RT of every reaction at temperatures T: [len(T), R] each."""
    a = m.nasa_array()  # [N, 7]
    T = np.asarray(T, dtype=np.float64)[:, None]
    lnT = np.log(T)
    hRT = a[:, 0] + T * (a[:, 1] / 2 + T * (a[:, 2] / 3 + T * (a[:, 3] / 4 + T * a[:, 4] / 5))) + a[:, 5] / T
    sR = a[:, 0] * lnT + T * (a[:, 1] + T * (a[:, 2] / 2 + T * (a[:, 3] / 3 + T * a[:, 4] / 4))) + a[:, 6]
    nu = m.stoich()  # [N, R]
    return -(hRT - sR) @ nu, hRT @ nu


def table(fit, T):
    """The tables' values at T: [len(T), R] for each function."""
    u = (np.log(T) - fit["u0"]) / fit["du"]
    iv = np.floor(u).astype(int)
    t = 2.0 * (u - iv) - 1.0
    c = fit["coef"][iv]  # [n, R, 2, d + 1]
    p = c[..., -1]
    for q in range(c.shape[-1] - 2, -1, -1):
        p = p * t[:, None, None] + c[..., q]
    return p[..., 0], p[..., 1]


@pytest.mark.parametrize("key,tol", [("h2_9", 1e-10), ("chon_53", 1e-9), ("chon_53", 1e-12)])
def test_tables_meet_the_tolerance(key, tol):
    m = standard_mechanism(key)
    cm = sc.Mechanism(m.to_text())
    fit = cm.thermo_fit(tol)
    assert 1 <= fit["degree"] <= 8 and fit["nint"] >= 1 and fit["max_err"] <= tol
    rng = np.random.default_rng(7)
    T = np.exp(rng.uniform(np.log(250.0), np.log(4000.0), 3000))
    g1, h1 = exact(m, T)
    g2, h2 = table(fit, T)
    # the check grid is finite: allow a small margin beyond it, and the
    # rounding of values of a few hundred
    bound = 1.5 * tol + 1e-13 * max(1.0, np.abs(g1).max())
    assert np.abs(g2 - g1).max() <= bound and np.abs(h2 - h1).max() <= bound


def test_degree_is_the_lowest_that_fits_the_budget():
    """The chosen degree is the cheapest to evaluate whose table fits 4 MiB:
    every lower degree needs a larger table (or cannot reach the tolerance
    within its interval limit), and asking for that degree gives the same
    grid."""
    cm = sc.Mechanism(standard_mechanism("chon_53").to_text())
    tol = 1e-9
    best = cm.thermo_fit(tol)
    d = best["degree"]
    assert best["coef"].nbytes <= 4 << 20
    for lower in range(1, d):
        try:
            f = cm.thermo_fit(tol, degree=lower)
        except RuntimeError:
            continue  # cannot reach tol within the interval limit
        assert f["coef"].nbytes > 4 << 20
    f = cm.thermo_fit(tol, degree=d)
    assert f["nint"] == best["nint"]


def test_fit_arguments():
    cm = sc.Mechanism(standard_mechanism("h2_9").to_text())
    for kw in (dict(tol=0.0), dict(tol=1e-9, Tmin=0.0), dict(tol=1e-9, Tmin=500.0, Tmax=400.0),
               dict(tol=1e-9, degree=9)):
        with pytest.raises(RuntimeError, match="thermo"):
            cm.thermo_fit(**kw)
