"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, conservation laws, thermodynamic identities, library routines
(NumPy, SciPy) and independently generated equilibrium states.

Each test names the mistake it would catch."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.oracle import Oracle, dense_solve, radau_coeffs
from synth.cells import equilibrium_tp, make_cells, mole_to_mass
from synth.mechgen import (P_REF, R_GAS, isomer_mechanism, single_reaction_mechanism,
                           standard_mechanism)


@pytest.fixture(scope="module")
def c1():
    cells = make_cells("C1", n=64)
    return cells, Oracle(cells["mech"].to_text())


@pytest.fixture(scope="module")
def c2():
    cells = make_cells("C2", n=96)
    return cells, Oracle(cells["mech"].to_text())


def _y(cells, i):
    return np.append(cells["Y"][i], cells["T"][i])


# --------------------------------------------------------------------------
# Radau IIA coefficients
# --------------------------------------------------------------------------

def test_radau_coefficients_satisfy_order_conditions():
    """B(5): sum_i b_i c_i^(q-1) = 1/q, q=1..5 (order 5) although only C(3)
    was used to build A; stiff accuracy b = last row.  A wrong node or a
    transposed A fails this."""
    c, A = radau_coeffs()
    b = A[2]
    for q in range(1, 6):
        assert abs(np.dot(b, c ** (q - 1)) - 1.0 / q) < 1e-14
    # D(1): sum_i b_i a_ij = b_j (1 - c_j)
    assert np.allclose(b @ A, b * (1 - c), atol=1e-14)
    # nodes are the roots of the Radau IIA polynomial d^2/dx^2 [x^2 (x-1)^3]
    P = np.polynomial.Polynomial([0, 0, 1]) * np.polynomial.Polynomial([-1, 1]) ** 3
    assert np.allclose(np.sort(P.deriv(2).roots().real), c, atol=1e-14)


# --------------------------------------------------------------------------
# thermodynamics
# --------------------------------------------------------------------------

@pytest.mark.parametrize("key", ["h2_9", "chon_53"])
def test_thermo_identities(key):
    """cp = dh/dT and cp/T = ds/dT (central differences), and h, s at 298.15 K
    equal the generator's targets.  Catches a wrong power/divisor in any
    NASA-7 term or a swapped a6/a7."""
    mech = standard_mechanism(key)
    o = Oracle(mech.to_text())
    for T in (300.0, 1000.0, 2500.0):
        d = 1e-4 * T
        cp, h, s = o.thermo(T)
        _, hp, sp = o.thermo(T + d)
        _, hm, sm = o.thermo(T - d)
        dh = ((T + d) * hp - (T - d) * hm) / (2 * d)  # d(h/R)/dT
        ds = (sp - sm) / (2 * d)
        assert np.allclose(dh, cp, rtol=1e-8, atol=1e-8)
        assert np.allclose(ds * T, cp, rtol=1e-7, atol=1e-7)
    cp, h, s = o.thermo(298.15)
    h298 = np.array([x.h298 for x in mech.species])
    s298 = np.array([x.s298 for x in mech.species])
    assert np.allclose(h * R_GAS * 298.15, h298, rtol=1e-12, atol=1e-6)
    assert np.allclose(s * R_GAS, s298, rtol=1e-12)


# --------------------------------------------------------------------------
# rate laws
# --------------------------------------------------------------------------

def test_arrhenius_plot_and_cgs_units():
    """ln kf against 1/T is a line of slope -Ea/R when b = 0 (np.polyfit), and
    the SI rate of a bimolecular reaction equals the cgs rate law evaluated in
    mol/cm^3 (units of A).  Catches a wrong sign of Ea, R in kJ or a wrong
    cgs->SI factor."""
    mech = single_reaction_mechanism("plain", b=0.0, Ea=55e3, log10A=12.3)
    o = Oracle(mech.to_text())
    Ts = np.linspace(500, 2500, 9)
    Y = np.array([0.4, 0.3, 0.0, 0.3])
    lnk = [math.log(o.rates(T, 101325.0, Y)[0][0]) for T in Ts]
    slope, icpt = np.polyfit(1.0 / Ts, lnk, 1)
    assert abs(slope + 55e3 / R_GAS) < 1e-6 * 55e3 / R_GAS
    # units: q [mol/m^3/s] * 1e-6 = A_cgs * C_H[mol/cm^3] * C_O[mol/cm^3]
    mech = single_reaction_mechanism("plain", b=0.0, Ea=0.0, log10A=12.3)
    o = Oracle(mech.to_text())
    T, p = 1500.0, 2 * 101325.0
    kf, kr, q, wdot, aux = o.rates(T, p, Y)
    rho = aux[0]
    W = mech.molar_masses()
    Ccgs = rho * Y / W * 1e-6
    assert abs(q[0] * 1e-6 - 10 ** 12.3 * Ccgs[0] * Ccgs[1]) < 1e-12 * abs(q[0] * 1e-6)


def test_third_body_unit_efficiencies_is_total_concentration():
    """With every efficiency 1, [M] is the total concentration p/(RT) (ideal
    gas), so a third-body reaction's rate is the plain rate times p/(RT)."""
    plain = Oracle(single_reaction_mechanism("plain").to_text())
    third = Oracle(single_reaction_mechanism("third").to_text())
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    for T, p in ((800.0, 101325.0), (2000.0, 5e5)):
        qp = plain.rates(T, p, Y)[2][0]
        qt = third.rates(T, p, Y)[2][0]
        # the same log10 A is one cgs order higher for the third-body form
        assert abs(qt - qp * 1e-6 * p / (R_GAS * T)) < 1e-12 * abs(qt)


def test_third_body_efficiency_enters_linearly():
    """[M] = sum_k alpha_k C_k: raising one efficiency by 1 adds exactly that
    species' concentration."""
    m1 = single_reaction_mechanism("third", eff={3: 1.0})
    m2 = single_reaction_mechanism("third", eff={3: 2.0})
    o1, o2 = Oracle(m1.to_text()), Oracle(m2.to_text())
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    T, p = 1200.0, 101325.0
    q1, q2 = o1.rates(T, p, Y)[2][0], o2.rates(T, p, Y)[2][0]
    rho = o1.rates(T, p, Y)[4][0]
    CN2 = rho * Y[3] / m1.molar_masses()[3]
    Mtot = p / (R_GAS * T)
    assert abs(q2 / q1 - (Mtot + CN2) / Mtot) < 1e-13


def test_troe_limits():
    """Fall-off: with Fcent = 1 (a = 0, T3 -> inf, T2 -> inf) the Troe form is
    the Lindemann form kf = kinf Pr/(1+Pr): Pr -> 0 gives k0 [M], Pr -> inf
    gives kinf, Pr = 1 gives kinf/2.  With a general Fcent the broadening at
    Pr -> 0 tends to Fcent^(1/(1+1/0.14^2)) (f -> -1/0.14)."""
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    T, p = 1000.0, 101325.0
    Mtot = p / (R_GAS * T)
    lind = (0.0, 1e30, 1000.0, 1e30)  # a, T3, T1, T2
    kinf = 10 ** 12.0 * 1e-6
    for lgPr in (-9.0, 0.0, 9.0):
        # Pr = k0 [M] / kinf with k0 = 10^lgA0 * 1e-12 (SI, one order higher)
        lgA0 = lgPr + 12.0 - 6.0 + 12.0 - math.log10(Mtot)
        m = single_reaction_mechanism("troe", troe=(lgA0, 0.0, 0.0) + lind, b=0.0, Ea=0.0,
                                      log10A=12.0)
        kf = Oracle(m.to_text()).rates(T, p, Y)[0][0]
        Pr = 10 ** lgPr
        if lgPr < 0:
            assert abs(kf / (10 ** lgA0 * 1e-12 * Mtot) - 1) < 1e-8
        elif lgPr > 0:
            assert abs(kf / kinf - 1) < 1e-8
        else:
            assert abs(kf / (0.5 * kinf) - 1) < 1e-12
    # general Fcent at Pr = 1, where f = c/(n - 0.14 c) (definition restated;
    # the Lindemann limits above are the independent pins)
    a, T3, T1, T2 = 0.3, 400.0, 2000.0, 5000.0
    Fc = (1 - a) * math.exp(-T / T3) + a * math.exp(-T / T1) + math.exp(-T2 / T)
    lgA0 = 12.0 - 6.0 + 12.0 - math.log10(Mtot)
    m = single_reaction_mechanism("troe", troe=(lgA0, 0.0, 0.0, a, T3, T1, T2), b=0.0, Ea=0.0,
                                  log10A=12.0)
    kf = Oracle(m.to_text()).rates(T, p, Y)[0][0]
    lFc = math.log10(Fc)
    c, n = -0.4 - 0.67 * lFc, 0.75 - 1.27 * lFc
    f = c / (n - 0.14 * c)
    assert abs(kf / (0.5 * kinf * 10 ** (lFc / (1 + f * f))) - 1) < 1e-12


def _troe_broadening(Fc, lgPr, T=1000.0, p=101325.0):
    """The oracle's broadening factor F = kf / (kinf Pr/(1+Pr)) of the single
    Troe reaction at centre value Fc and log10 Pr (all efficiencies 1, so
    [M] = p/(RT)).  Fc is set through (a, T3, T1, T2) = (Fc, ~0, ~inf, ~inf),
    for which the centre formula reduces to a."""
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    Mtot = p / (R_GAS * T)
    lgA0 = lgPr + 12.0 - 6.0 + 12.0 - math.log10(Mtot)
    m = single_reaction_mechanism("troe", troe=(lgA0, 0.0, 0.0, Fc, 1e-30, 1e30, 1e30), b=0.0, Ea=0.0,
                                  log10A=12.0)
    kf = Oracle(m.to_text()).rates(T, p, Y)[0][0]
    kinf = 10 ** 12.0 * 1e-6
    Pr = 10.0 ** lgPr
    return kf / (kinf * Pr / (1.0 + Pr))


@pytest.mark.parametrize("Fc", [0.12, 0.3, 0.55, 0.85])
def test_troe_broadening_properties(Fc):
    """Properties of the Troe broadening (Gilbert, Luther & Troe 1983) that
    pin each of its constants separately, for several centre values:
    (i) at log10 Pr = -c the curve passes through its centre, F = Fc (pins
        the two constants of c = -0.4 - 0.67 log10 Fc: two Fc values fix both);
    (ii) where log10 Pr + c = n/1.14 the width function f is 1, so
        log F = log Fc / 2 (pins n = 0.75 - 1.27 log10 Fc given c);
    (iii) where log10 Pr + c = n/0.14 the denominator of f vanishes, f is
        infinite and F = 1 exactly (pins the 0.14; a wrong value leaves f
        finite there and F visibly below 1).
    A mistyped constant moves the point where each property holds."""
    L = math.log10(Fc)
    c = -0.4 - 0.67 * L
    n = 0.75 - 1.27 * L
    assert abs(_troe_broadening(Fc, -c) / Fc - 1.0) < 1e-12
    assert abs(math.log10(_troe_broadening(Fc, n / 1.14 - c)) - L / 2.0) < 1e-12
    assert abs(_troe_broadening(Fc, n / 0.14 - c) - 1.0) < 1e-12
    # and a nearby point is clearly not at the pole (the check above is sharp)
    assert abs(_troe_broadening(Fc, 0.9 * n / 0.14 - c) - 1.0) > 1e-5


def test_troe_centre_special_cases():
    """The centre value Fc = (1-a) e^(-T/T3) + a e^(-T/T1) + e^(-T2/T): with
    a = 0 and T2 -> inf it is e^(-T/T3); with a = 1 and T2 -> inf it is
    e^(-T/T1); at the centre point (log10 Pr = -c) the oracle's F equals it."""
    T, p = 1400.0, 101325.0
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    Mtot = p / (R_GAS * T)
    for a, T3, T1, want in ((0.0, 900.0, 1e30, math.exp(-T / 900.0)), (1.0, 1e30, 2500.0, math.exp(-T / 2500.0))):
        L = math.log10(want)
        lgPr = 0.4 + 0.67 * L
        lgA0 = lgPr + 12.0 - 6.0 + 12.0 - math.log10(Mtot)
        m = single_reaction_mechanism("troe", troe=(lgA0, 0.0, 0.0, a, T3, T1, 1e30), b=0.0, Ea=0.0, log10A=12.0)
        kf = Oracle(m.to_text()).rates(T, p, Y)[0][0]
        Pr = 10.0 ** lgPr
        F = kf / (10 ** 12.0 * 1e-6 * Pr / (1.0 + Pr))
        assert abs(F / want - 1.0) < 1e-12


def test_parameter_derivative_of_rhs(c2):
    """om_dfdp_cs (d f / d dlnA_j, the parameter part of the adjoint's
    reference) against (i) central differences of the right-hand side in
    each dlnA_j and (ii) the closed form that follows from dlnA_j scaling the
    whole net rate q_j:  d f_k/d dlnA_j = W_k nu_kj q_j / rho and
    d f_T/d dlnA_j = -(sum_k h_k nu_kj) q_j / (rho cp), with q, rho and cp
    from om_rates and h_k from om_thermo.  A wrong reaction index, a missing
    reverse term or a stray factor fails one of them."""
    cells, o = c2
    mech = cells["mech"]
    W = mech.molar_masses()
    nu = mech.stoich()
    rng = np.random.default_rng(12)
    for i in (5, 40, 77):
        y = _y(cells, i)
        T, p = cells["T"][i], cells["p"][i]
        dl = rng.uniform(-0.3, 0.3, mech.n_reactions)
        F = o.dfdp_cs(y, p, dlnA=dl)
        eps = 1e-5
        # roundoff floor of a central difference of f: eps_mach |f| / eps
        floor = 1e-9 * (np.abs(o.rhs(y, p, dlnA=dl)) + np.abs(F).max(axis=1))
        for j in rng.choice(mech.n_reactions, 25, replace=False):
            dp, dm = dl.copy(), dl.copy()
            dp[j] += eps
            dm[j] -= eps
            cd = (o.rhs(y, p, dlnA=dp) - o.rhs(y, p, dlnA=dm)) / (2 * eps)
            assert np.all(np.abs(cd - F[:, j]) <= 1e-6 * np.abs(F[:, j]) + floor)
        kf, kr, q, wdot, aux = o.rates(T, p, y[:-1], dlnA=dl)
        rho, cp = aux[0], aux[1]
        _, hRT, _ = o.thermo(T)
        closed_Y = W[:, None] * nu * q[None, :] / rho
        closed_T = -(hRT * R_GAS * T) @ nu * q / (rho * cp)
        assert np.allclose(F[:-1], closed_Y, rtol=1e-10, atol=1e-12 * np.abs(closed_Y).max())
        assert np.allclose(F[-1], closed_T, rtol=1e-10, atol=1e-12 * np.abs(closed_T).max())


@pytest.mark.parametrize("key", ["h2_9", "chon_53", "chon_110"])
def test_mass_and_element_conservation_of_rates(key):
    """sum_k W_k wdot_k = 0 and sum_k a_ek wdot_k = 0 for every element at random
    states: a wrong stoichiometric sign or species index breaks it."""
    mech = standard_mechanism(key)
    o = Oracle(mech.to_text())
    rng = np.random.default_rng(1)
    A = mech.element_matrix()
    W = mech.molar_masses()
    nu = mech.stoich()
    for _ in range(10):
        Y = rng.dirichlet(np.ones(mech.n_species))
        T = rng.uniform(600, 2400)
        kf, kr, q, wdot, aux = o.rates(T, 101325.0 * rng.uniform(1, 10), Y)
        scale = np.sum(np.abs(W * wdot)) + 1e-300
        assert abs(np.dot(W, wdot)) <= 1e-13 * scale
        assert np.all(np.abs(A @ wdot) <= 1e-12 * np.sum(np.abs(A) * np.abs(wdot), 1) + 1e-300)
        # wdot is nu q (the generator's stoichiometry)
        assert np.allclose(wdot, nu @ q, rtol=1e-12, atol=1e-12 * np.abs(nu) @ np.abs(q))


def test_detailed_balance_at_gibbs_minimum(c2):
    """At the Gibbs-energy minimum computed by the generator (its own NASA-7
    evaluation and element-potential solve), each reaction's forward and
    reverse rates agree, so f(y_eq) = 0.  Pins Kc: its sign, the p0/(RT)
    factor and the g = h - Ts combination."""
    cells, o = c2
    mech = cells["mech"]
    rng = np.random.default_rng(3)
    for T, p in ((1300.0, 101325.0), (2300.0, 8e5), (1700.0, 3e5)):
        b = rng.dirichlet(np.ones(4)) + 0.05
        x = equilibrium_tp(mech, T, p, b[None, :])[0]
        Y = mole_to_mass(mech, x[None])[0]
        kf, kr, q, wdot, aux = o.rates(T, p, Y)
        C = aux[0] * Y / mech.molar_masses()
        for j, r in enumerate(mech.reactions):
            pf = np.prod([C[k] ** v for k, v in r.reac])
            pr = np.prod([C[k] ** v for k, v in r.prod])
            fwd, rev = kf[j] * pf, kr[j] * pr
            assert abs(fwd - rev) <= 1e-9 * max(fwd, rev) + 1e-300, (j, fwd, rev)


# --------------------------------------------------------------------------
# Jacobians and linear algebra
# --------------------------------------------------------------------------

def test_jacobian_complex_step_vs_central_differences(c1, c2):
    """Complex-step J v against a central difference of f along v (error
    O(eps^2)), on C1 and C2 states; and the forward-difference J close to it."""
    for cells, o in (c1, c2):
        rng = np.random.default_rng(2)
        for i in range(4):
            y, p = _y(cells, i), cells["p"][i]
            Jc = o.jac_cs(y, p)
            v = rng.normal(size=y.size) * np.maximum(np.abs(y), 1e-6)
            eps = 1e-6
            cd = (o.rhs(y + eps * v, p) - o.rhs(y - eps * v, p)) / (2 * eps)
            assert np.allclose(Jc @ v, cd, rtol=1e-5, atol=1e-6 * np.abs(Jc @ v).max())
            Jf = o.jac_fd(y, p)
            assert np.abs(Jf - Jc).max() <= 1e-3 * np.abs(Jc).max()


def test_jacobian_conservation_rows(c2):
    """sum_k Y_k = 1 and the element mass fractions are invariants, so the
    species rows of J sum to zero under those weights."""
    cells, o = c2
    mech = cells["mech"]
    N = mech.n_species
    A = mech.element_matrix() / mech.molar_masses()[None, :]
    for i in range(6):
        J = o.jac_cs(_y(cells, i), cells["p"][i])
        col = np.abs(J[:N]).sum(0) + 1e-300
        assert np.all(np.abs(J[:N].sum(0)) <= 1e-12 * col)
        assert np.all(np.abs(A @ J[:N]) <= 1e-11 * (np.abs(A) @ np.abs(J[:N])) + 1e-300)


def test_dense_solve_matches_numpy():
    rng = np.random.default_rng(4)
    for n in (3, 17, 55, 111):
        A = rng.normal(size=(n, n)) + n * np.eye(n) * rng.uniform(0, 1)
        b = rng.normal(size=n)
        x = dense_solve(A, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
        assert np.abs(A @ x - b).max() <= 1e-11 * np.abs(A).max() * np.abs(x).max()


# --------------------------------------------------------------------------
# integrator
# --------------------------------------------------------------------------

def test_isomer_closed_form():
    """A <=> B with equal enthalpy: T and rho constant, dY_A/dt = -kf Y_A + kr Y_B,
    so Y_A(t) = Y_eq + (Y_A0 - Y_eq) exp(-(kf+kr) t), Y_eq = 1/(1+K), K = e^0.7
    by construction of the two entropies."""
    mech = isomer_mechanism(log10A=9.0, b=0.3, Ea=50e3, ds_R=0.7)
    o = Oracle(mech.to_text())
    T, p = 1100.0, 2e5
    kf, kr, *_ = o.rates(T, p, [0.5, 0.5])
    assert abs(kf[0] / kr[0] - math.exp(0.7)) < 1e-13 * math.exp(0.7)
    k = kf[0] + kr[0]
    Yeq = 1.0 / (1.0 + math.exp(0.7))
    ts = np.array([0.1, 1.0, 3.0]) / k
    n = ts.size
    r = o.integrate(np.full(n, T), p, np.tile([0.9, 0.1], (n, 1)), ts, rtol=1e-12, atol=1e-18)
    exact = Yeq + (0.9 - Yeq) * np.exp(-k * ts)
    assert np.all(r["status"] == 0)
    assert np.allclose(r["Y"][:, 0], exact, rtol=1e-10, atol=0)
    assert np.allclose(r["T"], T, rtol=1e-13)


def test_matches_scipy_radau(c1):
    """SciPy's Radau on the oracle's right-hand side, with the complex-step
    Jacobian, agrees with the oracle integrator at tight tolerances."""
    cells, o = c1
    idx = [0, 5, 9]
    r = o.integrate(cells["T"][idx], cells["p"][idx], cells["Y"][idx], cells["dt"][idx],
                    rtol=1e-11, atol=1e-17)
    for n, i in enumerate(idx):
        p = cells["p"][i]
        sol = solve_ivp(lambda t, y: o.rhs(y, p), (0.0, cells["dt"][i]), _y(cells, i),
                        method="Radau", rtol=1e-12, atol=1e-18, jac=lambda t, y: o.jac_cs(y, p))
        yref = sol.y[:, -1]
        got = np.append(r["Y"][n], r["T"][n])
        assert np.allclose(got, yref, rtol=1e-8, atol=1e-14)


def test_conservation_and_enthalpy(c2):
    """sum Y = 1 and element mass fractions are conserved to roundoff; the
    adiabatic reactor keeps its mass-specific enthalpy (h = sum Y_k h_k/W_k)."""
    cells, o = c2
    mech = cells["mech"]
    A = mech.element_matrix() / mech.molar_masses()[None, :]
    W = mech.molar_masses()
    idx = np.arange(24)
    r = o.integrate(cells["T"][idx], cells["p"][idx], cells["Y"][idx], cells["dt"][idx],
                    rtol=1e-10, atol=1e-16)
    assert np.all(r["status"] == 0)
    assert np.abs(r["Y"].sum(1) - cells["Y"][idx].sum(1)).max() < 1e-13
    e0, e1 = A @ cells["Y"][idx].T, A @ r["Y"].T
    assert np.abs(e1 - e0).max() < 1e-12 * np.abs(e0).max()
    for n, i in enumerate(idx):
        h0 = o.thermo(cells["T"][i])[1] * R_GAS * cells["T"][i]
        h1 = o.thermo(r["T"][n])[1] * R_GAS * r["T"][n]
        H0 = np.sum(cells["Y"][i] * h0 / W)
        H1 = np.sum(r["Y"][n] * h1 / W)
        scale = np.sum(np.abs(cells["Y"][i] * h0 / W))
        assert abs(H1 - H0) < 1e-8 * scale


def test_equilibrated_cells_stay_put(c2):
    cells, o = c2
    idx = np.nonzero(cells["cls"] == 2)[0][:8]
    r = o.integrate(cells["T"][idx], cells["p"][idx], cells["Y"][idx], cells["dt"][idx],
                    rtol=1e-10, atol=1e-16)
    assert np.allclose(r["T"], cells["T"][idx], rtol=1e-12)
    assert np.allclose(r["Y"], cells["Y"][idx], rtol=1e-8, atol=1e-16)


def test_isothermal_long_time_reaches_gibbs_minimum(c1):
    """Held at fixed T for a long time, the reactor relaxes to the (T, p)
    Gibbs minimum of its elements (computed independently by the generator).
    The synthetic kinetics has slow modes, so the C1 compositions are held at
    3000 K and chained out to 1e9 s."""
    cells, o = c1
    mech = cells["mech"]
    A = mech.element_matrix()
    W = mech.molar_masses()
    for i in range(8):
        T, p = 3000.0, cells["p"][i]
        Y = cells["Y"][i][None]
        for tend in (1e-3, 1e1, 1e5, 1e9):
            r = o.integrate([T], p, Y, [tend], rtol=1e-10, atol=1e-15, isothermal=True,
                            max_steps=1000000)
            assert r["status"][0] == 0
            Y = r["Y"]
        b = (cells["Y"][i] / W) @ A.T
        yeq = mole_to_mass(mech, equilibrium_tp(mech, [T], [p], b[None]))[0]
        big = yeq > 1e-6
        assert np.allclose(Y[0][big], yeq[big], rtol=1e-9)
        assert np.allclose(Y[0], yeq, rtol=1e-5, atol=1e-13)


def test_tolerance_proportionality(c2):
    """Global error shrinks with the tolerance (brute-force convergence)."""
    cells, o = c2
    idx = np.nonzero(cells["cls"] == 1)[0][:6]
    args = (cells["T"][idx], cells["p"][idx], cells["Y"][idx], cells["dt"][idx])
    ref = o.integrate(*args, rtol=1e-12, atol=1e-18)
    errs = []
    for tol in (1e-5, 1e-7, 1e-9):
        r = o.integrate(*args, rtol=tol, atol=tol * 1e-6)
        errs.append(np.abs(r["T"] - ref["T"]).max() / ref["T"].max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8


def test_forward_sensitivity_isomer_closed_form():
    """Tangents of the A <=> B closed form: d/dY_A0 and d/d(dlnA) (dlnA scales
    kf and kr together, so only the relaxation rate changes)."""
    mech = isomer_mechanism(log10A=9.0, b=0.0, Ea=40e3, ds_R=0.7)
    o = Oracle(mech.to_text())
    T, p = 1000.0, 101325.0
    kf, kr, *_ = o.rates(T, p, [0.5, 0.5])
    k = kf[0] + kr[0]
    t = 1.5 / k
    Yeq = 1.0 / (1.0 + math.exp(0.7))
    s0 = np.zeros((1, 2, 3))
    s0[0, 0, 0] = 1.0  # direction dY_A0
    dpar = np.zeros((1, 2, 1))
    dpar[0, 1, 0] = 1.0  # direction d(dlnA)
    y, s, st = o.integrate_sens([T], p, np.array([[0.8, 0.2]]), [t], s0, dpar=dpar)
    assert st[0] == 0
    # perturbing Y_A0 alone raises the conserved total S = Y_A + Y_B, and
    # Y_eq = S/(1+K): dY_A(t)/dY_A0 = (1 - e^{-kt})/(1+K) + e^{-kt}
    e = math.exp(-k * t)
    assert abs(s[0, 0, 0] - ((1 - e) * Yeq + e)) < 1e-9
    # d/d delta: k -> k e^delta, Yeq unchanged: dY/d delta = -(Y0-Yeq) k t e^{-kt}
    assert abs(s[0, 1, 0] - (-(0.8 - Yeq) * k * t * math.exp(-k * t))) < 1e-9


def test_forward_sensitivity_vs_central_differences(c2):
    """Tangent of the integrated C2 reactor against central differences of
    the oracle integrator at tight tolerance (different algorithms)."""
    cells, o = c2
    i = int(np.nonzero(cells["cls"] == 1)[0][0])
    N = cells["mech"].n_species
    rng = np.random.default_rng(5)
    d = np.zeros(N + 1)
    d[-1] = 1.0  # temperature direction
    dp = rng.normal(size=o.R) * 0.1
    s0 = np.stack([d, np.zeros(N + 1)])[None]
    dpar = np.stack([np.zeros(o.R), dp])[None]
    y, s, st = o.integrate_sens([cells["T"][i]], cells["p"][i], cells["Y"][i][None], [cells["dt"][i]],
                                s0, dpar=dpar)
    assert st[0] == 0
    h = 1e-3
    args = dict(rtol=1e-12, atol=1e-20)
    rp = o.integrate([cells["T"][i] + h], cells["p"][i], cells["Y"][i][None], [cells["dt"][i]], **args)
    rm = o.integrate([cells["T"][i] - h], cells["p"][i], cells["Y"][i][None], [cells["dt"][i]], **args)
    fd = (rp["T"][0] - rm["T"][0]) / (2 * h)
    assert abs(s[0, 0, -1] - fd) < 1e-5 * max(1.0, abs(fd))
    e = 1e-4
    rp = o.integrate([cells["T"][i]], cells["p"][i], cells["Y"][i][None], [cells["dt"][i]], dlnA=e * dp, **args)
    rm = o.integrate([cells["T"][i]], cells["p"][i], cells["Y"][i][None], [cells["dt"][i]], dlnA=-e * dp, **args)
    fd = (rp["T"][0] - rm["T"][0]) / (2 * e)
    assert abs(s[0, 1, -1] - fd) < 1e-4 * max(1.0, abs(fd))
