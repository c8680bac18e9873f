"""Pins of the oracle's constant-volume reactor (rho fixed, p varies; energy
balance on internal energy).

* closed form: an exothermic first-order isomerisation A -> B with constant
  heat capacity and a temperature-independent rate; Y_A decays exponentially
  and T follows from u = const: T = T0 + (Y_A0 - Y_A)(a6_A - a6_B)/(a1 - 1)
  (NASA-7 a1 = cp/R, a6 = the enthalpy constant).  The constant-pressure
  reactor gives a1 instead of a1 - 1 in the denominator, so a heat capacity
  taken at the wrong constraint fails it;
* conservation along C2 integrations: mass fractions, elements and the
  mass-specific internal energy sum_k Y_k (h_k - R T)/W_k;
* at one state, the production rates of the constant-volume reactor at
  density rho equal the constant-pressure ones at p = rho R T / Wbar (same
  concentrations);
* the complex-step Jacobian of the constant-volume right-hand side agrees
  with central differences."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from synth.cells import make_cells
from synth.mechgen import ATOMIC_WEIGHT, R_GAS, Mechanism, Reaction, Species


def _exo_isomer(a1=4.5, dh_R=-6000.0, ds_R=30.0, log10A=3.0):
    comp = {"H": 1, "O": 1, "N": 1}
    W = sum(ATOMIC_WEIGHT[e] * v for e, v in comp.items()) / 1000.0
    a6A, a7A = 1000.0, 20.0
    nA = (a1, 0.0, 0.0, 0.0, 0.0, a6A, a7A)
    nB = (a1, 0.0, 0.0, 0.0, 0.0, a6A + dh_R, a7A + ds_R)
    sA = Species("A", dict(comp), "skeleton", W, nA, a6A * R_GAS, a7A * R_GAS)
    sB = Species("B", dict(comp), "skeleton", W, nB, (a6A + dh_R) * R_GAS, (a7A + ds_R) * R_GAS)
    rx = Reaction("plain", [(0, 1)], [(1, 1)], log10A, 0.0, 0.0)
    return Mechanism(elements=["H", "O", "N"], species=[sA, sB], reactions=[rx], name="exo_isomer"), W


@pytest.mark.parametrize("constv", [True, False])
def test_exothermic_isomer_closed_form(constv):
    a1, dh_R = 4.5, -6000.0
    mech, W = _exo_isomer(a1=a1, dh_R=dh_R)
    o = Oracle(mech.to_text())
    k = 10.0 ** 3.0
    T0, YA0 = 900.0, 0.8
    rho = 1.2
    p = rho if constv else rho * R_GAS * T0 / W
    ts = np.array([0.2, 1.0, 3.0]) / k
    n = ts.size
    r = o.integrate(np.full(n, T0), p, np.tile([YA0, 1 - YA0], (n, 1)), ts, rtol=1e-12, atol=1e-18,
                    constv=constv)
    assert np.all(r["status"] == 0)
    YA = YA0 * np.exp(-k * ts)
    # the reverse rate is exp(-(6000/T + 30)) of the forward one: below 1e-15
    assert np.allclose(r["Y"][:, 0], YA, rtol=1e-10, atol=0)
    c = (a1 - 1.0) if constv else a1
    T = T0 + (YA0 - YA) * (-dh_R) / c
    assert np.allclose(r["T"], T, rtol=1e-11, atol=0)


def test_constv_conserves_internal_energy_mass_and_elements():
    cells = make_cells("C2", n=96)
    mech = cells["mech"]
    o = Oracle(mech.to_text())
    W = mech.molar_masses()
    A = mech.element_matrix() / W[None, :]
    idx = np.nonzero(cells["cls"] == 1)[0][:12]     # near ignition: heat release
    idx = np.concatenate([idx, np.nonzero(cells["cls"] == 2)[0][:6]])
    Y0, T0 = cells["Y"][idx], cells["T"][idx]
    Wbar = 1.0 / (Y0 / W).sum(1)
    rho = cells["p"][idx] * Wbar / (R_GAS * T0)
    r = o.integrate(T0, rho, Y0, cells["dt"][idx], rtol=1e-10, atol=1e-16, constv=True)
    assert np.all(r["status"] == 0)
    assert np.abs(r["Y"].sum(1) - Y0.sum(1)).max() < 1e-13
    e0, e1 = A @ Y0.T, A @ r["Y"].T
    assert np.abs(e1 - e0).max() < 1e-12 * np.abs(e0).max()
    moved = 0
    for n in range(idx.size):
        u0 = (o.thermo(T0[n])[1] - 1.0) * R_GAS * T0[n]
        u1 = (o.thermo(r["T"][n])[1] - 1.0) * R_GAS * r["T"][n]
        U0 = np.sum(Y0[n] * u0 / W)
        U1 = np.sum(r["Y"][n] * u1 / W)
        scale = np.sum(np.abs(Y0[n] * u0 / W))
        assert abs(U1 - U0) < 1e-8 * scale, n
        moved += abs(r["T"][n] - T0[n]) > 1.0
    assert moved >= 3  # the pin is not vacuous: several cells heat up
    # the same cells at constant pressure end elsewhere
    rp = o.integrate(T0, cells["p"][idx], Y0, cells["dt"][idx], rtol=1e-10, atol=1e-16)
    assert np.abs(rp["T"] - r["T"]).max() > 1.0


def test_constv_rates_match_constp_at_same_concentrations():
    cells = make_cells("C2", n=32)
    mech = cells["mech"]
    o = Oracle(mech.to_text())
    W = mech.molar_masses()
    for i in range(0, 32, 5):
        T, Y = cells["T"][i], cells["Y"][i]
        Wbar = 1.0 / np.sum(Y / W)
        rho = 0.37 + 0.1 * i
        p = rho * R_GAS * T / Wbar
        _, _, qv, wv, auxv = o.rates(T, rho, Y, constv=True)
        _, _, qp, wp, auxp = o.rates(T, p, Y)
        assert abs(auxv[0] - rho) <= 1e-15 * rho and abs(auxp[0] - rho) <= 1e-13 * rho
        gross = np.abs(qp).max()
        assert np.allclose(qv, qp, rtol=1e-12, atol=1e-12 * gross)
        assert np.allclose(wv, wp, rtol=1e-12, atol=1e-12 * np.abs(wp).max())


def test_constv_jacobian_complex_step_vs_central_differences():
    cells = make_cells("C2", n=16)
    mech = cells["mech"]
    o = Oracle(mech.to_text())
    W = mech.molar_masses()
    rng = np.random.default_rng(3)
    for i in range(4):
        y = np.append(cells["Y"][i], cells["T"][i])
        rho = cells["p"][i] / (R_GAS * cells["T"][i] * np.sum(cells["Y"][i] / W))
        Jc = o.jac_cs(y, rho, constv=True)
        v = rng.normal(size=y.size) * np.maximum(np.abs(y), 1e-6)
        eps = 1e-6
        cd = (o.rhs(y + eps * v, rho, constv=True) - o.rhs(y - eps * v, rho, constv=True)) / (2 * eps)
        assert np.allclose(Jc @ v, cd, rtol=1e-5, atol=1e-6 * np.abs(Jc @ v).max())
        # a constant-volume Jacobian differs from the constant-pressure one
        Jp = o.jac_cs(y, cells["p"][i])
        assert np.abs(Jp - Jc).max() > 1e-6 * np.abs(Jc).max()
