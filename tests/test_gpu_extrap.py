"""The extrapolation baseline (sc_options.method = SC_METHOD_EXTRAP: linearly
implicit Euler on the step numbers 1..4, Aitken-Neville extrapolation to
order 4) through the C ABI.

* one step on the linear A <=> B problem multiplies the deviation from
  equilibrium by the method's stability function, computed here from its
  definition for a scalar problem (and checked to differ from exp(-z) by
  O(z^5), i.e. order 4);
* at rtol 1e-10 every cell of the C1 and C2 references meets the parity bar
  against the converged oracle (tests/golden);
* the queue and plain launches agree bit for bit, and its results agree
  with the Rosenbrock method's to the production tolerance;
* the adjoint rejects it."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def sc():
    import paper_2311_14941_amd as m
    m.ensure_built()
    return m


_CELLS = {}


def cells(key):
    from synth.cells import make_cells
    if key not in _CELLS:
        _CELLS[key] = make_cells(key)
    return _CELLS[key]


def to_gpu(torch, c, idx):
    d = "cuda:0"
    return (torch.tensor(c["T"][idx], dtype=torch.float64, device=d),
            torch.tensor(c["p"][idx], dtype=torch.float64, device=d),
            torch.tensor(np.ascontiguousarray(c["Y"][idx].T), dtype=torch.float64, device=d),
            torch.tensor(c["dt"][idx], dtype=torch.float64, device=d))


def excess(T, Y, Tref, Yref):
    eT = np.abs(T - Tref) / (1e-6 * np.abs(Tref))
    big = np.abs(Yref) > 1e-8
    eY = np.where(big, np.abs(Y - Yref) / (1e-6 * np.abs(Yref) + 1e-300), np.abs(Y - Yref) / 1e-12)
    return np.maximum(eT, eY.max(1))


def extrap_stability(z):
    """Deviation factor of one step H on y' = -k y (z = k H): substeps of the
    linearly implicit Euler method give (1 + z/j)^(-j) per column j; the
    columns are extrapolated for an error expansion in powers of H."""
    T = {}
    for j in range(1, 5):
        T[j, 1] = (1.0 + z / j) ** (-j)
        for l in range(1, j):
            T[j, l + 1] = T[j, l] + (T[j, l] - T[j - 1, l]) * (j - l) / l
    return T[4, 4]


def test_extrap_stability_function_isomer(torch, sc):
    from oracle.oracle import Oracle
    from synth.mechgen import isomer_mechanism
    # the scalar definition has order 4: local error ratio -> 2^5 on halving
    e = [abs(extrap_stability(z) - np.exp(-z)) for z in (0.04, 0.02)]
    assert 25.0 < e[0] / e[1] < 33.0
    mech = isomer_mechanism(log10A=9.0, b=0.0, Ea=40e3, ds_R=0.7)
    o = Oracle(mech.to_text())
    Tc, pc = 1000.0, 101325.0
    kf, kr, *_ = o.rates(Tc, pc, [0.5, 0.5])
    k = kf[0] + kr[0]
    Yeq = 1.0 / (1.0 + np.exp(0.7))
    plan = sc.Plan(sc.Mechanism(mech.to_text()), rtol=1e6, atol=1e6, method="extrap")  # accept the first step
    for z in (0.01, 0.5, 3.0, 50.0, 1e4):
        h = z / k
        T = torch.tensor([Tc], dtype=torch.float64, device="cuda:0")
        Y = torch.tensor([[0.9], [0.1]], dtype=torch.float64, device="cuda:0")
        r = plan.integrate(T, pc, Y, torch.tensor([h], dtype=torch.float64, device="cuda:0"))
        assert int(r["n_acc"][0]) == 1 and int(r["n_rej"][0]) == 0
        got = (r["Y"][0, 0].item() - Yeq) / (0.9 - Yeq)
        want = extrap_stability(z)
        # each substep forms y + dy with dy = -(deviation)(hk/(1 + hk)): at
        # large z the sum cancels to the deviation and keeps absolute
        # rounding of order eps |Y| per substep (ten substeps, extrapolation
        # weights up to 3), hence 4e-12 rather than the last bit
        assert abs(got - want) < 4e-12, (z, got, want)
        assert float(r["T"][0]) == Tc


@pytest.mark.parametrize("key,golden", [("C1", "c1_ref.npz"), ("C2", "c2_ref.npz")])
def test_extrap_tight_tolerance_parity(torch, sc, key, golden):
    c = cells(key)
    g = np.load(os.path.join(HERE, "golden", golden))
    idx = g["idx"]
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()), rtol=1e-10, atol=1e-16, max_steps=200000, method="extrap")
    T, p, Y, dt = to_gpu(torch, c, idx)
    r = plan.integrate(T, p, Y, dt)
    st = r["status"].cpu().numpy()
    assert np.all(st == 0), np.bincount(st)
    ex = excess(r["T"].cpu().numpy(), r["Y"].cpu().numpy().T, g["T"], g["Y"])
    print(f"{key} extrapolation: worst parity excess {ex.max():.3g} (<= 1 passes)")
    assert np.all(ex <= 1.0), (ex.max(), idx[np.argmax(ex)])


def test_extrap_launches_agree_and_match_rosenbrock(torch, sc):
    c = cells("C2")
    idx = np.arange(4096)
    T, p, Y, dt = to_gpu(torch, c, idx)
    mech = sc.Mechanism(c["mech"].to_text())
    a = sc.Plan(mech, method="extrap").integrate(T, p, Y, dt)
    q = sc.Plan(mech, method="extrap", mode="persistent", order="cost")
    b = q.integrate(T, p, Y, dt)
    b = q.integrate(T, p, Y, dt, out=b)
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert torch.equal(a[k], b[k]), k
    assert np.all(a["status"].cpu().numpy() == 0)
    ros = sc.Plan(mech).integrate(T, p, Y, dt)
    assert float(((a["T"] - ros["T"]).abs() / ros["T"]).max()) < 1e-4
    Y0, Y1 = c["Y"][idx], a["Y"].cpu().numpy().T
    assert np.abs(Y1.sum(1) - Y0.sum(1)).max() < 1e-13


def test_extrap_adjoint_rejected(torch, sc):
    c = cells("C2")
    T, p, Y, dt = to_gpu(torch, c, np.arange(8))
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()), method="extrap")
    with pytest.raises(sc.StiffchemError) as e:
        plan.adjoint(T, p, Y, dt, torch.ones_like(T), torch.zeros_like(Y))
    assert e.value.code == sc.SC_EUNSUPPORTED
