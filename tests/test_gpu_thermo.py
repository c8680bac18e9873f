"""Interpolated thermodynamics (sc_options.thermo_tol > 0: each reaction's
-dG/RT and dH/RT from piecewise polynomials in ln T, sparse kernels)
through the C ABI: right-hand side against the oracle's definition with
its exact thermodynamics, the Jacobian against the exact plan's, cells
outside the table's range bit for bit the exact path, integration at
rtol 1e-10 against the converged oracle references (the parity bar of the
exact kernels), and the refusals (dense kernels, VJP, adjoint)."""
import os

import numpy as np
import pytest

from test_gpu_parity import cells, gross_scale, parity_excess, to_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12  # largest error of the tables' -dG/RT and dH/RT


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


def _sample(c, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(c["T"].size, n, replace=False))


@pytest.mark.parametrize("key,ncell", [("C1", 64), ("C2", 48), ("C3", 24)])
def test_thermo_rhs_parity(torch, sc, key, ncell):
    """With the tables at 1e-12 the production rates stay within 1e-10 of
    the gross rates of the oracle's exact right-hand side (a relative error
    e in K_c moves a net rate by at most e times its reverse rate)."""
    from oracle import oracle as o_mod
    c = cells(key)
    mech = c["mech"]
    idx = _sample(c, ncell, 10)
    plan = sc.Plan(sc.Mechanism(mech.to_text()), linalg="sparse", thermo_tol=TOL)
    T, p, Y, _ = to_gpu(torch, c, idx)
    fT, fY = plan.rhs(T, p, Y)
    fT, fY = fT.cpu().numpy(), fY.cpu().numpy().T
    o = o_mod.Oracle(mech.to_text())
    worst = 0.0
    for n, i in enumerate(idx):
        f = o.rhs(np.append(c["Y"][i], c["T"][i]), c["p"][i])
        sY, sT = gross_scale(o, mech, c["T"][i], c["p"][i], c["Y"][i], None)
        worst = max(worst, (np.abs(fY[n] - f[:-1]) / (sY + 1e-300)).max(), abs(fT[n] - f[-1]) / (sT + 1e-300))
    assert worst < 1e-10, worst


def test_thermo_jacobian_and_range(torch, sc):
    """The Jacobian with the tables matches the exact plan's to 1e-8 of each
    cell's largest entry; cells whose T is below the table's range are the
    exact path bit for bit (right-hand side and Jacobian)."""
    c = cells("C2")
    idx = _sample(c, 64, 11)
    T, p, Y, _ = to_gpu(torch, c, idx)
    mech = sc.Mechanism(c["mech"].to_text())
    exact = sc.Plan(mech, linalg="sparse")
    tab = sc.Plan(mech, linalg="sparse", thermo_tol=TOL)
    Je, Jt = exact.jacobian(T, p, Y).cpu().numpy(), tab.jacobian(T, p, Y).cpu().numpy()
    scale = np.abs(Je).reshape(len(idx), -1).max(1)[:, None, None]
    assert np.all(np.abs(Jt - Je) <= 1e-8 * scale)
    # a table starting at 1000 K: the colder cells take the exact sums
    lo = sc.Plan(mech, linalg="sparse", thermo_tol=1e-10, thermo_Tmin=1000.0)
    cold = c["T"][idx] < 1000.0
    assert cold.sum() > 5 and (~cold).sum() > 5
    fe, fl = exact.rhs(T, p, Y), lo.rhs(T, p, Y)
    Jl = lo.jacobian(T, p, Y).cpu().numpy()
    ct = torch.tensor(cold, device=T.device)
    assert torch.equal(fe[0][ct], fl[0][ct]) and torch.equal(fe[1][:, ct], fl[1][:, ct])
    assert np.array_equal(Je[cold], Jl[cold])


@pytest.mark.parametrize("key,golden", [("C2", "c2_ref.npz"), ("C3", "c3_ref.npz")])
def test_thermo_integrate_tight_tolerance_parity(torch, sc, key, golden):
    """At rtol 1e-10 / atol 1e-16 with the tables at 1e-12, every stored
    reference cell meets the parity bar."""
    c = cells(key)
    g = np.load(os.path.join(HERE, "golden", golden))
    idx = g["idx"]
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()), rtol=1e-10, atol=1e-16, max_steps=200000, linalg="sparse",
                   thermo_tol=TOL)
    T, p, Y, dt = to_gpu(torch, c, idx)
    r = plan.integrate(T, p, Y, dt)
    assert np.all(r["status"].cpu().numpy() == 0)
    ex = parity_excess(r["T"].cpu().numpy(), r["Y"].cpu().numpy().T, g["T"], g["Y"])
    print(f"{key} interpolated thermo: worst parity excess {ex.max():.3g} over {idx.size} cells")
    assert np.all(ex <= 1.0), (ex.max(), idx[np.argmax(ex)])


def test_thermo_refusals(torch, sc):
    c = cells("C2")
    mech = sc.Mechanism(c["mech"].to_text())
    with pytest.raises(RuntimeError, match="sparse"):
        sc.Plan(mech, linalg="dense", thermo_tol=1e-10)
    with pytest.raises(RuntimeError, match="thermo"):
        sc.Plan(mech, linalg="sparse", thermo_tol=1e-10, thermo_Tmin=500.0, thermo_Tmax=400.0)
    plan = sc.Plan(mech, linalg="sparse", thermo_tol=1e-10)
    idx = _sample(c, 8, 12)
    T, p, Y, dt = to_gpu(torch, c, idx)
    with pytest.raises(RuntimeError, match="exact thermodynamics"):
        plan.vjp(T, p, Y, torch.ones_like(T), torch.zeros_like(Y))
    with pytest.raises(RuntimeError, match="exact thermodynamics"):
        plan.adjoint(T, p, Y, dt, torch.ones_like(T), torch.zeros_like(Y))
