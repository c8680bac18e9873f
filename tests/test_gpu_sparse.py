"""The sparse linear algebra kernels (the bordered system in minimum-degree
order, factorised and solved by the mechanism compiler's static level
schedule) through the C ABI: right-hand side, Jacobian and linear solve
against the oracle's definition, complex-step Jacobian and dense solve, for
the 9-, 53- and 110-species mechanisms (the last needs two state components
per lane); integration at rtol 1e-10 against the converged oracle references
(parity bar: T and Y > 1e-8 relative 1e-6, Y below absolute 1e-12); launch
modes bit for bit."""
import os

import numpy as np
import pytest

from test_gpu_parity import cells, gross_scale, parity_excess, to_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
KEYS = [("C1", 64), ("C2", 48), ("C3", 24)]


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


@pytest.fixture(scope="module")
def oracle_mod():
    from oracle import oracle as o
    return o


def _sample(c, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(c["T"].size, n, replace=False))


@pytest.mark.parametrize("key,ncell", KEYS)
def test_sparse_rhs_parity(torch, sc, oracle_mod, key, ncell):
    c = cells(key)
    mech = c["mech"]
    idx = _sample(c, ncell, 0)
    plan = sc.Plan(sc.Mechanism(mech.to_text()), linalg="sparse")
    T, p, Y, _ = to_gpu(torch, c, idx)
    rng = np.random.default_rng(1)
    dlnA = rng.normal(size=mech.n_reactions) * 0.3
    fT, fY = plan.rhs(T, p, Y, dlnA=dlnA)
    fT, fY = fT.cpu().numpy(), fY.cpu().numpy().T
    o = oracle_mod.Oracle(mech.to_text())
    worst = 0.0
    for n, i in enumerate(idx):
        f = o.rhs(np.append(c["Y"][i], c["T"][i]), c["p"][i], dlnA=dlnA)
        sY, sT = gross_scale(o, mech, c["T"][i], c["p"][i], c["Y"][i], dlnA)
        worst = max(worst, (np.abs(fY[n] - f[:-1]) / (sY + 1e-300)).max(), abs(fT[n] - f[-1]) / (sT + 1e-300))
    assert worst < 1e-12, worst


@pytest.mark.parametrize("key,ncell", KEYS)
@pytest.mark.parametrize("reactor", ["const_p", "const_v"])
def test_sparse_jacobian_parity(torch, sc, oracle_mod, key, ncell, reactor):
    """The Jacobian recovered from the bordered matrix (sigma eliminated,
    scaling undone) against the oracle's complex-step J, both reactors."""
    c = cells(key)
    mech = c["mech"]
    idx = _sample(c, ncell, 2)
    T, p, Y, _ = to_gpu(torch, c, idx)
    pa = c["p"][idx]
    if reactor == "const_v":
        W = mech.molar_masses()
        pa = c["p"][idx] / (8.314462618 * c["T"][idx] * (c["Y"][idx] / W).sum(1))
        p = torch.tensor(pa, device="cuda:0")
    plan = sc.Plan(sc.Mechanism(mech.to_text()), linalg="sparse", reactor=reactor)
    rng = np.random.default_rng(3)
    dlnA = rng.normal(size=mech.n_reactions) * 0.3
    J = plan.jacobian(T, p, Y, dlnA=dlnA).cpu().numpy()
    o = oracle_mod.Oracle(mech.to_text())
    worst = 0.0
    for n, i in enumerate(idx):
        Jc = o.jac_cs(np.append(c["Y"][i], c["T"][i]), pa[n], dlnA=dlnA, constv=reactor == "const_v")
        row = np.abs(Jc).max(1, keepdims=True) + 1e-300
        # (rows of trace species in cold cells can be 1e-60 or less: below
        # 1e-20 of the matrix's largest entry an underflowed product is not
        # an error of the Jacobian)
        floor = 1e-20 * np.abs(Jc).max()
        worst = max(worst, (np.abs(J[n] - Jc) / (1e-8 * np.abs(Jc) + 1e-12 * row + floor)).max())
    assert worst <= 1.0, worst


@pytest.mark.parametrize("key,ncell", KEYS)
def test_sparse_linsolve_parity(torch, sc, oracle_mod, key, ncell):
    """(I/hg - J) x = b through the bordered sparse LU (no pivoting, static
    minimum-degree order) against a dense solve of the complex-step matrix:
    residual and solution."""
    c = cells(key)
    mech = c["mech"]
    idx = _sample(c, ncell, 4)
    plan = sc.Plan(sc.Mechanism(mech.to_text()), linalg="sparse")
    T, p, Y, _ = to_gpu(torch, c, idx)
    n, m = idx.size, mech.n_species + 1
    rng = np.random.default_rng(5)
    b = rng.normal(size=(n, m))
    o = oracle_mod.Oracle(mech.to_text())
    for hg in (1e-9, 1e-6, 1e-3):
        x = plan.linsolve(T, p, Y, np.full(n, hg), b).cpu().numpy()
        for k, i in enumerate(idx):
            A = np.eye(m) / hg - o.jac_cs(np.append(c["Y"][i], c["T"][i]), c["p"][i])
            ref = np.linalg.solve(A, b[k])
            res = np.abs(A @ x[k] - b[k]).max() / (np.abs(A).max() * np.abs(x[k]).max() + np.abs(b[k]).max())
            assert res < 1e-12, (hg, i, res)
            assert np.allclose(x[k], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max()), (hg, i)


@pytest.mark.parametrize("key,golden", [("C1", "c1_ref.npz"), ("C2", "c2_ref.npz"), ("C3", "c3_ref.npz")])
def test_sparse_integrate_tight_tolerance_parity(torch, sc, key, golden):
    """Gate G1 for the sparse kernels: at rtol 1e-10 / atol 1e-16 every
    stored reference cell meets the parity bar (the 110-species C3 cells
    have per-cell dt from 1e-7 to 1e-3 s)."""
    c = cells(key)
    g = np.load(os.path.join(HERE, "golden", golden))
    idx = g["idx"]
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()), rtol=1e-10, atol=1e-16, max_steps=200000, linalg="sparse")
    T, p, Y, dt = to_gpu(torch, c, idx)
    r = plan.integrate(T, p, Y, dt)
    st = r["status"].cpu().numpy()
    assert np.all(st == 0), np.bincount(st)
    ex = parity_excess(r["T"].cpu().numpy(), r["Y"].cpu().numpy().T, g["T"], g["Y"])
    print(f"{key} sparse: worst parity excess {ex.max():.3g} over {idx.size} cells (<= 1 passes)")
    assert np.all(ex <= 1.0), (ex.max(), idx[np.argmax(ex)])


@pytest.mark.parametrize("key", ["C2", "C3"])
def test_sparse_launch_modes_bitwise(torch, sc, key):
    """Plain, static and queue launches of the sparse kernels give the same
    bits; so does the allocation-free entry point."""
    c = cells(key)
    idx = _sample(c, 2048, 6)
    T, p, Y, dt = to_gpu(torch, c, idx)
    mech = sc.Mechanism(c["mech"].to_text())
    a = sc.Plan(mech, linalg="sparse").integrate(T, p, Y, dt)
    assert np.all(a["status"].cpu().numpy() == 0)
    for cfg in (dict(mode="static"), dict(mode="persistent", order="cost")):
        q = sc.Plan(mech, linalg="sparse", **cfg)
        b = q.integrate(T, p, Y, dt)
        b = q.integrate(T, p, Y, dt, out=b)
        for k in ("T", "Y", "status", "n_acc", "n_rej"):
            assert torch.equal(a[k], b[k]), (cfg, k)
    q = sc.Plan(mech, linalg="sparse", mode="persistent", order="dt")
    b = q.integrate_noalloc(T, p, Y, dt)
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert torch.equal(a[k], b[k]), ("noalloc", k)


def test_sparse_matches_dense_and_conserves(torch, sc):
    """On the 53-species workload the sparse and dense kernels integrate the
    same ODE: at rtol 1e-10 they agree to the parity bar, and both keep the
    sum of mass fractions and the element totals to roundoff."""
    c = cells("C2")
    idx = _sample(c, 1024, 7)
    T, p, Y, dt = to_gpu(torch, c, idx)
    mech = sc.Mechanism(c["mech"].to_text())
    s = sc.Plan(mech, rtol=1e-10, atol=1e-16, linalg="sparse").integrate(T, p, Y, dt)
    d = sc.Plan(mech, rtol=1e-10, atol=1e-16, linalg="dense").integrate(T, p, Y, dt)
    ex = parity_excess(s["T"].cpu().numpy(), s["Y"].cpu().numpy().T, d["T"].cpu().numpy(),
                       d["Y"].cpu().numpy().T)
    assert ex.max() <= 1.0, ex.max()
    Y0, Y1 = c["Y"][idx], s["Y"].cpu().numpy().T
    assert np.abs(Y1.sum(1) - Y0.sum(1)).max() < 1e-13
    A = c["mech"].element_matrix() / c["mech"].molar_masses()[None, :]
    assert np.abs(Y1 @ A.T - Y0 @ A.T).max() < 1e-12 * np.abs(Y0 @ A.T).max()


# a 30-species mechanism: N + 2 = 32 positions, so two cells fit a wave
def _mech30():
    from synth.mechgen import make_mechanism
    return make_mechanism(30, 150, 15, 7, ["C", "H", "O", "N"], seed=402, pool_frac=0.3)


@pytest.mark.parametrize("key", ["C1", "m30"])
def test_cells_per_wave(torch, sc, oracle_mod, key):
    """Several cells per wave (4 for the 9-species mechanism, 2 for 30
    species) against one cell per wave: fixed steps agree to rounding (the
    per-cell arithmetic differs only in the order of its sums); at rtol
    1e-10 every cell meets the parity bar against the oracle at rtol 1e-11;
    plain, static and queue launches agree bit for bit on a batch that does
    not fill its last wave; an invalid input or a zero dt affects only its
    own cell."""
    if key == "C1":
        c = cells("C1")
        mech_s, n_max = c["mech"], 4
        idx = _sample(c, 61, 9)
        T0, p0, Y0, dt0 = c["T"][idx], c["p"][idx], c["Y"][idx], c["dt"][idx]
    else:
        mech_s, n_max = _mech30(), 2
        rng = np.random.default_rng(30)
        T0, p0 = rng.uniform(1000.0, 2000.0, 37), 101325.0 * rng.uniform(1.0, 5.0, 37)
        Y0, dt0 = rng.dirichlet(np.ones(mech_s.n_species), 37), np.full(37, 1e-6)
    d = "cuda:0"
    T, p = torch.tensor(T0, device=d), torch.tensor(p0, device=d)
    Y, dt = torch.tensor(np.ascontiguousarray(Y0.T), device=d), torch.tensor(dt0, device=d)
    mech = sc.Mechanism(mech_s.to_text())
    one = sc.Plan(mech, linalg="sparse", cells_per_wave=1, fixed_step=True)
    many = sc.Plan(mech, linalg="sparse", cells_per_wave=n_max, fixed_step=True)
    # five fixed steps over an interval short enough for them to be stable
    # (the cells need hundreds of steps over their own dt)
    dtf = torch.full_like(dt, 1e-10)
    h = dtf / 5
    a = one.integrate(T, p, Y, dtf, h=h)
    b = many.integrate(T, p, Y, dtf, h=h)
    assert torch.equal(a["status"], b["status"]) and torch.equal(a["n_acc"], b["n_acc"])
    ya = np.vstack([a["Y"].cpu().numpy(), a["T"].cpu().numpy()[None]])
    yb = np.vstack([b["Y"].cpu().numpy(), b["T"].cpu().numpy()[None]])
    scale = np.maximum(np.abs(ya), 1e-10 * np.abs(ya).max(0, keepdims=True))
    assert np.max(np.abs(ya - yb) / scale) < 1e-11
    # parity at a tight tolerance against the oracle
    o = oracle_mod.Oracle(mech_s.to_text())
    ref = o.integrate(T0, p0, Y0, dt0, rtol=1e-11, atol=1e-17, max_steps=200000)
    r = sc.Plan(mech, rtol=1e-10, atol=1e-16, max_steps=200000, linalg="sparse",
                cells_per_wave=n_max).integrate(T, p, Y, dt)
    assert np.all(r["status"].cpu().numpy() == 0)
    ex = parity_excess(r["T"].cpu().numpy(), r["Y"].cpu().numpy().T, ref["T"], ref["Y"])
    assert np.all(ex <= 1.0), ex.max()
    # launches, with a bad cell and a zero-dt cell among good ones
    T2, dt2 = T.clone(), dt.clone()
    T2[3] = float("nan")
    dt2[6] = 0.0
    outs = []
    for cfg in (dict(mode="plain"), dict(mode="static"), dict(mode="persistent", order="cost"),
                dict(mode="persistent", tile=2)):
        q = sc.Plan(mech, linalg="sparse", cells_per_wave=n_max, **cfg)
        o2 = q.integrate(T2, p, Y, dt2)
        if cfg.get("order") == "cost":
            o2 = q.integrate(T2, p, Y, dt2, out=o2)
        outs.append(o2)
    st = outs[0]["status"].cpu().numpy()
    assert st[3] == 4 and st[6] == 0 and np.all(np.delete(st, 3) == 0)
    assert torch.equal(outs[0]["Y"][:, 6], Y[:, 6]) and outs[0]["n_acc"][6].item() == 0
    keep = torch.arange(T.numel(), device=d) != 3  # the NaN cell's outputs are not compared
    for o2 in outs[1:]:
        for k in ("T", "status", "n_acc", "n_rej"):
            assert torch.equal(o2[k][keep], outs[0][k][keep]), k
        assert torch.equal(o2["Y"][:, keep], outs[0]["Y"][:, keep])
        assert o2["status"][3].item() == 4


def test_cells_per_wave_arguments(sc):
    from synth.mechgen import standard_mechanism
    m1 = sc.Mechanism(standard_mechanism("h2_9").to_text())
    m53 = sc.Mechanism(standard_mechanism("chon_53").to_text())
    for mech, kw in ((m53, dict(linalg="sparse", cells_per_wave=2)), (m1, dict(linalg="sparse", cells_per_wave=3)),
                     (m1, dict(linalg="dense", cells_per_wave=4))):
        with pytest.raises(RuntimeError, match="cells_per_wave"):
            sc.Plan(mech, **kw)
    sc.Plan(m1, linalg="sparse", cells_per_wave=4)
    sc.Plan(m53, linalg="sparse", cells_per_wave=1)
