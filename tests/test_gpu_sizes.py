"""Every kernel size variant at its largest mechanism: the kernels are
compiled for 16, 32, 56 and 64 padded state rows, and N + 1 = 16, 32, 56
and 64 (N = 15, 31, 55, 63 species, 63 being the largest supported) fill
them exactly; N = 24 is a ragged case.  For each: right-hand side, Jacobian
and vector-Jacobian product against the oracle's definition and complex-step
derivatives, integration at rtol 1e-10 against the oracle at rtol 1e-11 (the
parity bar), queue and plain launches bit for bit, and the adjoint's
recorded forward equal to the integration bit for bit; and, for the 32-
and 64-row adjoint kernels, fixed-step gradients against central
differences of the CPU map."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (species, reactions, pool fraction, seed): seeded synthetic C/H/O/N mechanisms
SIZES = {15: (15, 60, 0.15, 400), 24: (24, 120, 0.5, 400), 31: (31, 160, 0.5, 400),
         55: (55, 330, 0.15, 400), 63: (63, 400, 0.15, 400)}
# the sparse kernels hold the N + 2 positions of the bordered system in one
# slot per lane up to 64 positions (N = 62 fills them), two beyond (N = 63
# is the smallest two-slot case); N = 14 fills 16 positions
SPARSE_SIZES = {14: (14, 56, 0.15, 401), 62: (62, 390, 0.15, 401)}


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


_MECH = {}


def case(n_species, ncell=12):
    from oracle.oracle import Oracle
    from synth.mechgen import make_mechanism
    if n_species not in _MECH:
        n, r, pf, seed = SIZES.get(n_species) or SPARSE_SIZES[n_species]
        mech = make_mechanism(n, r, r // 10, r // 20, ["C", "H", "O", "N"], seed=seed, pool_frac=pf)
        _MECH[n_species] = (mech, Oracle(mech.to_text()))
    mech, o = _MECH[n_species]
    rng = np.random.default_rng(n_species)
    T = rng.uniform(1000.0, 2000.0, ncell)
    p = 101325.0 * rng.uniform(1.0, 5.0, ncell)
    Y = rng.dirichlet(np.ones(mech.n_species), ncell)
    return mech, o, T, p, Y


def _gpu(torch, T, p, Y, dt=None):
    d = "cuda:0"
    out = [torch.tensor(T, device=d), torch.tensor(p, device=d), torch.tensor(np.ascontiguousarray(Y.T), device=d)]
    if dt is not None:
        out.append(torch.tensor(dt, device=d))
    return out


def _gross(o, mech, T, p, Y):
    kf, kr, q, wdot, aux = o.rates(T, p, Y)
    rho, cp = aux[0], aux[1]
    W = mech.molar_masses()
    C = rho * Y / W
    g = np.zeros(mech.n_species)
    for j, r in enumerate(mech.reactions):
        pf = np.prod([C[k] ** v for k, v in r.reac])
        pr = np.prod([C[k] ** v for k, v in r.prod])
        M = sum(r.eff.get(k, 1.0) * C[k] for k in range(mech.n_species)) if r.kind == "third" else 1.0
        for k, v in r.reac + r.prod:
            g[k] += v * (abs(kf[j] * pf) + abs(kr[j] * pr)) * M
    h = o.thermo(T)[1] * 8.314462618 * T
    return W * g / rho, np.sum(np.abs(h) * g) / (rho * cp)


@pytest.mark.parametrize("ns", sorted(SIZES))
def test_size_rhs_jacobian_vjp(torch, sc, ns):
    mech, o, T, p, Y = case(ns)
    plan = sc.Plan(sc.Mechanism(mech.to_text()))
    assert plan.mech.info["n_padded"] in (16, 32, 56, 64)
    Tg, pg, Yg = _gpu(torch, T, p, Y)
    fT, fY = plan.rhs(Tg, pg, Yg)
    J = plan.jacobian(Tg, pg, Yg).cpu().numpy()
    rng = np.random.default_rng(1)
    w = rng.normal(size=(T.size, mech.n_species + 1))
    gT, gY = plan.vjp(Tg, pg, Yg, torch.tensor(w[:, -1], device="cuda:0"),
                      torch.tensor(np.ascontiguousarray(w[:, :-1].T), device="cuda:0"))
    fT, fY, gT, gY = fT.cpu().numpy(), fY.cpu().numpy().T, gT.cpu().numpy(), gY.cpu().numpy().T
    for c in range(T.size):
        y = np.append(Y[c], T[c])
        f = o.rhs(y, p[c])
        sY, sT = _gross(o, mech, T[c], p[c], Y[c])
        assert (np.abs(fY[c] - f[:-1]) / (sY + 1e-300)).max() < 1e-12
        assert abs(fT[c] - f[-1]) / (sT + 1e-300) < 1e-12
        Jc = o.jac_cs(y, p[c])
        row = np.abs(Jc).max(1, keepdims=True) + 1e-300
        assert (np.abs(J[c] - Jc) / (1e-8 * np.abs(Jc) + 1e-12 * row)).max() <= 1.0, (ns, c)
        g = Jc.T @ w[c]
        scale = np.abs(Jc.T) @ np.abs(w[c]) + 1e-300
        got = np.append(gY[c], gT[c])
        assert (np.abs(got - g) / (1e-8 * np.abs(g) + 1e-12 * scale)).max() <= 1.0, (ns, c)


@pytest.mark.parametrize("ns", sorted(SIZES))
def test_size_integration_parity_and_launches(torch, sc, ns):
    mech, o, T, p, Y = case(ns)
    dt = np.full(T.size, 1e-6)
    ref = o.integrate(T, p, Y, dt, rtol=1e-11, atol=1e-17, max_steps=200000)
    assert np.all(ref["status"] == 0)
    m = sc.Mechanism(mech.to_text())
    Tg, pg, Yg, dtg = _gpu(torch, T, p, Y, dt)
    r = sc.Plan(m, rtol=1e-10, atol=1e-16, max_steps=200000).integrate(Tg, pg, Yg, dtg)
    assert np.all(r["status"].cpu().numpy() == 0)
    T1, Y1 = r["T"].cpu().numpy(), r["Y"].cpu().numpy().T
    assert np.all(np.abs(T1 - ref["T"]) <= 1e-6 * ref["T"]), ns
    big = np.abs(ref["Y"]) > 1e-8
    assert np.all(np.abs(Y1 - ref["Y"])[big] <= 1e-6 * np.abs(ref["Y"])[big]), ns
    assert np.all(np.abs(Y1 - ref["Y"])[~big] <= 1e-12), ns
    # production tolerance: queue vs plain launch, and the adjoint's recorded forward
    a = sc.Plan(m).integrate(Tg, pg, Yg, dtg)
    q = sc.Plan(m, mode="persistent", order="cost")
    b = q.integrate(Tg, pg, Yg, dtg)
    b = q.integrate(Tg, pg, Yg, dtg, out=b)
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert torch.equal(a[k], b[k]), (ns, k)
    adj = sc.Plan(m).adjoint(Tg, pg, Yg, dtg, torch.ones_like(Tg), torch.zeros_like(Yg), forward_out=True)
    assert np.all(adj["status"].cpu().numpy() == 0)
    assert torch.equal(adj["T"], a["T"]) and torch.equal(adj["Y"], a["Y"]), ns
    assert bool(torch.isfinite(adj["g_dlnA"]).all())


# interval (and, for 63 species, a 1000 K start) where six fixed steps give
# a map smooth enough that its central differences agree with themselves at
# half the step to 1e-5 or better
@pytest.mark.parametrize("ns,T0,dt", [(31, None, 1e-7), (63, 1000.0, 3e-9)])
def test_size_adjoint_fixed_steps(torch, sc, ns, T0, dt):
    """The 32- and 64-row adjoint kernels: gradients of a random weighting of
    (T1, Y1) with respect to (T0, Y0) and to four random directions in
    log A, through six fixed steps, against central differences of the CPU
    fixed-step map (tests/frozen_map.py), which the device map also
    matches."""
    from frozen_map import fd_gradient, fixed_map
    mech, o, T, p, Y = case(ns, ncell=2)
    if T0 is not None:
        T = np.full(T.size, T0)
    N, R = mech.n_species, mech.n_reactions
    rng = np.random.default_rng(7)
    dlnA = rng.normal(size=R) * 0.1
    dt = np.full(T.size, dt)
    nsteps = 6
    plan = sc.Plan(sc.Mechanism(mech.to_text()), fixed_step=True, max_steps=1000)
    Tg, pg, Yg, dtg = _gpu(torch, T, p, Y, dt)
    h = dtg / nsteps
    wY = rng.normal(size=(T.size, N)) * 1e2
    wT = rng.normal(size=T.size) * 1e-2
    out = plan.integrate(Tg, pg, Yg, dtg, dlnA=dlnA, h=h)
    r = plan.adjoint(Tg, pg, Yg, dtg, torch.tensor(wT, device="cuda:0"),
                     torch.tensor(np.ascontiguousarray(wY.T), device="cuda:0"), dlnA=dlnA, h=h,
                     per_cell=True, forward_out=True)
    assert torch.equal(r["T"], out["T"]) and torch.equal(r["Y"], out["Y"])
    assert np.all(r["status"].cpu().numpy() == 0)
    gT0, gY0 = r["gT0"].cpu().numpy(), r["gY0"].cpu().numpy().T
    gc = r["g_dlnA_cell"].cpu().numpy()
    T1, Y1 = out["T"].cpu().numpy(), out["Y"].cpu().numpy().T
    dirs = rng.normal(size=(4, R))
    for c in range(T.size):
        y0 = np.append(Y[c], T[c])
        hn = dt[c] / nsteps
        y1 = fixed_map(o, y0, p[c], dt[c], hn, dlnA)
        scale = np.append(np.maximum(np.abs(y1[:-1]), 1e-8), abs(y1[-1]))
        assert np.max(np.abs(np.append(Y1[c], T1[c]) - y1) / scale) < 1e-8, (ns, c)
        w = np.append(wY[c], wT[c])
        g_fd, gp_fd = fd_gradient(o, y0, p[c], dt[c], hn, w, dlnA, dirs)
        ref = np.append(g_fd, gp_fd)
        got = np.append(np.append(gY0[c], gT0[c]), dirs @ gc[:, c])
        den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        err = np.max(np.abs(got - ref) / den)
        print(f"N={ns} cell {c}: adjoint vs central differences {err:.3g}")
        assert err < 1e-4, (ns, c, err)


@pytest.mark.parametrize("ns", [14, 15, 62, 63])
def test_size_sparse_parity(torch, sc, ns):
    """The sparse linear algebra at the edges of its one- and two-slot
    layouts: Jacobian (recovered from the bordered matrix) against the
    complex-step derivative, one linear solve against a dense solve of the
    complex-step matrix (normwise residual; the solution where the matrix is
    well conditioned), integration at rtol 1e-10 against the oracle at rtol
    1e-11 (the parity bar), and queue and plain launches bit for bit."""
    mech, o, T, p, Y = case(ns)
    m = sc.Mechanism(mech.to_text())
    plan = sc.Plan(m, linalg="sparse")
    Tg, pg, Yg = _gpu(torch, T, p, Y)
    J = plan.jacobian(Tg, pg, Yg).cpu().numpy()
    n1 = mech.n_species + 1
    rng = np.random.default_rng(ns)
    hg = np.full(T.size, 1e-7)
    b = rng.normal(size=(T.size, n1))
    x = plan.linsolve(Tg, pg, Yg, torch.tensor(hg, device="cuda:0"),
                      torch.tensor(b, device="cuda:0")).cpu().numpy()
    for c in range(T.size):
        y = np.append(Y[c], T[c])
        Jc = o.jac_cs(y, p[c])
        row = np.abs(Jc).max(1, keepdims=True) + 1e-300
        assert (np.abs(J[c] - Jc) / (1e-8 * np.abs(Jc) + 1e-12 * row)).max() <= 1.0, (ns, c)
        M = np.eye(n1) / hg[c] - Jc
        ref = np.linalg.solve(M, b[c])
        res = np.abs(M @ x[c] - b[c]).max() / (np.abs(M).max() * np.abs(x[c]).max() + np.abs(b[c]).max())
        # (normwise backward error of the unpivoted sparse LU; these random
        # states make the matrix nearly singular, hence 1e-11)
        assert res < 1e-11, (ns, c, res)
        # the solution itself only where the matrix's conditioning bounds its
        # error (these random states give condition numbers up to 1e18, where
        # any two backward-stable solves may differ completely)
        if np.linalg.cond(M) < 1e8:
            assert np.allclose(x[c], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max()), (ns, c)
    dt = np.full(T.size, 1e-6)
    ref = o.integrate(T, p, Y, dt, rtol=1e-11, atol=1e-17, max_steps=200000)
    assert np.all(ref["status"] == 0)
    Tg, pg, Yg, dtg = _gpu(torch, T, p, Y, dt)
    # a first step of dt / 1000 (the caller's carried step): one of these
    # random 14-species states is so stiff that a first attempt over the
    # whole dt and four shorter retries all overflow, in the dense and the
    # sparse kernels alike, and the controller gives the cell up
    h0 = dtg * 1e-3
    r = sc.Plan(m, rtol=1e-10, atol=1e-16, max_steps=200000, linalg="sparse").integrate(Tg, pg, Yg, dtg, h=h0)
    assert np.all(r["status"].cpu().numpy() == 0)
    T1, Y1 = r["T"].cpu().numpy(), r["Y"].cpu().numpy().T
    assert np.all(np.abs(T1 - ref["T"]) <= 1e-6 * ref["T"]), ns
    big = np.abs(ref["Y"]) > 1e-8
    assert np.all(np.abs(Y1 - ref["Y"])[big] <= 1e-6 * np.abs(ref["Y"])[big]), ns
    assert np.all(np.abs(Y1 - ref["Y"])[~big] <= 1e-12), ns
    a = sc.Plan(m, linalg="sparse").integrate(Tg, pg, Yg, dtg)
    q = sc.Plan(m, mode="persistent", order="cost", linalg="sparse")
    bq = q.integrate(Tg, pg, Yg, dtg)
    bq = q.integrate(Tg, pg, Yg, dtg, out=bq)
    for k in ("T", "Y", "status", "n_acc", "n_rej"):
        assert torch.equal(a[k], bq[k]), (ns, k)
