"""Parity of the device's vector-Jacobian product and discrete adjoint.

* sc_vjp against the oracle's complex-step Jacobian and complex-step
  derivative with respect to the rate multipliers (transposed, applied to a
  random weight);
* sc_adjoint with the step sequence fixed, against central differences of
  the same fixed-step Rosenbrock map evaluated on the CPU with the oracle's
  right-hand side (tests/frozen_map.py), including a run long enough for
  checkpoint thinning and segment recomputation;
* sc_adjoint with error control at a tight tolerance, against the oracle's
  forward sensitivities (tests/golden/c4_sens.npz), per entry
  |g - g_ref| <= 1e-4 max(|g_ref|, 1e-3 max|g_ref|);
* the isomerisation A <=> B, whose sensitivities have a closed form;
* the recorded forward equals sc_integrate bit for bit; schedule and
  workspace budget do not change a bit; failure and edge cases.
"""
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


@pytest.fixture(scope="module")
def oracle_mod():
    from oracle import oracle as o
    return o


_CELLS = {}


def cells(key, n=None):
    from synth.cells import make_cells
    k = (key, n)
    if k not in _CELLS:
        _CELLS[k] = make_cells(key, n=n)
    return _CELLS[k]


def dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


def state_gpu(torch, c, idx):
    return (dev(torch, c["T"][idx]), dev(torch, c["p"][idx]), dev(torch, c["Y"][idx].T),
            dev(torch, c["dt"][idx]))


def gross_param_scale(o, mech, T, p, Y, w, dlnA):
    """Per reaction: (|forward| + |reverse| rate) times the absolute weight of
    its production terms, the size of the terms whose roundoff q_j carries
    (near equilibrium q_j is a small difference of the two)."""
    kf, kr, q, wdot, aux = o.rates(T, p, Y, dlnA)
    rho, cp = aux[0], aux[1]
    W = mech.molar_masses()
    C = rho * Y / W
    hRT = o.thermo(T)[1]
    RT = 8.314462618 * T
    out = np.zeros(mech.n_reactions)
    for j, r in enumerate(mech.reactions):
        pf = np.prod([C[k] ** v for k, v in r.reac])
        pr = np.prod([C[k] ** v for k, v in r.prod])
        M = 1.0
        if r.kind == "third":
            M = sum(r.eff.get(k, 1.0) * C[k] for k in range(mech.n_species))
        gross = (abs(kf[j] * pf) + abs(kr[j] * pr)) * M
        sig = sum(v * (W[k] * abs(w[k]) + abs(w[-1]) / cp * abs(hRT[k]) * RT) for k, v in r.reac + r.prod)
        out[j] = gross * sig / rho
    return out


@pytest.mark.parametrize("key,ncell", [("C1", 64), ("C2", 48)])
def test_vjp_parity(torch, sc, oracle_mod, key, ncell):
    """J^T w and (df/d dlnA)^T w against the oracle's complex-step derivatives."""
    c = cells(key)
    mech = c["mech"]
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(c["T"].size, ncell, replace=False))
    plan = sc.Plan(sc.Mechanism(mech.to_text()))
    T, p, Y, _ = state_gpu(torch, c, idx)
    N, R = mech.n_species, mech.n_reactions
    dlnA = rng.normal(size=R) * 0.3
    # weights of both signs and of the scales of the adjoint of (Y, T)
    wY = rng.normal(size=(ncell, N)) * 10.0 ** rng.uniform(-3, 3, size=(ncell, N))
    wT = rng.normal(size=ncell) * 1e-3
    gT, gY, gc = plan.vjp(T, p, Y, dev(torch, wT), dev(torch, wY.T), dlnA=dlnA, per_cell=True)
    gT, gY, gc = gT.cpu().numpy(), gY.cpu().numpy().T, gc.cpu().numpy()
    o = oracle_mod.Oracle(mech.to_text())
    worst_y = worst_p = 0.0
    for n, i in enumerate(idx):
        y = np.append(c["Y"][i], c["T"][i])
        w = np.append(wY[n], wT[n])
        Jc = o.jac_cs(y, c["p"][i], dlnA=dlnA)
        g_ref = Jc.T @ w
        row = np.abs(Jc).max(1) + 1e-300
        tol = (1e-8 * np.abs(Jc) + 1e-12 * row[:, None]).T @ np.abs(w)
        g = np.append(gY[n], gT[n])
        worst_y = max(worst_y, np.max(np.abs(g - g_ref) / tol))
        Fc = o.dfdp_cs(y, c["p"][i], dlnA=dlnA)
        gp_ref = Fc.T @ w
        tolp = 1e-8 * (np.abs(Fc).T @ np.abs(w)) + 1e-12 * gross_param_scale(
            o, mech, c["T"][i], c["p"][i], c["Y"][i], w, dlnA) + 1e-300
        worst_p = max(worst_p, np.max(np.abs(gc[:, n] - gp_ref) / tolp))
    assert worst_y <= 1.0, worst_y
    assert worst_p <= 1.0, worst_p


def _fixed_case(torch, sc, oracle_mod, key, idx, nsteps, dt_scale, npar=6, rel=1e-5):
    """Adjoint of the fixed-step map over dt_scale * dt vs central differences
    on the CPU (the interval is shortened where the cells' rates would make
    a handful of fixed steps meaningless)."""
    from frozen_map import fd_gradient, fixed_map
    c = cells(key)
    mech = c["mech"]
    N, R = mech.n_species, mech.n_reactions
    rng = np.random.default_rng(5)
    dlnA = rng.normal(size=R) * 0.1
    plan = sc.Plan(sc.Mechanism(mech.to_text()), fixed_step=True, max_steps=max(1000, 2 * nsteps))
    T, p, Y, dt = state_gpu(torch, c, idx)
    dt = dt * dt_scale
    dtn = c["dt"][idx] * dt_scale
    h = dt / nsteps
    wY = rng.normal(size=(idx.size, N)) * 1e2
    wT = rng.normal(size=idx.size) * 1e-2
    out = plan.integrate(T, p, Y, dt, dlnA=dlnA, h=h)
    r = plan.adjoint(T, p, Y, dt, dev(torch, wT), dev(torch, wY.T), dlnA=dlnA, h=h, per_cell=True,
                     forward_out=True)
    assert torch.equal(r["T"], out["T"]) and torch.equal(r["Y"], out["Y"])
    assert np.all(r["status"].cpu().numpy() == 0)
    assert np.all(r["n_acc"].cpu().numpy() == out["n_acc"].cpu().numpy())
    gT0, gY0 = r["gT0"].cpu().numpy(), r["gY0"].cpu().numpy().T
    gc = r["g_dlnA_cell"].cpu().numpy()
    T1, Y1 = out["T"].cpu().numpy(), out["Y"].cpu().numpy().T
    o = oracle_mod.Oracle(mech.to_text())
    dirs = rng.normal(size=(npar, R))
    worst_map = worst_g = 0.0
    for n, i in enumerate(idx):
        y0 = np.append(c["Y"][i], c["T"][i])
        hn = dtn[n] / nsteps
        y1 = fixed_map(o, y0, c["p"][i], dtn[n], hn, dlnA)
        y1_dev = np.append(Y1[n], T1[n])
        scale = np.append(np.maximum(np.abs(y1[:-1]), 1e-8), abs(y1[-1]))
        worst_map = max(worst_map, np.max(np.abs(y1_dev - y1) / scale))
        w = np.append(wY[n], wT[n])
        g_fd, gp_fd = fd_gradient(o, y0, c["p"][i], dtn[n], hn, w, dlnA, dirs)
        g = np.append(gY0[n], gT0[n])
        gp = dirs @ gc[:, n]
        ref = np.append(g_fd, gp_fd)
        got = np.append(g, gp)
        den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        worst_g = max(worst_g, np.max(np.abs(got - ref) / den))
    print(f"{key} fixed {nsteps} steps: map {worst_map:.3g}, gradient {worst_g:.3g}")
    assert worst_map < 1e-8, worst_map
    assert worst_g < rel, worst_g


def test_adjoint_fixed_steps_h2(torch, sc, oracle_mod):
    _fixed_case(torch, sc, oracle_mod, "C1", np.array([3, 100, 517, 900]), 8, 1e-2)


def test_adjoint_fixed_steps_chon53(torch, sc, oracle_mod):
    c = cells("C2")
    cls = c["cls"]
    idx = np.array([np.nonzero(cls == k)[0][0] for k in (0, 1, 2)] + [np.nonzero(cls == 1)[0][5]])
    # trace species of hot equilibrated cells make this map strongly curved:
    # the central differences themselves carry ~1e-5 there, so this case
    # uses the gradient bar (1e-4) rather than 1e-5
    _fixed_case(torch, sc, oracle_mod, "C2", idx, 6, 0.1, npar=4, rel=1e-4)


def test_adjoint_fixed_steps_stratified_c4(torch, sc):
    """66 cells of the gradient workload (22 per class), six fixed steps
    over dt/10: the device map equals the CPU map to 1e-8 and the discrete
    adjoint (all 54 initial-state components and four rate-multiplier
    directions) equals the stored central differences of that map
    (tests/golden/c4_fd.npz) to 1e-4 relative, floored at 1e-3 of the
    largest entry (the differences' own noise reaches ~1e-5 on the trace
    species of hot equilibrated cells)."""
    gz = np.load(os.path.join(HERE, "golden", "c4_fd.npz"))
    # cells with a converged central-difference reference: the differences at
    # the stored steps and at half of them agree to 1e-5 (floored as below)
    full = np.concatenate([gz["g"], gz["gp"]], 1)
    half = np.concatenate([gz["g_half"], gz["gp_half"]], 1)
    with np.errstate(invalid="ignore"):
        dref = np.maximum(np.abs(full), 1e-3 * np.abs(full).max(1, keepdims=True))
        ok = np.isfinite(full).all(1) & ((np.abs(full - half) / dref).max(1) <= 1e-5)
    print(f"{ok.sum()} of {ok.size} cells have converged central differences")
    assert ok.sum() >= 40, ok.sum()  # 44 of the stored 66 (the rest: stiff near-ignition cells)
    g = {k: (gz[k][ok] if gz[k].ndim and gz[k].shape[0] == ok.size else gz[k]) for k in gz.files}
    c = cells("C4")
    mech = c["mech"]
    idx = g["idx"]
    nsteps = int(g["nsteps"])
    plan = sc.Plan(sc.Mechanism(mech.to_text()), fixed_step=True, max_steps=1000)
    T, p, Y, _ = state_gpu(torch, c, idx)
    dt = dev(torch, g["dt"])
    h = dt / nsteps
    dlnA = g["dlnA"]
    out = plan.integrate(T, p, Y, dt, dlnA=dlnA, h=h)
    r = plan.adjoint(T, p, Y, dt, dev(torch, g["wT"]), dev(torch, g["wY"].T), dlnA=dlnA, h=h, per_cell=True)
    assert np.all(r["status"].cpu().numpy() == 0) and np.all(out["status"].cpu().numpy() == 0)
    y1 = np.concatenate([out["Y"].cpu().numpy().T, out["T"].cpu().numpy()[:, None]], 1)
    scale = np.concatenate([np.maximum(np.abs(g["y1"][:, :-1]), 1e-8), np.abs(g["y1"][:, -1:])], 1)
    worst_map = np.max(np.abs(y1 - g["y1"]) / scale)
    got = np.concatenate([r["gY0"].cpu().numpy().T, r["gT0"].cpu().numpy()[:, None],
                          (g["dirs"] @ r["g_dlnA_cell"].cpu().numpy()).T], 1)
    ref = np.concatenate([g["g"], g["gp"]], 1)
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max(1, keepdims=True))
    err = (np.abs(got - ref) / den).max(1)
    for k in range(3):
        print(f"class {k}: worst gradient error {err[g['cls'] == k].max():.3g}")
    print(f"map {worst_map:.3g}, gradient {err.max():.3g} over {idx.size} cells")
    assert worst_map < 1e-8, worst_map
    assert err.max() < 1e-4, (err.max(), idx[np.argmax(err)])


def test_adjoint_dot_product_linear(torch, sc):
    """Dot-product test on a problem whose fixed-step map is exactly linear
    in the mass fractions (the isomerisation A <=> B: equal molar masses and
    enthalpies keep rho and T constant): for a perturbation dY of the
    initial mass fractions (between two valid states), <lambda_N,
    Y_N(Y0 + dY) - Y_N(Y0)> equals <lambda_0, dY> with lambda_0 the adjoint
    of lambda_N, to roundoff."""
    from synth.mechgen import isomer_mechanism
    mech = isomer_mechanism(log10A=9.0, b=0.0, Ea=40e3, ds_R=0.7)
    plan = sc.Plan(sc.Mechanism(mech.to_text()), fixed_step=True, max_steps=1000)
    rng = np.random.default_rng(9)
    n = 32
    T = np.full(n, 1000.0)
    p = np.full(n, 101325.0)
    Y0 = rng.dirichlet([1.0, 1.0], n)
    # a second valid state as the perturbation's end point: the map is linear,
    # so the perturbation may be large, which keeps the difference of the two
    # forward results clear of their cancellation (a 1e-3 perturbation loses
    # three digits of it)
    dY = rng.dirichlet([1.0, 1.0], n) - Y0
    # (k_f + k_r) dt = 2.4: a perturbation of the composition has partly
    # relaxed (a longer dt would leave only the equilibrium, which a
    # zero-sum perturbation does not move, and the check would compare
    # roundoff with roundoff)
    dt = np.full(n, 2e-7)
    h = dt / rng.integers(3, 40, n)
    lam = rng.normal(size=(n, 2))
    a = plan.integrate(dev(torch, T), dev(torch, p), dev(torch, Y0.T), dev(torch, dt), h=dev(torch, h))
    b = plan.integrate(dev(torch, T), dev(torch, p), dev(torch, (Y0 + dY).T), dev(torch, dt), h=dev(torch, h))
    r = plan.adjoint(dev(torch, T), dev(torch, p), dev(torch, Y0.T), dev(torch, dt), dev(torch, np.zeros(n)),
                     dev(torch, lam.T), h=dev(torch, h))
    lhs = np.sum(lam * (b["Y"].cpu().numpy().T - a["Y"].cpu().numpy().T), 1)
    rhs = np.sum(r["gY0"].cpu().numpy().T * dY, 1)
    # relative 1e-10, floored at the roundoff of the two forward maps
    # (eps |lambda| |Y| per step and component)
    floor = 1e-16 * np.sum(np.abs(lam), 1) * (dt / h)
    assert np.all(np.abs(lhs - rhs) <= 1e-10 * np.abs(lhs) + floor), np.max(np.abs(lhs - rhs) / np.abs(lhs))
    # and the temperature adjoint of this isothermal map is the chain through k(T): finite
    assert np.all(np.isfinite(r["gT0"].cpu().numpy()))


def test_adjoint_segment_recompute(torch, sc, oracle_mod):
    """2500 fixed steps: more than the 2048 checkpoint slots, so the recorder
    thins its checkpoints and the reverse sweep recomputes segments."""
    _fixed_case(torch, sc, oracle_mod, "C1", np.array([700]), 2500, 1e-2, npar=2)


def _sens_worst(torch, sc, plan, c, idx, g, N, k_no):
    T, p, Y, dt = state_gpu(torch, c, idx)
    s = g["s"]  # [cell, direction, component]; directions: N+1 unit, then parameter
    worst = np.zeros(idx.size)
    for comp in (N, k_no):
        gT1 = torch.zeros_like(T)
        gY1 = torch.zeros_like(Y)
        if comp == N:
            gT1.fill_(1.0)
        else:
            gY1[comp].fill_(1.0)
        r = plan.adjoint(T, p, Y, dt, gT1, gY1, per_cell=True)
        assert np.all(r["status"].cpu().numpy() == 0)
        g0 = np.concatenate([r["gY0"].cpu().numpy().T, r["gT0"].cpu().numpy()[:, None]], 1)
        gp = np.einsum("cdr,rc->cd", g["dpar"], r["g_dlnA_cell"].cpu().numpy())
        got = np.concatenate([g0, gp], 1)
        ref = s[:, :, comp]
        den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max(1, keepdims=True))
        worst = np.maximum(worst, (np.abs(got - ref) / den).max(1))
    return worst


def test_adjoint_vs_forward_sensitivity(torch, sc):
    """Error-controlled adjoint at rtol 1e-10 against the oracle's forward
    sensitivities at rtol 1e-10 (stored): outputs T1 and Y1 of the species
    of composition {N:1, O:1}, all 54 initial-state directions and 16 random
    rate-multiplier directions, 8 cells per class.  Steps are capped at
    dt/32: error control alone lets an equilibrated cell cross dt in one
    step, whose derivative damps fast perturbations by the method's R(h
    lambda) instead of exp(h lambda) (reported below, not gated)."""
    g = np.load(os.path.join(HERE, "golden", "c4_sens.npz"))
    c = cells("C4")
    idx = g["idx"]
    assert np.array_equal(c["T"][idx], g["T0"]) and np.array_equal(c["Y"][idx], g["Y0"])
    mech = c["mech"]
    N = mech.n_species
    k_no = next(k for k, s in enumerate(mech.species) if s.comp == {"N": 1, "O": 1})
    text = mech.to_text()
    free = _sens_worst(torch, sc, sc.Plan(sc.Mechanism(text), rtol=1e-10, atol=1e-16), c, idx, g, N, k_no)
    capped = _sens_worst(torch, sc, sc.Plan(sc.Mechanism(text), rtol=1e-10, atol=1e-16, hmax_frac=1 / 32),
                         c, idx, g, N, k_no)
    cls = g["cls"]
    for k in range(3):
        print(f"class {k}: worst relative error, steps by error control only {free[cls == k].max():.3g}, "
              f"capped at dt/32 {capped[cls == k].max():.3g}")
    assert capped.max() <= 1e-4, capped


def test_adjoint_isomer_closed_form(torch, sc):
    """A <=> B at constant T: Y_A(t) = Y_Ainf + (Y_A0 - Y_Ainf) exp(-k t) with
    k = (kf + kr) e^dlnA and Y_Ainf = kr/(kf + kr) (Y_A0 + Y_B0)."""
    from synth.mechgen import isomer_mechanism
    mech = isomer_mechanism(log10A=9.0, b=0.0, Ea=40e3, ds_R=0.7)
    plan = sc.Plan(sc.Mechanism(mech.to_text()), rtol=1e-10, atol=1e-16)
    n = 8
    Tv = np.linspace(900.0, 1300.0, n)
    YA = np.linspace(0.9, 0.2, n)
    Yv = np.stack([YA, 1 - YA])
    dt = 1e-7  # k dt from about 1 to 5 over the temperature range
    dl = np.array([0.3])
    T, p, Y = dev(torch, Tv), dev(torch, np.full(n, 101325.0)), dev(torch, Yv)
    dtt = dev(torch, np.full(n, dt))
    gY1 = torch.zeros_like(Y)
    gY1[0].fill_(1.0)
    r = plan.adjoint(T, p, Y, dtt, torch.zeros_like(T), gY1, dlnA=dl, per_cell=True)
    # closed form: kf from the Arrhenius law (cgs A of a first-order reaction
    # is already s^-1), K = exp(ds_R) (equal enthalpies), kr = kf / K
    kf = 10.0 ** 9.0 * np.exp(-40e3 / (8.314462618 * Tv))
    kr = kf / np.exp(0.7)
    k = (kf + kr) * np.exp(dl[0])
    tot = Yv[0] + Yv[1]
    yinf = kr / (kf + kr) * tot
    e = np.exp(-k * dt)
    dA = e + kr / (kf + kr) * (1 - e)       # dY_A / dY_A0
    dB = kr / (kf + kr) * (1 - e)           # dY_A / dY_B0
    dd = -(Yv[0] - yinf) * k * dt * e       # dY_A / d dlnA
    gY0 = r["gY0"].cpu().numpy()
    gd = r["g_dlnA_cell"].cpu().numpy()[0]
    np.testing.assert_allclose(gY0[0], dA, rtol=1e-7)
    np.testing.assert_allclose(gY0[1], dB, rtol=1e-7)
    np.testing.assert_allclose(gd, dd, rtol=1e-6)
    np.testing.assert_allclose(r["g_dlnA"].cpu().numpy()[0], dd.sum(), rtol=1e-6)


def test_adjoint_forward_bitwise_and_schedule_invariance(torch, sc):
    """The recording pass reproduces sc_integrate exactly; neither the cell
    order nor a budget that admits fewer resident waves changes any bit."""
    c = cells("C2")
    rng = np.random.default_rng(8)
    idx = np.sort(rng.choice(c["T"].size, 2048, replace=False))
    mech = c["mech"]
    plan = sc.Plan(sc.Mechanism(mech.to_text()))
    T, p, Y, dt = state_gpu(torch, c, idx)
    dlnA = rng.normal(size=mech.n_reactions) * 0.05
    out = plan.integrate(T, p, Y, dt, dlnA=dlnA)
    gT1 = dev(torch, rng.normal(size=idx.size))
    gY1 = dev(torch, rng.normal(size=(mech.n_species, idx.size)))
    a = plan.adjoint(T, p, Y, dt, gT1, gY1, dlnA=dlnA, forward_out=True, per_cell=True)
    assert torch.equal(a["T"], out["T"]) and torch.equal(a["Y"], out["Y"])
    assert torch.equal(a["n_acc"], out["n_acc"]) and torch.equal(a["status"], out["status"])
    cost = out["n_acc"] + out["n_rej"]
    b = plan.adjoint(T, p, Y, dt, gT1, gY1, dlnA=dlnA, cost=cost, per_cell=True,
                     budget=40 * plan.adjoint_slot_bytes() + 8 * mech.n_reactions * idx.size)
    assert b["peak_bytes"] <= 40 * plan.adjoint_slot_bytes() + 8 * mech.n_reactions * idx.size + (1 << 24)
    for k in ("gT0", "gY0", "g_dlnA", "g_dlnA_cell"):
        assert torch.equal(a[k], b[k]), k
    assert torch.isfinite(a["gY0"]).all() and torch.isfinite(a["g_dlnA"]).all()
    # the sum over cells is the per-cell array summed
    np.testing.assert_allclose(a["g_dlnA"].cpu().numpy(), a["g_dlnA_cell"].cpu().numpy().sum(1), rtol=1e-12,
                               atol=1e-12 * np.abs(a["g_dlnA_cell"].cpu().numpy()).sum())


def test_adjoint_edge_cases(torch, sc):
    c = cells("C1")
    mech = c["mech"]
    N, R = mech.n_species, mech.n_reactions
    plan = sc.Plan(sc.Mechanism(mech.to_text()))
    idx = np.arange(6)
    T, p, Y, dt = state_gpu(torch, c, idx)
    dt = dt.clone()
    dt[1] = 0.0               # no step: the cotangent passes through
    T = T.clone()
    T[2] = float("nan")       # bad input
    gT1 = dev(torch, np.arange(6) + 1.0)
    gY1 = dev(torch, np.ones((N, 6)))
    r = plan.adjoint(T, p, Y, dt, gT1, gY1, per_cell=True)
    st = r["status"].cpu().numpy()
    assert st[2] == sc.CELL_BAD_INPUT and st[1] == 0
    assert r["gT0"][1].item() == 2.0 and torch.all(r["gY0"][:, 1] == 1.0)
    assert torch.all(r["g_dlnA_cell"][:, 1] == 0.0)
    assert torch.isnan(r["gT0"][2]) and torch.isnan(r["g_dlnA"]).all()
    # max_steps reached: status and NaN gradients
    p1 = sc.Plan(sc.Mechanism(mech.to_text()), max_steps=1)
    r1 = p1.adjoint(T[3:], p[3:], Y[:, 3:].contiguous(), dt[3:], gT1[3:], gY1[:, 3:].contiguous())
    st1 = r1["status"].cpu().numpy()
    assert np.any(st1 == sc.CELL_MAX_STEPS)
    assert torch.isnan(r1["gT0"][torch.as_tensor(st1 != 0, device="cuda:0")]).all()
    # empty batch: g_dlnA is zero
    e = plan.adjoint(T[:0], p[:0], Y[:, :0].contiguous(), dt[:0], gT1[:0], gY1[:, :0].contiguous())
    assert torch.all(e["g_dlnA"] == 0.0)
    # a budget below one wave's workspace is refused
    with pytest.raises(sc.StiffchemError) as ei:
        plan.adjoint(T, p, Y, dt, gT1, gY1, budget=1024)
    assert ei.value.code == sc.SC_EBUDGET


def test_autograd_function(torch, sc):
    """torch.autograd through chem_integrate equals the direct adjoint call,
    and a second-order-free loss gets gradients for T0, Y0 and dlnA."""
    c = cells("C4")
    mech = c["mech"]
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(c["T"].size, 256, replace=False))
    plan = sc.Plan(sc.Mechanism(mech.to_text()))
    T, p, Y, dt = state_gpu(torch, c, idx)
    T0 = T.clone().requires_grad_(True)
    Y0 = Y.clone().requires_grad_(True)
    dlnA = torch.zeros(mech.n_reactions, dtype=torch.float64, device="cuda:0", requires_grad=True)
    k_no = next(k for k, s in enumerate(mech.species) if s.comp == {"N": 1, "O": 1})
    T1, Y1, _ = sc.chem_integrate(T0, Y0, dlnA, p, dt, plan)
    loss = (T1 * 1e-3).sum() + Y1[k_no].sum()
    loss.backward()
    gT1 = torch.full_like(T, 1e-3)
    gY1 = torch.zeros_like(Y)
    gY1[k_no] = 1.0
    r = plan.adjoint(T, p, Y, dt, gT1, gY1, dlnA=dlnA.detach())
    assert torch.equal(T0.grad, r["gT0"]) and torch.equal(Y0.grad, r["gY0"])
    assert torch.equal(dlnA.grad, r["g_dlnA"])
