"""Seeded synthetic cell states (input generator only).

Each CFD cell of the paper is an independent homogeneous gas-phase reactor
(Sec. 1) and the flame holds cold, reacting and burnt gas side by side
(Sec. 2.4); with local time stepping every cell carries its own time step
(Sec. 2.5).  The workloads below reproduce that mix synthetically:

* ``C1``: 9-species {H,O,N} mechanism, 1024 cells at 1 atm, T0 uniform in
  [1000, 2200] K, mass fractions Dirichlet(1), dt = 1e-5 s;
* ``C2``: 53-species C/H/O/N mechanism, 65,536 cells at 1-10 atm (log-uniform),
  T0 log-uniform in [300, 2400] K, a third each unburnt (T0 < 600 K),
  near ignition (600-1200 K) and equilibrated (> 1200 K), dt = 1e-4 s;
* ``C3``: 110-species mechanism, 262,144 cells of the C2 classes, per-cell
  dt log-uniform in [1e-7, 1e-3] s;
* ``C4``: the C2 mechanism and classes, 16,384 cells, dt = 1e-4 s;
* ``C5``: the C3 mechanism, 65,536 cells, 20 chained substeps of 5e-5 s.

Unburnt cells are a Dirichlet mix of fuel (H2, CH4, NH3), oxidiser (O2)
and inert (N2) with no radicals; near-ignition cells add a radical pool
(H, O, OH, HO2) of total mass fraction 10^U[-4,-2]; equilibrated cells sit
at the Gibbs-energy minimum of such a mixture's elements at (T0, p).

The Gibbs minimum needs the standard Gibbs function of each species; it is
evaluated here from the NASA-7 coefficients only to place those cells on the
equilibrium manifold.  Neither the oracle nor the device library calls this
module's arithmetic: they read the mechanism text and the arrays it returns.
"""
from __future__ import annotations

import numpy as np

from .mechgen import P_REF, standard_mechanism

CONFIGS = {
    "C1": dict(mech="h2_9", n=1024, seed=201, kind="dirichlet", dt=1e-5),
    "C2": dict(mech="chon_53", n=65536, seed=202, kind="classes", dt=1e-4),
    "C3": dict(mech="chon_110", n=262144, seed=203, kind="classes", dt=("loguniform", 1e-7, 1e-3)),
    "C4": dict(mech="chon_53", n=16384, seed=204, kind="classes", dt=1e-4),
    "C5": dict(mech="chon_110", n=65536, seed=205, kind="classes", dt=5e-5, substeps=20),
    # the uneven batch of C3 (classes, per-cell LTS dt log-uniform in
    # [1e-7, 1e-3] s) on the 53-species mechanism
    "C3s": dict(mech="chon_53", n=262144, seed=203, kind="classes", dt=("loguniform", 1e-7, 1e-3)),
    # the chained substeps of C5 on the 53-species mechanism
    "C5s": dict(mech="chon_53", n=65536, seed=205, kind="classes", dt=5e-5, substeps=20),
}

FUELS = ("H2", "CH4", "NH3")
RADICALS = ("H", "O", "OH", "HO2")


def gibbs_rt(nasa, T):
    """Standard-state g/RT of every species at temperatures T (NASA-7)."""
    T = np.asarray(T, dtype=np.float64)[..., None]
    a = nasa
    lnT = np.log(T)
    h = a[:, 0] + a[:, 1] * T / 2 + a[:, 2] * T**2 / 3 + a[:, 3] * T**3 / 4 + a[:, 4] * T**4 / 5 + a[:, 5] / T
    s = a[:, 0] * lnT + a[:, 1] * T + a[:, 2] * T**2 / 2 + a[:, 3] * T**3 / 3 + a[:, 4] * T**4 / 4 + a[:, 6]
    return h - s


def _logsumexp(z, axis=-1):
    m = np.max(z, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    return (m + np.log(np.sum(np.exp(z - m), axis=axis, keepdims=True))).squeeze(axis)


def equilibrium_tp(mech, T, p, b, iters=200, tol=1e-13):
    """Mole fractions at the Gibbs minimum at fixed (T, p) (element-potential
    form).  ``b[c, e]`` is the element abundance of cell c (any scale).

    The optimum has ln x_k = -g_k/RT - ln(p/p0) + sum_e lam_e a_ek; Newton on
    (lam, ln t) solves sum_k x_k = 1 and (A x)_e = t b_e in log form.
    Returns x[c, k].  Species holding an element absent from a cell get 0.
    """
    A = mech.element_matrix()  # [E, N]
    E, N = A.shape
    T = np.atleast_1d(np.asarray(T, np.float64))
    p = np.atleast_1d(np.asarray(p, np.float64))
    b = np.atleast_2d(np.asarray(b, np.float64))
    nc = T.shape[0]
    mu0 = -gibbs_rt(mech.nasa_array(), T) - np.log(p / P_REF)[:, None]  # [nc, N]
    present = b > 0  # [nc, E]
    # species with an element missing from the cell are excluded
    excl = (A[None, :, :] > 0) & (~present[:, :, None])  # [nc, E, N]
    excl = excl.any(axis=1)
    mu0 = np.where(excl, -np.inf, mu0)
    lnb = np.log(np.where(present, b / b.sum(1, keepdims=True), 1.0))
    logA = np.where(A > 0, np.log(np.where(A > 0, A, 1.0)), -np.inf)  # [E, N]
    lam, done = _newton(A, logA, mu0, present, lnb, iters, tol, damped=False)
    if not done.all():
        # Newton can cycle on strongly lopsided element mixtures: those cells
        # start again with a backtracking line search on the residual
        bad = np.nonzero(~done)[0]
        lam_b, done_b = _newton(A, logA, mu0[bad], present[bad], lnb[bad], iters, tol, damped=True)
        lam[bad] = lam_b
        if not done_b.all():
            raise RuntimeError(f"equilibrium did not converge for {np.sum(~done_b)} cells")
    lnx = mu0 + lam @ A
    lnx -= _logsumexp(lnx)[:, None]
    return np.exp(lnx)


def _newton(A, logA, mu0, present, lnb, iters, tol, damped):
    """Newton on the element-potential equations (see equilibrium_tp);
    returns (lambda, converged).  damped: halve each step until the largest
    residual decreases (at most 40 times)."""
    E = A.shape[0]
    nc = mu0.shape[0]
    lam = np.zeros((nc, E))
    lnt = np.zeros(nc)

    def residual(lam_, lnt_):
        lnx = mu0 + lam_ @ A  # [nc, N]
        r0 = _logsumexp(lnx)
        lnAx = _logsumexp(lnx[:, None, :] + logA[None, :, :])  # [nc, E]
        re = np.where(present, lnAx - lnb - lnt_[:, None], 0.0)
        return np.concatenate([r0[:, None], re], axis=1), lnx, r0, lnAx

    done = np.zeros(nc, bool)
    for it in range(iters):
        res, lnx, r0, lnAx = residual(lam, lnt)
        err = np.abs(res).max(1)
        done = err < tol
        if done.all():
            break
        x = np.exp(lnx - r0[:, None])  # normalised weights
        Ax = x @ A.T  # [nc, E]
        J = np.zeros((nc, E + 1, E + 1))
        J[:, 0, :E] = Ax
        w = np.exp(lnx[:, None, :] - lnAx[:, :, None])  # x_k / (Ax)_e  [nc, E, N]
        w = np.where(np.isfinite(w), w, 0.0)
        J[:, 1:, :E] = np.einsum("cen,fn,en->cef", w, A, A)
        J[:, 1:, E] = -1.0
        # rows/cols of absent elements: identity (lambda_e unused)
        for e in range(E):
            miss = ~present[:, e]
            J[miss, 1 + e, :] = 0.0
            J[miss, :, e] = 0.0
            J[miss, 1 + e, e] = 1.0
        d = np.linalg.solve(J, -res[..., None])[..., 0]
        step = np.max(np.abs(d[:, :E]), axis=1)
        scale = np.minimum(1.0, 4.0 / np.maximum(step, 1e-300))
        d *= scale[:, None]
        d[done] = 0.0
        if damped:
            alpha = np.ones(nc)
            for _ in range(40):
                rt = np.abs(residual(lam + alpha[:, None] * d[:, :E], lnt + alpha * d[:, E])[0]).max(1)
                worse = (rt >= err) & ~done
                if not worse.any():
                    break
                alpha[worse] *= 0.5
            d *= alpha[:, None]
        lam += d[:, :E]
        lnt += d[:, E]
    return lam, done


def mole_to_mass(mech, x):
    W = mech.molar_masses()
    y = x * W
    return y / y.sum(-1, keepdims=True)


def _unburnt_mix(mech, rng, n):
    N = mech.n_species
    names = [s.name for s in mech.species]
    comps = [f for f in FUELS if f in names] + ["O2", "N2"]
    idx = [mech.index(c) for c in comps]
    w = rng.dirichlet(np.ones(len(idx)), size=n)
    Y = np.zeros((n, N))
    Y[:, idx] = w
    return Y


def make_cells(key, n=None, seed=None):
    """Cell states of workload ``key`` ('C1'..'C5').

    Returns a dict with float64 arrays T[n], p[n], Y[n, N] (mass fractions),
    dt[n] and int array cls[n] (0 unburnt, 1 near ignition, 2 equilibrated,
    -1 for the Dirichlet workload), plus the mechanism object.
    """
    cfg = CONFIGS[key]
    mech = standard_mechanism(cfg["mech"])
    n = cfg["n"] if n is None else n
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    N = mech.n_species
    if cfg["kind"] == "dirichlet":
        T = rng.uniform(1000.0, 2200.0, n)
        p = np.full(n, 101325.0)
        Y = rng.dirichlet(np.ones(N), size=n)
        cls = np.full(n, -1, np.int32)
    else:
        u = rng.uniform(0.0, 1.0, n)
        T = 300.0 * 8.0**u
        p = 101325.0 * 10.0 ** rng.uniform(0.0, 1.0, n)
        cls = np.where(T < 600.0, 0, np.where(T < 1200.0, 1, 2)).astype(np.int32)
        Y = _unburnt_mix(mech, rng, n)
        # near ignition: add a radical pool of total mass 10^U[-4,-2]
        rad = [mech.index(r) for r in RADICALS if r in [s.name for s in mech.species]]
        mrad = 10.0 ** rng.uniform(-4.0, -2.0, n)
        wr = rng.dirichlet(np.ones(len(rad)), size=n)
        sel = cls == 1
        Y[sel] *= (1.0 - mrad[sel])[:, None]
        Y[np.ix_(np.nonzero(sel)[0], rad)] += (mrad[sel, None] * wr[sel])
        # equilibrated: Gibbs minimum of the mixture's elements at (T, p)
        sel = np.nonzero(cls == 2)[0]
        if sel.size:
            A = mech.element_matrix()
            W = mech.molar_masses()
            b = (Y[sel] / W) @ A.T  # element moles per kg
            x = np.empty((sel.size, N))
            for s0 in range(0, sel.size, 4096):
                s1 = min(sel.size, s0 + 4096)
                x[s0:s1] = equilibrium_tp(mech, T[sel[s0:s1]], p[sel[s0:s1]], b[s0:s1])
            Y[sel] = mole_to_mass(mech, x)
    dtc = cfg["dt"]
    if isinstance(dtc, tuple):
        _, lo, hi = dtc
        dt = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n)
    else:
        dt = np.full(n, float(dtc))
    return dict(T=T, p=p, Y=Y, dt=dt, cls=cls, mech=mech, key=key,
                substeps=cfg.get("substeps", 1))


def stratified(cls, per_class, seed=0):
    """Indices of an equal-count sample of each class (sorted)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in np.unique(cls):
        idx = np.nonzero(cls == c)[0]
        out.append(rng.choice(idx, size=min(per_class, idx.size), replace=False))
    return np.sort(np.concatenate(out))
