"""Test infrastructure: CPU reference of zonal reference-cell mapping.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  Sec. 2.5 of the paper adopts the load-balanced solver's zonal
reference-cell mapping: in regions of low reactivity the chemistry is not
solved cell by cell; the solution of a reference cell is mapped onto the
other cells of its zone.  The paper gives no formulas, so this module fixes
a reading (each step below is what the device path computes, written out
plainly):

1. Low reactivity is measured by a mixture fraction Z between a fuel and an
   oxidiser stream, from Bilger's coupling function (Bilger 1988): per unit
   mass of mixture, beta = 2 n_C + n_H / 2 - n_O in moles of element atoms,
   i.e. beta = sum_k (2 a_Ck + a_Hk / 2 - a_Ok) Y_k / W_k, and
   Z = (beta - beta_ox) / (beta_fuel - beta_ox).  Z is 0 in pure oxidiser, 1
   in pure fuel and linear in the mass fractions between them.
2. A cell is mappable when its inputs are finite, T > 0, p > 0, dt > 0 and
   Z < z_tol.
3. Zones: temperature bands of width dT, index iT = floor(T / dT) with
   iT < ceil(T_MAX / dT), and, when dlnp > 0, bands of ln p of width dlnp,
   index ip = floor(ln p / dlnp) with 0 <= ip < ceil(ln P_MAX / dlnp) (p in
   Pa); a mappable cell outside those ranges is not mapped.
4. The reference cell of a zone is its mappable cell of lowest index; it is
   integrated like any other cell.
5. Every other mappable cell of the zone takes the reference's change
   scaled to its own step, as a mean rate over the step:
   y1 = y0 + (y1_ref - y0_ref) dt / dt_ref for T and each Y_k; its step
   counts are zero and its status that of the reference.
"""
from __future__ import annotations

import math

import numpy as np

T_MAX = 10000.0  # K: temperature bands cover [0, T_MAX)
P_MAX = 1e9      # Pa: pressure bands cover [1 Pa, P_MAX)


def parse_species(text):
    """Element names, per-species element counts [N, E] and molar masses
    [N] (kg/mol) from the mechanism text's ELEMENTS and SP lines."""
    elements, comp, W = [], [], []
    for line in text.splitlines():
        f = line.split()
        if not f:
            continue
        if f[0] == "ELEMENTS":
            elements = f[2:2 + int(f[1])]
        elif f[0] == "SP":
            W.append(float(f[2]))
            comp.append([float(v) for v in f[3:3 + len(elements)]])
    return elements, np.array(comp, np.float64), np.array(W, np.float64)


def bilger_weights(text):
    """Per-species weights w_k of beta = sum_k w_k Y_k (mol/kg): carbon
    counts 2, hydrogen 1/2, oxygen -1 per atom (elements a mechanism does
    not have count nothing; nitrogen and others are inert here)."""
    elements, comp, W = parse_species(text)
    coef = {"C": 2.0, "H": 0.5, "O": -1.0}
    a = np.zeros(len(W))
    for e, name in enumerate(elements):
        a += coef.get(name, 0.0) * comp[:, e]
    return a / W


def mixture_fraction(w, Y, Y_fuel, Y_ox):
    """Z of each row of Y [cells, N] between the two streams.  beta is
    summed species by species in index order."""
    def beta(y):
        s = 0.0
        for k in range(len(w)):
            s += w[k] * y[k]
        return s
    b_f, b_o = beta(Y_fuel), beta(Y_ox)
    return np.array([(beta(y) - b_o) / (b_f - b_o) for y in np.atleast_2d(Y)])


def zones(T, p, Y, dt, w, Y_fuel, Y_ox, z_tol, dT, dlnp):
    """Zone key of every cell (None: not mappable).  Keys are (iT, ip)."""
    Z = mixture_fraction(w, Y, Y_fuel, Y_ox)
    keys = []
    for c in range(len(T)):
        ok = (math.isfinite(Z[c]) and math.isfinite(T[c]) and math.isfinite(p[c]) and math.isfinite(dt[c])
              and T[c] > 0.0 and p[c] > 0.0 and dt[c] > 0.0 and Z[c] < z_tol)
        iT = ip = 0
        if ok:
            iT = math.floor(T[c] / dT)
            ok = iT < math.ceil(T_MAX / dT)
        if ok and dlnp > 0.0:
            ip = math.floor(math.log(p[c]) / dlnp)
            ok = 0 <= ip < math.ceil(math.log(P_MAX) / dlnp)
        keys.append((iT, ip) if ok else None)
    return keys


def references(keys):
    """ref[c]: c itself for cells that are integrated (not mappable, or the
    lowest index of their zone), else the zone's reference cell."""
    first = {}
    ref = np.arange(len(keys), dtype=np.int32)
    for c, k in enumerate(keys):
        if k is None:
            continue
        if k not in first:
            first[k] = c
        ref[c] = first[k]
    return ref


def map_results(ref, T0, Y0, dt, T1, Y1, status, n_acc, n_rej):
    """Step 5: fill the mapped cells of (T1, Y1 [cells, N], status,
    n_acc, n_rej) from their references' results.  Returns new arrays."""
    T1, Y1 = T1.copy(), Y1.copy()
    status, n_acc, n_rej = status.copy(), n_acc.copy(), n_rej.copy()
    for c in range(len(ref)):
        r = ref[c]
        if r == c:
            continue
        s = dt[c] / dt[r]
        T1[c] = T0[c] + (T1[r] - T0[r]) * s
        Y1[c] = Y0[c] + (Y1[r] - Y0[r]) * s
        status[c] = status[r]
        n_acc[c] = 0
        n_rej[c] = 0
    return T1, Y1, status, n_acc, n_rej


def integrate_mapped(oracle, text, T0, p, Y0, dt, Y_fuel, Y_ox, z_tol, dT, dlnp=0.0, **kw):
    """The whole mapped integration with the oracle's integrator for the
    cells that are integrated.  Returns the oracle.integrate dict plus ref."""
    T0, p, dt = (np.asarray(a, np.float64) for a in (T0, p, dt))
    Y0 = np.asarray(Y0, np.float64)
    w = bilger_weights(text)
    ref = references(zones(T0, p, Y0, dt, w, Y_fuel, Y_ox, z_tol, dT, dlnp))
    own = np.flatnonzero(ref == np.arange(len(ref)))
    n, N = Y0.shape
    T1, Y1 = np.zeros(n), np.zeros((n, N))
    st, na, nr = (np.zeros(n, np.int32) for _ in range(3))
    r = oracle.integrate(T0[own], p[own], Y0[own], dt[own], **kw)
    T1[own], Y1[own], st[own], na[own], nr[own] = r["T"], r["Y"], r["status"], r["n_acc"], r["n_rej"]
    T1, Y1, st, na, nr = map_results(ref, T0, Y0, dt, T1, Y1, st, na, nr)
    return dict(T=T1, Y=Y1, status=st, n_acc=na, n_rej=nr, ref=ref)
