"""Test infrastructure: CPU reference of the operator-split, locally
time-stepped driver.  Only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.

Sec. 2.5 of the paper advances every cell with its own time step, the
largest its local CFL number allows, and integrates the chemistry of each
cell as an independent reactor between transport updates.  The transport
operator here is the simplest one with that structure: first-order upwind
advection along +x with the cell's velocity u, plus diffusion with one
coefficient D, on a uniform nx x ny grid of spacing dx.  With Co = u dt/dx
and Fo = D dt/dx^2 one update of a cell value q reads

    q' = q - Co (q - q_W) + Fo (q_E + q_W + q_N + q_S - 4 q),

with ghost values: q_W at x = 0 is the inflow profile (Dirichlet), and the
east, south and north ghosts copy the boundary cell (zero gradient).  A
split step is the chemistry over dt of every cell followed by one transport
update of every mass fraction and of the temperature.

Parity status: the transport is pinned by closed forms (a pure-advection
shift at Co = 1, the discrete cosine modes of diffusion), conservation and
the maximum principle; the chemistry is the oracle's integrator.
"""
from __future__ import annotations

import numpy as np


def transport2d(q, u, dt, dx, D, inflow, nx, ny):
    """One update of the rows of q [ncomp, ny*nx] (cell c = iy*nx + ix);
    u, dt [ny*nx]; inflow [ncomp, ny].  Returns a new array."""
    q = np.asarray(q, np.float64)
    ncomp = q.shape[0]
    g = np.empty((ncomp, ny + 2, nx + 2))      # grid with one ghost layer
    g[:, 1:-1, 1:-1] = q.reshape(ncomp, ny, nx)
    g[:, 1:-1, 0] = inflow                     # west: inflow
    g[:, 1:-1, -1] = g[:, 1:-1, -2]            # east: zero gradient
    g[:, 0, 1:-1] = g[:, 1, 1:-1]              # south
    g[:, -1, 1:-1] = g[:, -2, 1:-1]            # north
    qc = g[:, 1:-1, 1:-1]
    qw, qe = g[:, 1:-1, :-2], g[:, 1:-1, 2:]
    qs, qn = g[:, :-2, 1:-1], g[:, 2:, 1:-1]
    co = (np.asarray(u) * np.asarray(dt) / dx).reshape(ny, nx)
    fo = (D * np.asarray(dt) / (dx * dx)).reshape(ny, nx)
    out = qc - co * (qc - qw) + fo * (qe + qw + qn + qs - 4.0 * qc)
    return out.reshape(ncomp, ny * nx)


def split_run(oracle, field, steps, rtol=1e-6, atol=1e-12, nthreads=0):
    """``steps`` split steps of the field (a dict with T, p, Y [cells, N],
    u, dt, dx, D, inflow_T, inflow_Y [N, ny], nx, ny): chemistry of every
    cell over its own dt with the oracle's integrator, then one transport
    update of Y and T.  Returns (T, Y [cells, N], per-step chemistry
    status arrays)."""
    T = np.array(field["T"], np.float64)
    Y = np.array(field["Y"], np.float64)
    nx, ny = field["nx"], field["ny"]
    inflow = np.vstack([field["inflow_Y"], field["inflow_T"][None, :]])
    status = []
    for _ in range(steps):
        r = oracle.integrate(T, field["p"], Y, field["dt"], rtol=rtol, atol=atol, nthreads=nthreads)
        status.append(r["status"])
        q = np.vstack([r["Y"].T, r["T"][None, :]])
        q = transport2d(q, field["u"], field["dt"], field["dx"], field["D"], inflow, nx, ny)
        Y, T = q[:-1].T.copy(), q[-1].copy()
    return T, Y, status
