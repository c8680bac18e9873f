"""Write the stored central-difference gradients of the fixed-step map for
the adjoint parity test on the gradient workload.

Only the oracle (oracle/), the seeded input generators (synth/) and the CPU
fixed-step Rosenbrock map (tests/frozen_map.py, which evaluates the step
formula with the oracle's right-hand side and complex-step Jacobian) are
called.  For 66 cells of the 16,384-cell 53-species workload (22 per class:
unburnt, near ignition, equilibrated; seed 21), with seeded rate-constant
log multipliers dlnA ~ N(0, 0.1^2), six fixed steps over dt/10 and a seeded
random output weight w (mass fractions ~ N(0, 100^2), T ~ N(0, 0.01^2)):
the map's value and the central differences of <w, map> in every initial
state component and four seeded parameter directions (frozen_map.fd_gradient).

Run:  python tests/golden/make_fd_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from frozen_map import fd_gradient, fixed_map  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from synth.cells import make_cells, stratified  # noqa: E402

PER_CLASS = 22
NSTEPS = 6
DT_SCALE = 0.1
NPAR = 4


def main():
    c = make_cells("C4")
    mech = c["mech"]
    N, R = mech.n_species, mech.n_reactions
    o = Oracle(mech.to_text())
    idx = stratified(c["cls"], PER_CLASS, seed=21)
    rng = np.random.default_rng(22)
    dlnA = rng.normal(size=R) * 0.1
    wY = rng.normal(size=(idx.size, N)) * 1e2
    wT = rng.normal(size=idx.size) * 1e-2
    dirs = rng.normal(size=(NPAR, R))
    dt = c["dt"][idx] * DT_SCALE
    y1 = np.empty((idx.size, N + 1))
    g = np.empty((idx.size, N + 1))
    gp = np.empty((idx.size, NPAR))
    g2, gp2 = np.empty_like(g), np.empty_like(gp)
    for n, i in enumerate(idx):
        y0 = np.append(c["Y"][i], c["T"][i])
        h = dt[n] / NSTEPS
        try:
            y1[n] = fixed_map(o, y0, c["p"][i], dt[n], h, dlnA)
            w = np.append(wY[n], wT[n])
            g[n], gp[n] = fd_gradient(o, y0, c["p"][i], dt[n], h, w, dlnA, dirs)
            # the same differences at half the steps: where the two differ by
            # more than 1e-5 the differences themselves are not converged
            g2[n], gp2[n] = fd_gradient(o, y0, c["p"][i], dt[n], h, w, dlnA, dirs, scale=0.5)
        except np.linalg.LinAlgError:
            # six fixed steps are no error control: for a few stiff cells a
            # perturbed stage matrix is numerically singular; no reference
            y1[n], g[n], gp[n], g2[n], gp2[n] = np.nan, np.nan, np.nan, np.nan, np.nan
        print(f"cell {n + 1}/{idx.size}", flush=True)
    np.savez_compressed(os.path.join(HERE, "c4_fd.npz"), idx=idx, dlnA=dlnA, wY=wY, wT=wT, dirs=dirs, dt=dt,
                        nsteps=NSTEPS, y1=y1, g=g, gp=gp, g_half=g2, gp_half=gp2, cls=c["cls"][idx])


if __name__ == "__main__":
    main()
