"""Write the stored forward-sensitivity reference for the adjoint parity test.

Only the oracle (oracle/) and the seeded input generators (synth/) are
called.  For 24 cells of the 16,384-cell 53-species workload (8 per class:
unburnt, near ignition, equilibrated; seed 11), the oracle integrates the
tangent system  s' = J s + (df/d dlnA) d  alongside the state (Radau IIA,
complex-step derivatives) for the 54 unit initial-state directions and 16
seeded Gaussian directions of the rate-constant log multipliers.  The
reference is the rtol 1e-10 run; a 1e-9 run gives the error estimate stored
beside it.

Run:  python tests/golden/make_sens_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from synth.cells import make_cells, stratified  # noqa: E402

N_PER_CLASS = 8
N_PAR_DIRS = 16


def main():
    c = make_cells("C4")
    o = Oracle(c["mech"].to_text())
    N, R = o.N, o.R
    idx = stratified(c["cls"], N_PER_CLASS, seed=11)
    n = idx.size
    nd = N + 1 + N_PAR_DIRS
    s0 = np.zeros((n, nd, N + 1))
    for d in range(N + 1):
        s0[:, d, d] = 1.0
    dpar = np.zeros((n, nd, R))
    dpar[:, N + 1:, :] = np.random.default_rng(12).standard_normal((n, N_PAR_DIRS, R))
    args = (c["T"][idx], c["p"][idx], c["Y"][idx], c["dt"][idx], s0, dpar)
    y, s, st = o.integrate_sens(*args, rtol=1e-10, atol=1e-16)
    y9, s9, st9 = o.integrate_sens(*args, rtol=1e-9, atol=1e-15)
    if np.any(st != 0) or np.any(st9 != 0):
        raise RuntimeError(f"sensitivity integration failed: {st} {st9}")
    err = np.abs(s - s9)
    # convergence of the two outputs the test uses: T and the {N:1, O:1} species
    k_no = next(k for k, sp in enumerate(c["mech"].species) if sp.comp == {"N": 1, "O": 1})
    for comp in (N, k_no):
        ref = s[:, :, comp]
        den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max(1, keepdims=True))
        worst = np.max(err[:, :, comp] / den)
        print(f"component {comp}: worst relative change 1e-9 -> 1e-10: {worst:.3g}", flush=True)
        if worst > 1e-6:
            raise RuntimeError("sensitivity reference not converged")
    np.savez_compressed(os.path.join(HERE, "c4_sens.npz"), idx=idx, y=y, s=s, s_err=err, dpar=dpar[:, N + 1:, :],
                        T0=c["T"][idx], p=c["p"][idx], Y0=c["Y"][idx], dt=c["dt"][idx], cls=c["cls"][idx])


if __name__ == "__main__":
    main()
