"""Write the stored oracle references used by the GPU parity tests.

Only the oracle (oracle/) and the seeded input generators (synth/) are
called.  References are converged solutions: the oracle at (rtol, atol) =
(1e-11, 1e-17), accepted when it agrees with a (1e-10, 1e-16) run to 5e-2 of
the parity tolerance in every component (else one level tighter) (relative 1e-6 on T and on mass
fractions above 1e-8, absolute 1e-12 below); see reference() for the
per-cell choice of level.

Run:  python tests/golden/make_golden.py [c1] [c2]  (C1 all 1024 cells, C2 a 4,098-cell
                                                    stratified sample: constant pressure)
      python tests/golden/make_golden.py constv    (C2 sample as constant-volume
                                                    reactors: c2v_ref.npz)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from synth.cells import make_cells, stratified  # noqa: E402


def parity_excess(T, Y, Tref, Yref):
    """max over components of |err| / tolerance (<= 1 passes)."""
    eT = np.abs(T - Tref) / (1e-6 * np.abs(Tref))
    big = np.abs(Yref) > 1e-8
    eY = np.where(big, np.abs(Y - Yref) / (1e-6 * np.abs(Yref) + 1e-300), np.abs(Y - Yref) / 1e-12)
    return np.maximum(eT, eY.max(1))


LEVELS = [(1e-9, 1e-15), (1e-10, 1e-16), (1e-11, 1e-17)]
TIGHTEST = (1e-12, 1e-18)  # run only for cells whose 1e-10 and 1e-11 runs still differ
ACCEPT = 5e-2  # consecutive levels must agree to this fraction of the tolerance
MAX_STEPS = 20000


def reference(o, T, p, Y, dt, constv=False):
    """Per cell, the tightest level that succeeds and agrees with the level
    below it to ACCEPT of the parity tolerance.  (Hot equilibrated cells can
    fail at 1e-11: the roundoff of their large forward and reverse rates
    exceeds that tolerance, so those cells use the 1e-10 level.)"""
    runs = [o.integrate(T, p, Y, dt, rtol=r, atol=a, max_steps=MAX_STEPS, constv=constv) for r, a in LEVELS]
    n = T.shape[0]
    Tref, Yref = np.empty(n), np.empty_like(Y)
    level = np.full(n, -1)
    agree = np.full(n, np.inf)
    for lv in (2, 1):
        ok = (runs[lv]["status"] == 0) & (runs[lv - 1]["status"] == 0)
        ex = parity_excess(runs[lv - 1]["T"], runs[lv - 1]["Y"], runs[lv]["T"], runs[lv]["Y"])
        take = ok & (ex <= ACCEPT) & (level < 0)
        Tref[take], Yref[take] = runs[lv]["T"][take], runs[lv]["Y"][take]
        level[take], agree[take] = lv, ex[take]
    miss = np.nonzero(level < 0)[0]
    if miss.size:
        # one level tighter for the cells whose last two levels still differ
        r4 = o.integrate(T[miss], p[miss], Y[miss], dt[miss], rtol=TIGHTEST[0], atol=TIGHTEST[1],
                         max_steps=MAX_STEPS, constv=constv)
        ex = parity_excess(runs[2]["T"][miss], runs[2]["Y"][miss], r4["T"], r4["Y"])
        take = (r4["status"] == 0) & (runs[2]["status"][miss] == 0) & (ex <= ACCEPT)
        sel = miss[take]
        Tref[sel], Yref[sel] = r4["T"][take], r4["Y"][take]
        level[sel], agree[sel] = 3, ex[take]
    if np.any(level < 0):
        raise RuntimeError(f"reference did not converge for cells {np.nonzero(level < 0)[0]}")
    print(f"  levels used: {np.bincount(level, minlength=4)}, worst agreement {agree.max():.3g}",
          flush=True)
    return dict(T=Tref, Y=Yref, level=level, n_acc=runs[1]["n_acc"]), agree.max()


C2_PER_CLASS = 1366  # 4,098 of the 65,536 cells, a third from each class


def main(which=("c1", "c2")):
    out = {}
    if "c1" in which:
        # C1: all 1024 cells
        c1 = make_cells("C1")
        o1 = Oracle(c1["mech"].to_text())
        ref, conv = reference(o1, c1["T"], c1["p"], c1["Y"], c1["dt"])
        np.savez_compressed(os.path.join(HERE, "c1_ref.npz"), idx=np.arange(c1["T"].size), T=ref["T"],
                            Y=ref["Y"], level=ref["level"], n_acc=ref["n_acc"], conv=conv)
        out["c1"] = conv
    if "c2" in which:
        # C2: a stratified sample of the full 65,536-cell batch
        c2 = make_cells("C2")
        o2 = Oracle(c2["mech"].to_text())
        idx = stratified(c2["cls"], C2_PER_CLASS, seed=11)
        ref, conv = reference(o2, c2["T"][idx], c2["p"][idx], c2["Y"][idx], c2["dt"][idx])
        np.savez_compressed(os.path.join(HERE, "c2_ref.npz"), idx=idx, T=ref["T"], Y=ref["Y"],
                            level=ref["level"], n_acc=ref["n_acc"], conv=conv)
        out["c2"] = conv
    if "c3" in which:
        # C3 (110 species, per-cell dt 1e-7..1e-3 s): 16 cells per class
        c3 = make_cells("C3")
        o3 = Oracle(c3["mech"].to_text())
        idx = stratified(c3["cls"], 16, seed=13)
        ref, conv = reference(o3, c3["T"][idx], c3["p"][idx], c3["Y"][idx], c3["dt"][idx])
        np.savez_compressed(os.path.join(HERE, "c3_ref.npz"), idx=idx, T=ref["T"], Y=ref["Y"],
                            level=ref["level"], n_acc=ref["n_acc"], conv=conv)
        out["c3"] = conv
    print(out)


def main_constv():
    """The C2 stratified sample (16 cells per class, seed 11) as rigid
    vessels: each cell's density is that of its (p, T0, Y0) state."""
    from synth.mechgen import R_GAS
    c2 = make_cells("C2")
    o2 = Oracle(c2["mech"].to_text())
    idx = stratified(c2["cls"], 16, seed=11)
    W = c2["mech"].molar_masses()
    rho = c2["p"][idx] / (R_GAS * c2["T"][idx] * (c2["Y"][idx] / W).sum(1))
    ref, conv = reference(o2, c2["T"][idx], rho, c2["Y"][idx], c2["dt"][idx], constv=True)
    np.savez_compressed(os.path.join(HERE, "c2v_ref.npz"), idx=idx, rho=rho, T=ref["T"], Y=ref["Y"],
                        level=ref["level"], n_acc=ref["n_acc"], conv=conv)
    print({"c2v": conv})


if __name__ == "__main__":
    if sys.argv[1:] == ["constv"]:
        main_constv()
    elif sys.argv[1:]:
        main(sys.argv[1:])
    else:
        main()
