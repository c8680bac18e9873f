"""Launch-configuration autotuner for uneven batches.

The paper balances chemistry load across MPI ranks at run time (Sec. 2.5,
dynamic load balancing).  On one GPU the equivalent choices are the launch
mode (one workgroup per cell, a static cell-to-workgroup mapping, or the
persistent queue), the queue tile (cells per pull), the grid size and the
cell order (index, longest dt first, or most steps first using the counts of
a previous call), and, with the sparse linear algebra, the number of cells
integrated side by side in one wave.  ``tune`` times each candidate on the
caller's batch (or a sample of it) and keeps the fastest; results are cached
in a JSON file keyed by mechanism size, batch size and device architecture.
"""
from __future__ import annotations

import json
import os
import time

CACHE = os.environ.get("STIFFCHEM_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune_cache.json"))

CANDIDATES = (
    [dict(mode="plain", tile=1, grid=0, order="none"),
     dict(mode="static", tile=1, grid=0, order="none")]
    + [dict(mode="persistent", tile=t, grid=0, order=o) for t in (1, 2, 4) for o in ("none", "dt", "cost")]
)


def _key(mech, n, torch, device, rtol, atol):
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    return f"N{mech.N}-R{mech.R}-n{n}-{arch}-rtol{rtol:g}-atol{atol:g}"


def tune(mech, T, p, Y, dt, device=0, rtol=1e-6, atol=1e-12, candidates=CANDIDATES, reps=2,
         use_cache=True, verbose=False, reactor="const_p", method="ros4", cost=None, linalg="auto"):
    """Returns (best config dict, {config name: ms}); the config holds the
    Plan keywords mode, tile, grid, order and cells_per_wave.  Every launch
    candidate of one cells_per_wave setting must give bitwise identical
    results (the per-cell arithmetic does not depend on the launch); the
    tuner checks that and raises if not.

    cost: (n_acc, n_rej) per cell, the predicted work the "cost" order sorts
    by (e.g. the counts of the previous operator-split substep).  Without it
    the tuner uses the counts of an identical earlier call on the same cells,
    which are exact: an upper bound of what cost ordering can gain."""
    import torch

    from . import Plan
    key = _key(mech, T.shape[0], torch, device, rtol, atol) + ("" if reactor == "const_p" else "/" + reactor) + (
        "" if method == "ros4" else "/" + method) + ("/exact-cost" if cost is None else "/predicted-cost")
    cache = {}
    if use_cache and os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["times"]
    times = {}
    prev = None if cost is None else {"n_acc": cost[0], "n_rej": cost[1]}
    # cells per wave: the sparse kernels fit 4 cells of up to 16 positions
    # (N + 2), 2 of up to 32; launches of one such setting give identical
    # bits, different settings agree to rounding (checked against the
    # integrator's tolerance)
    npos = mech.N + 2
    cpws = [1] if linalg != "sparse" else [c for c in (1, 2, 4) if c == 1 or npos <= 64 // c]
    ref_any = None
    for cpw in cpws:
        ref = None
        for cfg0 in candidates:
            cfg = dict(cfg0, cells_per_wave=cpw)
            out, name, best = _time(Plan, mech, device, rtol, atol, reactor, method, linalg, cfg, prev, reps, T, p, Y,
                                    dt, torch)
            times[name] = best * 1e3
            if ref is None:
                ref = {k: v.clone() for k, v in out.items()}
                if prev is None:
                    prev = {"n_acc": ref["n_acc"], "n_rej": ref["n_rej"]}
                if ref_any is None:
                    ref_any = ref
                elif not torch.allclose(ref["T"], ref_any["T"], rtol=10 * rtol, atol=0.0):
                    raise RuntimeError(f"cells_per_wave {cpw} changed the results beyond rounding")
            else:
                for k in ("T", "Y", "status", "n_acc", "n_rej"):
                    if not torch.equal(ref[k], out[k]):
                        raise RuntimeError(f"launch configuration {name} changed the results ({k})")
            if verbose:
                print(f"  {name}: {best * 1e3:.2f} ms", flush=True)
    best_name = min(times, key=times.get)
    best_cfg = next(dict(c, cells_per_wave=w) for w in cpws for c in candidates if _name(dict(c, cells_per_wave=w))
                    == best_name)
    if use_cache:
        cache[key] = {"best": best_cfg, "times": times}
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    return best_cfg, times


def _name(cfg):
    return f"{cfg['mode']}/t{cfg['tile']}/g{cfg['grid']}/{cfg['order']}" + (
        f"/c{cfg['cells_per_wave']}" if cfg.get("cells_per_wave", 1) != 1 else "")


def _time(Plan, mech, device, rtol, atol, reactor, method, linalg, cfg, prev, reps, T, p, Y, dt, torch):
    """Best-of-reps wall time of one configuration; returns (outputs, name, seconds)."""
    plan = Plan(mech, device=device, rtol=rtol, atol=atol, reactor=reactor, method=method, linalg=linalg, **cfg)
    out = None
    if cfg["order"] == "cost":
        # an output buffer whose counts are overwritten with the predicted
        # (or an identical earlier call's) counts before every timed call
        out = plan.integrate(T, p, Y, dt)
    best = float("inf")
    for _ in range(reps):
        if cfg["order"] == "cost" and prev is not None:
            out["n_acc"].copy_(prev["n_acc"])
            out["n_rej"].copy_(prev["n_rej"])
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        out = plan.integrate(T, p, Y, dt, out=out)
        torch.cuda.synchronize(device)
        best = min(best, time.perf_counter() - t0)
    return out, _name(cfg), best
