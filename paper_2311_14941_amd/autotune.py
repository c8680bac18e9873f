"""Launch-configuration autotuner for uneven batches.

The paper balances chemistry load across MPI ranks at run time (Sec. 2.5,
dynamic load balancing).  On one GPU the equivalent choices are the launch
mode (one workgroup per cell, a static cell-to-workgroup mapping, or the
persistent queue), the queue tile (cells per pull), the grid size and the
cell order (index, longest dt first, or most steps first using the counts of
a previous call).  ``tune`` times each candidate on the caller's batch (or a
sample of it) and keeps the fastest; results are cached in a JSON file keyed
by mechanism size, batch size and device architecture.
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
    """Returns (best config dict, {config name: ms}).  Every candidate must give
    bitwise identical results (the per-cell arithmetic does not depend on the
    launch); the tuner checks that and raises if not.

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
    times, ref = {}, None
    prev = None if cost is None else {"n_acc": cost[0], "n_rej": cost[1]}
    for cfg in candidates:
        plan = Plan(mech, device=device, rtol=rtol, atol=atol, reactor=reactor, method=method, linalg=linalg,
                    **cfg)
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
        name = f"{cfg['mode']}/t{cfg['tile']}/g{cfg['grid']}/{cfg['order']}"
        times[name] = best * 1e3
        if ref is None:
            ref = {k: v.clone() for k, v in out.items()}
            if prev is None:
                prev = {"n_acc": ref["n_acc"], "n_rej": ref["n_rej"]}
        else:
            for k in ("T", "Y", "status", "n_acc", "n_rej"):
                if not torch.equal(ref[k], out[k]):
                    raise RuntimeError(f"launch configuration {name} changed the results ({k})")
        if verbose:
            print(f"  {name}: {best * 1e3:.2f} ms", flush=True)
    best_name = min(times, key=times.get)
    best_cfg = next(c for c in candidates if f"{c['mode']}/t{c['tile']}/g{c['grid']}/{c['order']}" == best_name)
    if use_cache:
        cache[key] = {"best": best_cfg, "times": times}
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    return best_cfg, times
