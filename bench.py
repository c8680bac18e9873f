"""Benchmark: cells/s integrated at rtol 1e-6 on the 53-species workload.

One "step" = one integration of the whole batch (65,536 cells of the seeded
53-species / 325-reaction C/H/O/N mechanism, 1-10 atm, T0 log-uniform in
[300, 2400] K with unburnt / near-ignition / equilibrated thirds, dt = 1e-4 s,
rtol 1e-6, atol 1e-12) through the C ABI, inputs resident in HBM.  The
timed region is K steps bracketed by device synchronisation; per-launch
kernel time comes from HIP events recorded on the launch stream.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
Single GPU only: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak (256 CU x 128 flop/clk x 2.4 GHz)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cells, budget_s=15.0, constv=False):
    """The oracle (plain dense Radau IIA, FD Jacobian) at the production
    tolerance on a stratified sample of the same batch, all host threads.
    constv: the cells' "p" entries are densities of constant-volume reactors."""
    from oracle.oracle import Oracle, max_threads
    from synth.cells import stratified
    o = Oracle(cells["mech"].to_text())
    threads = max_threads()
    done, t_used, per = 0, 0.0, 8
    sample = stratified(cells["cls"], 2048, seed=5)
    rng = np.random.default_rng(5)
    sample = rng.permutation(sample)
    # warm-up on a few cells, then time batches until the budget is used
    o.integrate(cells["T"][sample[:4]], cells["p"][sample[:4]], cells["Y"][sample[:4]], cells["dt"][sample[:4]],
                rtol=1e-6, atol=1e-12, nthreads=threads, constv=constv)
    pos = 0
    while t_used < budget_s and pos < sample.size:
        idx = sample[pos:pos + per * threads]
        pos += idx.size
        t0 = time.perf_counter()
        r = o.integrate(cells["T"][idx], cells["p"][idx], cells["Y"][idx], cells["dt"][idx], rtol=1e-6, atol=1e-12,
                        nthreads=threads, constv=constv)
        t_used += time.perf_counter() - t0
        done += idx.size
        assert np.all(r["status"] == 0)
    return dict(value=done / t_used, unit="cells/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
                sample=f"{done} cells stratified over the three classes of the same batch (seed 5), "
                       f"{t_used:.1f} s of CPU wall time on {threads} threads, rtol 1e-6 atol 1e-12")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=65536)
    ap.add_argument("--mode", default="auto", choices=["auto", "plain", "persistent", "static"],
                    help="launch configuration; auto: the autotuner's pick on a 16,384-cell sample")
    ap.add_argument("--order", default="none", choices=["none", "dt", "cost"],
                    help="persistent mode: cell order (cost: the previous call's step counts)")
    ap.add_argument("--tile", type=int, default=1)
    ap.add_argument("--linalg", default="sparse", choices=["auto", "dense", "sparse"],
                    help="linear algebra of the implicit stages (default sparse, the faster family; auto: "
                         "the library's choice, dense up to 63 species; the extrapolation baseline runs dense)")
    ap.add_argument("--cells-per-wave", type=int, default=0,
                    help="sparse linear algebra: cells per 64-lane wave (0: the most that fit)")
    ap.add_argument("--method", default="ros4", choices=["ros4", "extrap"],
                    help="c2/c2v: integration method (extrap: the extrapolation baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--spinup", type=int, default=400,
                    help="lts workload: untimed split steps before the warm-up and the timed steps")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="c1/c2: time the tuned launch only (no launch variants, host-to-host or parity "
                         "blocks; for profiler runs)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c2v", "c1", "c3", "c3s", "c5", "c5s", "lts", "copy"],
                    help="c2: the headline (default); c2v: the same cells as constant-volume reactors; "
                         "c1: the 9-species workload's 1,024 cells (tiled to --cells); "
                         "c3: the uneven batch on the 110-species mechanism, queue vs static mapping "
                         "(c3s: on the 53-species one); "
                         "c5: 20 chained substeps of the 110-species mechanism, forward and gradient "
                         "(c5s: 53 species); lts: split steps (chemistry + "
                         "transport) of the 170 x 170 flame field with local time steps; copy: a plain "
                         "device copy of known size (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the batch of independent "
              "cells would shard by predicted cost across GPUs, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2311_14941_amd as sc
    from synth.cells import make_cells

    sc.ensure_built()
    if args.workload in ("c3", "c3s"):
        return bench_uneven(args)
    if args.workload in ("c5", "c5s"):
        return bench_chained(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "lts":
        return bench_lts(args)
    if args.method == "extrap":
        args.linalg = "dense"  # the baseline integrator exists in the dense family only
    c1 = args.workload == "c1"
    log("bench: generating the " + ("C1" if c1 else "C2") + " workload")
    cells = make_cells("C1" if c1 else "C2")
    constv = args.workload == "c2v"
    if c1:
        args.no_gradient = True  # the gradient workload is the 53-species one
    if args.method != "ros4":
        args.no_gradient = True  # the adjoint is the Rosenbrock method's
    if constv:
        # rigid vessels at each cell's initial density; the "p" input is rho
        W = cells["mech"].molar_masses()
        cells["p"] = cells["p"] * (1.0 / (cells["Y"] / W).sum(1)) / (8.314462618 * cells["T"])
        args.no_gradient = True
    n = args.cells
    idx = np.arange(n) % cells["T"].size
    dev = "cuda:0"
    T = torch.tensor(cells["T"][idx], dtype=torch.float64, device=dev)
    p = torch.tensor(cells["p"][idx], dtype=torch.float64, device=dev)
    Y = torch.tensor(np.ascontiguousarray(cells["Y"][idx].T), dtype=torch.float64, device=dev)
    dt = torch.tensor(cells["dt"][idx], dtype=torch.float64, device=dev)
    mech = sc.Mechanism(cells["mech"].to_text())
    reactor = "const_v" if constv else "const_p"
    # predicted per-cell work for the cost order: the step counts of a
    # perturbed copy of the batch (T0 and p within +-1%), standing in for the
    # previous operator-split substep's counts; never the batch's own counts
    log("bench: predicted cost from a perturbed copy of the batch")
    pred = predicted_cost(sc, torch, mech, T, p, Y, dt, reactor, args.method)
    if args.mode == "auto":
        from paper_2311_14941_amd import autotune
        log("bench: autotuning the launch configuration on a 16,384-cell sample")
        s_ = torch.tensor(np.random.default_rng(0).choice(n, 16384, replace=False), device=dev)
        launch, tune_ms = autotune.tune(mech, T[s_].contiguous(), p[s_].contiguous(), Y[:, s_].contiguous(),
                                        dt[s_].contiguous(), use_cache=False, reps=1, reactor=reactor,
                                        method=args.method, linalg=args.linalg,
                                        cost=(pred[0][s_].contiguous(),
                                                                  pred[1][s_].contiguous()))
    else:
        launch = dict(mode=args.mode, tile=args.tile, grid=0, order=args.order)
        tune_ms = None
    # cells per wave is a sparse-family setting (the dense kernels take one cell per wave)
    cpw = launch.pop("cells_per_wave", args.cells_per_wave)
    if args.linalg != "sparse":
        cpw = 0
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, reactor=reactor, method=args.method, linalg=args.linalg,
                   cells_per_wave=cpw, **launch)
    use_pred = launch["mode"] == "persistent" and launch["order"] == "cost"
    stream = torch.cuda.current_stream()
    out = None

    def run_once(o_):
        if use_pred and o_ is not None:
            o_["n_acc"].copy_(pred[0])
            o_["n_rej"].copy_(pred[1])
        return plan.integrate(T, p, Y, dt, out=o_)

    log(f"bench: warmup {args.warmup}")
    out = plan.integrate(T, p, Y, dt, out=dict(T=torch.empty_like(T), Y=torch.empty_like(Y),
                                                status=torch.empty(n, dtype=torch.int32, device=dev),
                                                n_acc=pred[0].clone(), n_rej=pred[1].clone()))
    for _ in range(max(0, args.warmup - 1)):
        out = run_once(out)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        out = run_once(out)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    st = out["status"].cpu().numpy()
    nacc = out["n_acc"].cpu().numpy().astype(np.int64)
    nrej = out["n_rej"].cpu().numpy().astype(np.int64)
    failed = int(np.sum(st != 0))
    if failed:
        log(f"bench: WARNING {failed} cells failed: {np.bincount(st)}")
    ms_per_step = wall * 1e3 / args.steps
    value = n / (wall / args.steps)
    # algorithmic FP64 work of one launch: every attempted step costs the
    # Jacobian pass, the factorisation, two new right-hand sides and four solves
    flops = float((nacc + nrej).sum()) * step_flops(mech.info, args.method)
    kern_s = float(np.mean(launch_ms)) / 1e3
    achieved = flops / kern_s / 1e12
    res = {
        "metric": "cells/s integrated @rtol 1e-6, " + ("9" if c1 else "53") + "-species mech" + (
            ", constant-volume reactor" if constv else "") + (
            ", extrapolation baseline" if args.method == "extrap" else "") + (
            "; gradient/forward time ratio" if not constv and not c1 and args.method == "ros4" else ""),
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"C1: the 1,024 reactor cells of the seeded 9-species/24-reaction H/O/N "
                                f"mechanism (3 third-body), 1 atm, T0 1000-2200 K, Dirichlet compositions, dt "
                                f"1e-5 s, tiled to {n:,} cells, rtol 1e-6, atol 1e-12") if c1 else
                               "C2: 65,536 reactor cells, seeded 53-species/325-reaction C/H/O/N "
                               "mechanism (30 third-body, 15 Troe), 1-10 atm, T0 300-2400 K in thirds "
                               "(unburnt/near-ignition/equilibrated), dt 1e-4 s, rtol 1e-6, atol 1e-12" + (
                                   "; constant-volume reactors at each cell's initial density" if constv else ""),
                   "cells": n, "launch": launch, "autotune_sample_ms": tune_ms,
                   "failed_cells": failed,
                   "cost_order_counts": ("predicted: step counts of a perturbed copy of the batch (T0, p within "
                                         "+-1%), copied in before every timed call" if use_pred else None),
                   "kernel": kernel_name(launch, args.linalg, mech.N, cpw), "linalg": args.linalg,
                   "cells_per_wave": resolved_cpw(args.linalg, mech.N, cpw),
                   "steps_per_cell_mean": float((nacc + nrej).mean()),
                   # where the work is: share of attempted steps and mean per cell by class
                   # (unburnt / near ignition / equilibrated)
                   "steps_by_class": None if c1 else {
                       name: {"share": float((nacc + nrej)[cells["cls"][idx] == k].sum() / max(1, (nacc + nrej).sum())),
                              "mean": float((nacc + nrej)[cells["cls"][idx] == k].mean())}
                       for k, name in enumerate(("unburnt", "near_ignition", "equilibrated"))},
                   "accepted_mean": float(nacc.mean()), "rejected_mean": float(nrej.mean()),
                   "gradient_forward_ratio": None},
        "paper_context": "the paper reports no chemistry throughput; its combined CPU strategy is >= 31x the "
                         "standard solver on a whole ~29,000-cell CFD run (16 MPI subdomains + OpenMP, CPU)",
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": None if constv or c1 else measured_traffic(launch, kernel_name(launch, args.linalg,
                                                                                                mech.N, cpw)),
                     "kernel_ms": kern_s * 1e3, "flops_per_launch": flops},
    }
    # the same batch through the other launches (results bitwise equal):
    # plain one-workgroup-per-cell, the queue in index order, and the queue
    # ordered by the batch's own exact counts (an upper bound: a real call
    # cannot know them)
    if args.no_extras:
        print(json.dumps(res), flush=True)
        return
    variants = {}
    for name, cfg, counts in (("plain", dict(mode="plain"), None),
                              ("persistent_index_order", dict(mode="persistent", order="none"), None),
                              ("persistent_cost_exact_upper_bound", dict(mode="persistent", order="cost"),
                               (out["n_acc"].clone(), out["n_rej"].clone()))):
        pp = sc.Plan(mech, rtol=1e-6, atol=1e-12, reactor=reactor, method=args.method, linalg=args.linalg,
                     cells_per_wave=cpw, **cfg)
        o2 = pp.integrate(T, p, Y, dt)
        ms = []
        for _ in range(2):
            if counts is not None:
                o2["n_acc"].copy_(counts[0])
                o2["n_rej"].copy_(counts[1])
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            o2 = pp.integrate(T, p, Y, dt, out=o2)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        variants[name] = {"ms": min(ms), "identical": bool(torch.equal(o2["T"], out["T"]) and
                                                            torch.equal(o2["Y"], out["Y"]))}
    res["config"]["launch_variants"] = variants
    res["config"]["plain_launch_ms"] = variants["plain"]["ms"]
    # host-to-host: state from host memory, integrate, results back to host
    res["config"]["host_to_host_ms"] = host_to_host_ms(torch, plan, cells, idx, dev, pred if use_pred else None)
    if args.linalg == "sparse" and args.method == "ros4":
        log("bench: interpolated thermodynamics")
        res["thermo_interp"] = thermo_interp(sc, torch, mech, T, p, Y, dt, out, pred if use_pred else None, launch,
                                             cpw, reactor, stream, kern_s * 1e3)
    if not constv and args.method == "ros4":
        log("bench: parity of the timed output against the stored oracle reference")
        res["parity"] = parity_block(sc, torch, mech, cells, idx, out, T, p, Y, dt, reactor, args,
                                     golden="c1_ref.npz" if c1 else "c2_ref.npz")
    if not args.no_gradient:
        log("bench: gradient/forward ratio on the 16,384-cell batch")
        grad = gradient_ratio(sc, torch, mech_text=cells["mech"].to_text(), launch=launch)
        res["config"]["gradient_forward_ratio"] = grad["ratio"]
        res["gradient"] = grad
        # the setting whose gradients the forward-sensitivity test validates:
        # steps capped at dt/32, forward and adjoint alike
        log("bench: gradient/forward ratio with steps capped at dt/32")
        res["gradient"]["steps_capped_dt_over_32"] = gradient_ratio(sc, torch, mech_text=cells["mech"].to_text(),
                                                                    launch=launch, hmax_frac=1.0 / 32)
    if not args.no_cpu_baseline and not c1:
        log("bench: CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(cells, constv=constv)
    print(json.dumps(res), flush=True)


def predicted_cost(sc, torch, mech, T, p, Y, dt, reactor, method):
    """Per-cell (n_acc, n_rej) of a perturbed copy of the batch: T0 and p each
    scaled by a seeded factor in [0.99, 1.01].  The cost order sorts by these
    counts, as it would by the previous operator-split substep's in a flow
    solver (close to, not equal to, the counts of the call itself)."""
    g = np.random.default_rng(99)
    n = T.shape[0]
    fT = torch.tensor(1.0 + g.uniform(-0.01, 0.01, n), device=T.device)
    fp = torch.tensor(1.0 + g.uniform(-0.01, 0.01, n), device=T.device)
    r = sc.Plan(mech, rtol=1e-6, atol=1e-12, reactor=reactor, method=method).integrate(T * fT, p * fp, Y, dt)
    return r["n_acc"].clone(), r["n_rej"].clone()


def host_to_host_ms(torch, plan, cells, idx, dev, pred):
    """One integration from host arrays: copy the state in, integrate, copy
    the results out (wall time, synchronous)."""
    Th, ph = cells["T"][idx], cells["p"][idx]
    Yh, dth = np.ascontiguousarray(cells["Y"][idx].T), cells["dt"][idx]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = torch.from_numpy(Th).to(dev)
    p = torch.from_numpy(ph).to(dev)
    Y = torch.from_numpy(Yh).to(dev)
    dt = torch.from_numpy(dth).to(dev)
    o = None
    if pred is not None:
        n = T.shape[0]
        o = dict(T=torch.empty_like(T), Y=torch.empty_like(Y), status=torch.empty(n, dtype=torch.int32, device=dev),
                 n_acc=pred[0].clone(), n_rej=pred[1].clone())
    r = plan.integrate(T, p, Y, dt, out=o)
    T1, Y1, st = r["T"].cpu().numpy(), r["Y"].cpu().numpy(), r["status"].cpu().numpy()
    ms = (time.perf_counter() - t0) * 1e3
    assert T1.shape == Th.shape and Y1.shape == Yh.shape and st.shape == Th.shape
    return ms


def parity_excess(T, Y, Tref, Yref):
    """Per cell: max over components of |error| / tolerance (the parity bar:
    relative 1e-6 on T and on mass fractions above 1e-8, absolute 1e-12 below;
    <= 1 passes)."""
    eT = np.abs(T - Tref) / (1e-6 * np.abs(Tref))
    big = np.abs(Yref) > 1e-8
    eY = np.where(big, np.abs(Y - Yref) / (1e-6 * np.abs(Yref) + 1e-300), np.abs(Y - Yref) / 1e-12)
    return np.maximum(eT, eY.max(1))


def thermo_interp(sc, torch, mech, T, p, Y, dt, ref, pred, launch, cpw, reactor, stream, exact_ms, tol=1e-9):
    """The same batch and launch with interpolated thermodynamics (each
    reaction's -dG/RT and dH/RT from the mechanism compiler's tables in
    ln T, at most tol absolute error): the tables' degree and size, the
    kernel time against the exact thermodynamics, and the results against
    the exact run under the parity bar."""
    t0 = time.perf_counter()
    fit = mech.thermo_fit(tol)
    fit_s = time.perf_counter() - t0
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, reactor=reactor, linalg="sparse", cells_per_wave=cpw,
                   thermo_tol=tol, **launch)
    n = T.numel()
    o = plan.integrate(T, p, Y, dt, out=dict(T=torch.empty_like(T), Y=torch.empty_like(Y),
                                             status=torch.empty(n, dtype=torch.int32, device=T.device),
                                             n_acc=torch.zeros(n, dtype=torch.int32, device=T.device),
                                             n_rej=torch.zeros(n, dtype=torch.int32, device=T.device)))
    ms = []
    for _ in range(2):
        if pred is not None:
            o["n_acc"].copy_(pred[0])
            o["n_rej"].copy_(pred[1])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        o = plan.integrate(T, p, Y, dt, out=o)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    Tt, Yt = o["T"].cpu().numpy(), o["Y"].cpu().numpy().T
    Te, Ye = ref["T"].cpu().numpy(), ref["Y"].cpu().numpy().T
    ex = parity_excess(Tt, Yt, Te, Ye)
    steps = (o["n_acc"] + o["n_rej"]).double().mean().item()
    return {"tol": tol, "degree": fit["degree"], "intervals": fit["nint"], "range_K": [250.0, 4000.0],
            "table_bytes": int(fit["coef"].nbytes), "fit_max_err": fit["max_err"], "host_fit_s": fit_s,
            "kernel_ms": min(ms), "exact_kernel_ms": exact_ms, "speedup": exact_ms / min(ms),
            "steps_per_cell_mean": steps, "failed_cells": int((o["status"] != 0).sum().item()),
            "vs_exact_thermo": {"bar": "T and Y > 1e-8 to relative 1e-6, Y <= 1e-8 to absolute 1e-12",
                                "within_bar": float(np.mean(ex <= 1.0)), "worst_excess": float(ex.max()),
                                "max_rel_dT": float(np.max(np.abs(Tt - Te) / Te))}}


RTOL_SWEEP = (1e-7, 1e-8, 1e-9, 1e-10)


def parity_block(sc, torch, mech, cells, idx, out, T, p, Y, dt, reactor, args, golden="c2_ref.npz"):
    """Parity of the timed run against the converged oracle reference of the
    batch's stored sample (tests/golden/c2_ref.npz: 4,098 stratified cells of
    the 53-species batch; c1_ref.npz: all 1,024 cells of the 9-species
    workload; both written by the oracle alone): pass fraction and worst
    excess at the production tolerance, then the loosest rtol (atol = 1e-6
    rtol, the production ratio) at which every sample cell passes, and the
    whole batch's throughput there."""
    g = np.load(os.path.join(ROOT, "tests", "golden", golden))
    ref_idx = g["idx"]
    n = T.shape[0]
    if n < cells["T"].size or not np.array_equal(idx[ref_idx], ref_idx):
        return {"note": "batch is not the full 65,536-cell workload; no stored reference for it"}
    ri = torch.tensor(ref_idx, device=T.device)
    cls = cells["cls"][ref_idx]

    def summary(T1, Y1, st):
        ex = parity_excess(T1, Y1, g["T"], g["Y"])
        ok = st == 0
        return {"pass_fraction": float(np.mean((ex <= 1.0) & ok)), "worst_excess": float(ex.max()),
                "p99_excess": float(np.percentile(ex, 99)), "median_excess": float(np.median(ex)),
                "by_class": {name: {"pass_fraction": float(np.mean(ex[cls == k] <= 1.0)),
                                    "worst_excess": float(ex[cls == k].max())}
                             for k, name in enumerate(("unburnt", "near_ignition", "equilibrated"))
                             if np.any(cls == k)}}

    sample = "stratified cells" if golden == "c2_ref.npz" else "cells (every cell of the workload)"
    res = {"reference": "oracle (Radau IIA, converged to 5e-2 of the bar between rtol 1e-10 and 1e-11), "
                        f"{ref_idx.size} {sample} of the batch",
           "bar": "T and Y > 1e-8 to relative 1e-6, Y <= 1e-8 to absolute 1e-12; excess = error / bar",
           "production_rtol_1e-6": summary(out["T"][ri].cpu().numpy(), out["Y"][:, ri].cpu().numpy().T,
                                           out["status"][ri].cpu().numpy())}
    Ts, ps, Ys, dts = T[ri].contiguous(), p[ri].contiguous(), Y[:, ri].contiguous(), dt[ri].contiguous()
    sweep, loosest = {}, None
    for rt in RTOL_SWEEP:
        r = sc.Plan(mech, rtol=rt, atol=rt * 1e-6, reactor=reactor, max_steps=200000,
                    linalg=args.linalg).integrate(Ts, ps, Ys, dts)
        s_ = summary(r["T"].cpu().numpy(), r["Y"].cpu().numpy().T, r["status"].cpu().numpy())
        sweep[f"{rt:g}"] = {"pass_fraction": s_["pass_fraction"], "worst_excess": s_["worst_excess"]}
        if s_["pass_fraction"] == 1.0:
            loosest = rt
            break
    res["rtol_sweep_on_sample"] = sweep
    if loosest is not None:
        best = None
        for mode, order in (("persistent", "none"), ("plain", "none")):
            pl = sc.Plan(mech, rtol=loosest, atol=loosest * 1e-6, reactor=reactor, max_steps=200000, mode=mode,
                         order=order, linalg=args.linalg)
            o2 = pl.integrate(T, p, Y, dt)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            o2 = pl.integrate(T, p, Y, dt, out=o2)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            if best is None or ms < best[0]:
                best = (ms, mode, int((o2["status"] != 0).sum()), float((o2["n_acc"] + o2["n_rej"]).double().mean()))
        res["loosest_all_pass"] = {"rtol": loosest, "atol": loosest * 1e-6, "value": n / (best[0] / 1e3),
                                   "unit": "cells/s", "ms": best[0], "launch": best[1], "failed_cells": best[2],
                                   "steps_per_cell_mean": best[3]}
    return res


KERNEL_SOURCES = ("paper_2311_14941_amd/csrc/core.hpp", "paper_2311_14941_amd/csrc/kernels.hip",
                  "paper_2311_14941_amd/csrc/sparse.hip", "paper_2311_14941_amd/csrc/devmech.hpp")


def step_flops(info, method):
    """Algorithmic FP64 flops of one attempted step, whichever kernel runs
    it: the mechanism compiler's count with the linear algebra of its static
    sparse schedule (the bordered LU and solves as scheduled; a dense kernel
    does more arithmetic for the same result).  Rosenbrock: Jacobian pass
    with its right-hand side, one factorisation, two more right-hand sides,
    four solves, control.  Extrapolation: one Jacobian pass and
    factorisation per column (four), six more right-hand sides and ten
    solves."""
    if method == "ros4":
        return info["flops_step_sparse"]
    jac = info["flops_jac"] - 6 * info["n_state"] ** 2 + 20 * info["n_state"]  # border formation, not dense rows
    return 4 * (jac + info["flops_lu_sparse"]) + 6 * info["flops_rhs"] + 10 * info["flops_solve_sparse"]


def resolved_cpw(linalg, N, requested=0):
    """Cells per wave a plan runs: the sparse kernels fit 4 cells of up to
    16 positions (N + 2), 2 of up to 32, else 1; the dense kernels 1."""
    if linalg != "sparse" and not (linalg == "auto" and N + 1 > 64):
        return 1
    return requested or (4 if N + 2 <= 16 else 2 if N + 2 <= 32 else 1)


def kernel_name(launch, linalg, N, cpw=0):
    """The integration kernel a launch runs (for the profile summaries):
    template arguments <slots per lane, cells per wave> for the sparse kernels."""
    mode = launch["mode"]
    if linalg == "sparse" or (linalg == "auto" and N + 1 > 64):
        vpl = 1 if N + 2 <= 64 else 2
        g = resolved_cpw(linalg, N, cpw)
        return {"plain": f"k_integrate_sp<{vpl},{g}>", "persistent": f"k_integrate_sp_persistent<{vpl},{g}>",
                "static": f"k_integrate_sp_static<{vpl},{g}>"}[mode]
    npd = 16 if N + 1 <= 16 else 32 if N + 1 <= 32 else 56 if N + 1 <= 56 else 64
    return {"plain": f"k_integrate<{npd}>", "persistent": f"k_integrate_persistent<{npd}>",
            "static": f"k_integrate_static<{npd}>"}[mode]


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launch, kernel):
    """HBM bytes per launch of the integration kernel from the committed
    counter runs (profiles/k_integrate_c2_traffic.json: FETCH_SIZE and
    WRITE_SIZE of the kernel, each divided by the bytes-per-byte ratio the
    same counter reads for a plain copy of known size), or None when the
    kernel sources changed since those runs or they cover another kernel or
    launch configuration."""
    path = os.path.join(ROOT, "profiles", "k_integrate_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_digest") != kernel_digest() or t.get("launch") != launch or t.get("kernel") != kernel:
        return None
    return t["traffic_bytes"]


def bench_copy(args):
    """A plain device copy of 2^27 doubles (1 GiB read + 1 GiB written),
    timed; under rocprofv3 --pmc its FETCH_SIZE / WRITE_SIZE per dispatch
    give the counters' bytes per true byte."""
    import torch
    n = 1 << 27
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    nbytes = n * 8
    print(json.dumps({"metric": "device copy", "bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
                      "GB/s": 2 * nbytes / ms / 1e6, "steps": args.steps}), flush=True)


def bench_chained(args):
    """20 chained substeps of 5e-5 s over 65,536 cells (53-species
    mechanism, C2 classes, seed 205), the state and step size carried:
    forward as one captured HIP graph, and the gradient of the final T and
    Y1 of the {N:1, O:1} species through torch.autograd (20 sc_integrate
    calls forward, 20 sc_adjoint calls backward).  Reports both times, their
    ratio and the device memory held."""
    import torch
    import paper_2311_14941_amd as sc
    from synth.cells import make_cells
    key = "C5" if args.workload == "c5" else "C5s"
    log(f"bench: generating the chained-substep batch {key}")
    c = make_cells(key)
    nsub = c["substeps"]
    dev = "cuda:0"
    T = torch.tensor(c["T"], device=dev)
    p = torch.tensor(c["p"], device=dev)
    Y = torch.tensor(np.ascontiguousarray(c["Y"].T), device=dev)
    dt = torch.tensor(c["dt"], device=dev)
    mech = sc.Mechanism(c["mech"].to_text())
    if mech.N + 1 <= 64:
        # with the gradient: the forward and the adjoint's recording pass run
        # the same (dense) kernels, so the recorded trajectory is the forward's
        args.linalg = "dense"
    # launch: the persistent queue in index order unless --mode says otherwise
    # (the captured graph replays the same launches; a cost order would need
    # the previous substep's counts sorted inside the graph)
    mode = "persistent" if args.mode == "auto" else args.mode
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, linalg=args.linalg, mode=mode)
    plan.adjoint_budget = 64 << 30  # the workload's device-memory cap for the adjoint's checkpoints
    k_no = next(k for k, s_ in enumerate(c["mech"].species) if s_.comp == {"N": 1, "O": 1})
    log("bench: capture + forward")
    chain = sc.Chain(plan, T, p, Y, dt, nsub)
    chain.run(T, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tf, Yf, _, steps = chain.run(T, Y)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3
    if mech.N + 1 > 64:
        # the adjoint is the dense family's (N <= 63): forward only here
        line = {"metric": "chained substeps: forward wall time", "unit": "ms", "value": fwd_ms,
                "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                "config": {"workload": f"{key}: 65,536 cells, {mech.N}-species mechanism, C2 classes, 20 chained "
                                       "substeps of 5e-5 s (state and step size carried), rtol 1e-6",
                           "substeps": nsub, "linalg": args.linalg, "mode": mode,
                           "gradient": "not run: the adjoint supports up to 63 species (dense family)"},
                "forward_graph_ms": fwd_ms, "cells_per_s": T.numel() * nsub / (fwd_ms / 1e3),
                "steps_per_cell_mean": float(steps.double().mean().item()),
                "failed_cells_last_substep": int((chain.status != 0).sum().item())}
        print(json.dumps(line), flush=True)
        return
    log("bench: gradient through autograd")
    torch.cuda.reset_peak_memory_stats()
    free0, total = torch.cuda.mem_get_info()
    T0 = T.clone().requires_grad_(True)
    Y0 = Y.clone().requires_grad_(True)
    dl = torch.zeros(mech.R, dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tk, Yk, h = T0, Y0, None
    for _ in range(nsub):
        Tk, Yk, h = sc.chem_integrate(Tk, Yk, dl, p, dt, plan, h=h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = Tk.sum() + Yk[k_no].sum()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    free1, _ = torch.cuda.mem_get_info()
    same = bool(torch.equal(Tk.detach(), Tf) and torch.equal(Yk.detach(), Yf))
    line = {"metric": "chained substeps: forward and gradient wall time", "unit": "ms",
            "value": (t2 - t1) * 1e3 / fwd_ms, "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{key}: 65,536 cells, {mech.N}-species mechanism, C2 classes, 20 chained "
                                   "substeps of 5e-5 s (state and step size carried), rtol 1e-6, adjoint "
                                   "workspace capped at 64 GB", "substeps": nsub, "linalg": args.linalg,
                       "mode": mode},
            "forward_graph_ms": fwd_ms, "autograd_forward_ms": (t1 - t0) * 1e3,
            "backward_ms": (t2 - t1) * 1e3, "gradient_forward_ratio": (t2 - t1) * 1e3 / fwd_ms,
            "graph_and_autograd_forward_identical": same,
            "steps_per_cell_mean": float(steps.double().mean().item()),
            "torch_peak_bytes": int(torch.cuda.max_memory_allocated()),
            "device_bytes_in_use_after": int(total - free1), "device_bytes_in_use_before": int(total - free0),
            "adjoint_slot_bytes": int(plan.adjoint_slot_bytes()),
            "grad_finite": bool(torch.isfinite(T0.grad).all() and torch.isfinite(dl.grad).all())}
    print(json.dumps(line), flush=True)


def gradient_ratio(sc, torch, mech_text, launch, reps=3, hmax_frac=0.0):
    """Wall time of sc_adjoint (recording forward + reverse sweep with
    recompute) over that of sc_integrate, same 16,384 cells (53-species
    mechanism, C2 classes, dt 1e-4 s, seed 204) and options; outputs T1 and
    Y1 of the {N:1, O:1} species, gradients for T0, Y0 and all dlnA.
    hmax_frac > 0 caps every step (forward and adjoint) at hmax_frac dt."""
    from synth.cells import make_cells
    c = make_cells("C4")
    dev = "cuda:0"
    T = torch.tensor(c["T"], device=dev)
    p = torch.tensor(c["p"], device=dev)
    Y = torch.tensor(np.ascontiguousarray(c["Y"].T), device=dev)
    dt = torch.tensor(c["dt"], device=dev)
    mech = sc.Mechanism(mech_text)
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, hmax_frac=hmax_frac, **launch)
    k_no = next(k for k, s_ in enumerate(c["mech"].species) if s_.comp == {"N": 1, "O": 1})
    gT1 = torch.ones_like(T)
    gY1 = torch.zeros_like(Y)
    gY1[k_no] = 1.0
    out = plan.integrate(T, p, Y, dt)
    cost = out["n_acc"] + out["n_rej"]
    r = plan.adjoint(T, p, Y, dt, gT1, gY1, cost=cost)
    torch.cuda.synchronize()

    def timed(fn):
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ms))

    fwd = timed(lambda: plan.integrate(T, p, Y, dt, out=out))
    adj = timed(lambda: plan.adjoint(T, p, Y, dt, gT1, gY1, cost=cost))
    st = r["status"].cpu().numpy()
    return {"ratio": adj / fwd, "forward_ms": fwd, "adjoint_ms": adj, "cells": int(T.numel()),
            "hmax_frac": hmax_frac, "steps_per_cell_mean": float((out["n_acc"] + out["n_rej"]).double().mean()),
            "failed_cells": int(np.sum(st != 0)), "peak_workspace_bytes": int(r["peak_bytes"]),
            "g_dlnA_finite": bool(torch.isfinite(r["g_dlnA"]).all().item())}


def bench_uneven(args):
    """Uneven batch C3: 262,144 cells of the C2 classes with per-cell dt
    log-uniform in [1e-7, 1e-3] s (step counts spread > 100x) on the seeded
    110-species / 700-reaction mechanism (sparse linear algebra: two state
    components per lane), or with --workload c3s the same batch on the
    53-species mechanism.  Static cell-to-workgroup mapping and the plain
    one-workgroup-per-cell launch (baselines) against the persistent queue
    in the configuration the autotuner picks; cost orders sort by predicted
    counts (a perturbed copy of the batch), never the call's own."""
    import torch
    import paper_2311_14941_amd as sc
    from paper_2311_14941_amd import autotune
    from synth.cells import make_cells
    key = "C3s" if args.workload == "c3s" else "C3"
    log(f"bench: generating the uneven batch {key}")
    cells = make_cells(key)
    n = cells["T"].size
    dev = "cuda:0"
    T = torch.tensor(cells["T"], device=dev)
    p = torch.tensor(cells["p"], device=dev)
    Y = torch.tensor(np.ascontiguousarray(cells["Y"].T), device=dev)
    dt = torch.tensor(cells["dt"], device=dev)
    mech = sc.Mechanism(cells["mech"].to_text())
    log("bench: predicted cost from a perturbed copy of the batch")
    pred = predicted_cost(sc, torch, mech, T, p, Y, dt, "const_p", "ros4")
    log("bench: autotuning on a 16,384-cell sample")
    s = np.random.default_rng(0).choice(n, 16384, replace=False)
    ts = torch.tensor(s, device=dev)
    best, times = autotune.tune(mech, T[ts].contiguous(), p[ts].contiguous(), Y[:, ts].contiguous(),
                                dt[ts].contiguous(), use_cache=False, reps=1, verbose=True, linalg=args.linalg,
                                cost=(pred[0][ts].contiguous(), pred[1][ts].contiguous()))

    def timed(plan, cost):
        out = plan.integrate(T, p, Y, dt)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(args.steps):
            if cost is not None:
                out["n_acc"].copy_(cost[0])
                out["n_rej"].copy_(cost[1])
            a.record()
            out = plan.integrate(T, p, Y, dt, out=out)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms)), out

    res, ref = {}, None
    for name, cfg in (("static", dict(mode="static")), ("plain", dict(mode="plain")),
                      ("persistent_index_order", dict(mode="persistent", order="none")),
                      ("persistent_tuned", best)):
        log(f"bench: {name}")
        cost = pred if cfg.get("order") == "cost" else None
        ms, out = timed(sc.Plan(mech, linalg=args.linalg, **cfg), cost)
        res[name] = ms
        if ref is None:
            ref = out
        res[name + "_identical"] = bool(torch.equal(ref["T"], out["T"]) and torch.equal(ref["Y"], out["Y"]))
    # the exact-count order (the batch's own counts: an upper bound)
    ms, _ = timed(sc.Plan(mech, linalg=args.linalg, mode="persistent", order="cost"),
                  (ref["n_acc"].clone(), ref["n_rej"].clone()))
    res["persistent_cost_exact_upper_bound"] = ms
    steps = (out["n_acc"] + out["n_rej"]).cpu().numpy()
    st = out["status"].cpu().numpy()
    N = mech.N
    line = {"metric": "uneven batch: cells/s, persistent queue vs static mapping", "unit": "cells/s",
            "value": n / (res["persistent_tuned"] / 1e3), "n_gpus": 1, "steps": args.steps,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{key}: 262,144 cells, {N}-species/{mech.R}-reaction mechanism, C2 classes, "
                                   "dt log-uniform 1e-7..1e-3 s, rtol 1e-6, atol 1e-12", "tuned": best,
                       "linalg": args.linalg, "kernel": kernel_name(best, args.linalg, N),
                       "failed_cells": int(np.sum(st != 0))},
            "ms": res, "speedup_vs_static": res["static"] / res["persistent_tuned"],
            "speedup_vs_plain": res["plain"] / res["persistent_tuned"],
            "steps_per_cell": {"mean": float(steps.mean()), "p50": float(np.median(steps)),
                               "p10": float(np.percentile(steps, 10)), "max": int(steps.max()),
                               "spread_max_over_p10": float(steps.max() / max(1, np.percentile(steps, 10)))},
            "tuning_sample_ms": times}
    flops = float(steps.sum()) * mech.info["flops_step_sparse"]
    achieved = flops / (res["persistent_tuned"] / 1e3) / 1e12
    line["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "flops_per_launch": flops}
    print(json.dumps(line), flush=True)


def bench_lts(args):
    """Operator-split steps with local time stepping: the 170 x 170
    (28,900-cell) synthetic jet-flame field of the 53-species mechanism,
    each cell's dt from its CFL and diffusion limits (spread about 50x).  A
    step = chemistry of every cell over its own dt (persistent queue, cost
    order from the previous step, carried step sizes) + one transport update
    of the 54 state rows.  The field first runs --spinup untimed split
    steps (the flame settles into its steady LTS state within about 350),
    then W warm-up and K timed steps.  Per-kernel times from HIP events on
    the launch stream."""
    import torch
    import paper_2311_14941_amd as sc
    from paper_2311_14941_amd.driver import SplitDriver
    from synth.field import flame_field
    log("bench: generating the flame field")
    f = flame_field()
    n, N = f["nx"] * f["ny"], f["N"]
    mech = sc.Mechanism(f["mech"].to_text())
    launch = dict(mode="persistent", tile=1, grid=0, order="cost") if args.mode == "auto" else \
        dict(mode=args.mode, tile=args.tile, grid=0, order=args.order)
    plan = sc.Plan(mech, rtol=1e-6, atol=1e-12, linalg=args.linalg, **launch)
    d = SplitDriver(plan, f["nx"], f["ny"], f["p"], f["u"], f["dt"], f["dx"], f["D"], f["inflow_T"], f["inflow_Y"])
    dev = "cuda:0"
    T0 = torch.tensor(f["T"], device=dev)
    Y0 = torch.tensor(np.ascontiguousarray(f["Y"].T), device=dev)
    d.load(T0, Y0)
    spin = args.spinup + args.warmup
    log(f"bench: {spin} untimed split steps (spin-up to the steady LTS state + warm-up)")
    t0 = time.perf_counter()
    d.step(spin)
    torch.cuda.synchronize()
    spin_s = time.perf_counter() - t0
    steps0 = d.steps.clone()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"bench: timing {args.steps} split steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in ev:
        e[0].record(stream)
        d.chemistry()
        e[1].record(stream)
        d.transport()
        e[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chem_ms = [e[0].elapsed_time(e[1]) for e in ev]
    tr_ms = [e[1].elapsed_time(e[2]) for e in ev]
    steps = (d.steps - steps0).cpu().numpy()
    failed = int(d.failed.sum())
    flops = float(steps.sum()) * step_flops(mech.info, "ros4") / args.steps
    # where the cells and the integrator steps are: by inflow stream row and
    # by the settled local temperature
    Tset = d.T.cpu().numpy()
    zones = {"stream_jet": f["stream"] == 0, "stream_pilot": f["stream"] == 1, "stream_coflow": f["stream"] == 2,
             "T_below_600K": Tset < 600.0, "T_600_1500K": (Tset >= 600.0) & (Tset < 1500.0),
             "T_above_1500K": Tset >= 1500.0}
    by_zone = {k: {"cells_share": float(z.mean()), "steps_share": float(steps[z].sum() / max(1, steps.sum())),
                   "steps_per_cell_per_split_step": float(steps[z].mean() / args.steps) if z.any() else 0.0}
               for k, z in zones.items()}
    chem_s = float(np.mean(chem_ms)) / 1e3
    achieved = flops / chem_s / 1e12
    tr_bytes = 2 * (N + 1) * n * 8 + 2 * n * 8 + (N + 1) * f["ny"] * 8
    tr_gbs = tr_bytes / (float(np.mean(tr_ms)) / 1e3) / 1e9
    ysum = float((d.Y.sum(0) - 1.0).abs().max())
    line = {"metric": "LTS split steps: cells/s (chemistry + transport), 53-species mechanism", "unit": "cells/s",
            "value": n * args.steps / wall, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "170 x 170 synthetic jet flame (28,900 cells: fuel jet, 1880 K pilot, air "
                                   "coflow), 53-species mechanism, 1 atm, local dt = 0.5 min(dx/u, dx^2/4D) "
                                   f"({f['dt'].min():.2e}..{f['dt'].max():.2e} s), rtol 1e-6, atol 1e-12",
                       "cells": n, "launch": launch, "linalg": args.linalg,
                       "kernel": kernel_name(launch, args.linalg, mech.N), "chemistry_ms": float(np.mean(chem_ms)),
                       "transport_ms": float(np.mean(tr_ms)), "steps_per_cell_per_split_step": float(steps.mean()) / args.steps,
                       "failed_cells": failed, "max_abs_sum_Y_minus_1": ysum, "spinup_steps": args.spinup,
                       "spinup_s": spin_s, "T_max": float(d.T.max()),
                       "cells_above_1000K": int((d.T > 1000.0).sum()), "work_by_zone": by_zone},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel_ms": chem_s * 1e3,
                         "flops_per_launch": flops},
            "transport_roofline": {"bound": "hbm", "achieved": tr_gbs, "peak": 8000.0, "unit": "GB/s",
                                   "frac": tr_gbs / 8000.0, "traffic": None, "bytes_per_launch": tr_bytes}}
    # the same chemistry step from the settled state through the plain and
    # the static launch (results must be bitwise equal to the queue's)
    T1, Y1, h1 = d.T.clone(), d.Y.clone(), d.h.clone()
    cnt = (d.n_acc.clone(), d.n_rej.clone())

    def one_step(drv):
        drv.load(T1, Y1, h1)
        drv.n_acc.copy_(cnt[0])
        drv.n_rej.copy_(cnt[1])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        drv.chemistry()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b), drv.q[1].clone()

    ref_ms, ref_q = one_step(d)
    for name in ("plain", "static"):
        e = SplitDriver(sc.Plan(mech, rtol=1e-6, atol=1e-12, mode=name, linalg=args.linalg), f["nx"], f["ny"],
                        f["p"], f["u"], f["dt"], f["dx"], f["D"], f["inflow_T"], f["inflow_Y"])
        ms, q = one_step(e)
        line["config"][f"{name}_launch_chemistry_ms"] = ms
        line["config"][f"{name}_launch_identical"] = bool(torch.equal(q, ref_q))
    line["config"]["queue_chemistry_ms_same_step"] = ref_ms
    log("bench: zonal reference-cell mapping")
    line["mapping"] = lts_mapping(sc, torch, mech, f, launch, one_step, ref_q, ref_ms, T1, Y1, h1, cnt, args)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on a sample of the field")
        line["cpu_baseline"] = cpu_baseline_lts(f)
    print(json.dumps(line), flush=True)


MAP_Z_TOL, MAP_DT = 1e-3, 2.0


def lts_mapping(sc, torch, mech, f, launch, one_step, ref_q, ref_ms, T1, Y1, h1, cnt, args):
    """Zonal reference-cell mapping on the settled field: cells whose
    mixture fraction between the jet and the air stream is below 1e-3 share
    the chemistry of the lowest-index cell of their 2 K temperature band.
    From the same settled state: one chemistry step mapped against the
    unmapped one (how many cells are mapped, the time, and the change in
    the result: the mapping's approximation, measured against the parity
    bar), then K timed split steps with the mapping."""
    from paper_2311_14941_amd.driver import SplitDriver
    mp = dict(Y_fuel=f["Y_fuel"], Y_ox=f["Y_ox"], z_tol=MAP_Z_TOL, dT=MAP_DT, dlnp=0.0)
    e = SplitDriver(sc.Plan(mech, rtol=1e-6, atol=1e-12, linalg=args.linalg, **launch), f["nx"], f["ny"], f["p"],
                    f["u"], f["dt"], f["dx"], f["D"], f["inflow_T"], f["inflow_Y"], mapping=mp)
    ms, q = one_step(e)
    ref = e.ref.cpu().numpy()
    mapped = ref != np.arange(ref.size)
    N = mech.N
    a, b = ref_q.cpu().numpy(), q.cpu().numpy()
    exc = parity_excess(b[N], b[:N].T, a[N], a[:N].T)  # mapped result against the integrated one
    out = {"z_tol": MAP_Z_TOL, "dT_band_K": MAP_DT, "streams": "fuel: the jet mixture; oxidiser: air",
           "cells_mapped": int(mapped.sum()), "mapped_share": float(mapped.mean()),
           "references": int(np.unique(ref[mapped]).size),
           "chemistry_ms_same_step": ms, "unmapped_chemistry_ms_same_step": ref_ms,
           "speedup_same_step": ref_ms / ms,
           "vs_unmapped_same_step": {
               "bar": "T and Y > 1e-8 to relative 1e-6, Y <= 1e-8 to absolute 1e-12 (excess = error / bar)",
               "mapped_cells_within_bar": float(np.mean(exc[mapped] <= 1.0)) if mapped.any() else None,
               "worst_excess_mapped": float(exc[mapped].max()) if mapped.any() else None,
               "max_abs_dT_K": float(np.abs(b[N] - a[N]).max()),
               "integrated_cells_identical": bool(np.array_equal(a[:, ~mapped], b[:, ~mapped]))}}
    # K split steps with the mapping, from the settled state
    e.load(T1, Y1, h1)
    e.n_acc.copy_(cnt[0])
    e.n_rej.copy_(cnt[1])
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x in ev:
        x[0].record(stream)
        e.chemistry()
        x[1].record(stream)
        e.transport()
        x[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["split_steps_ms"] = wall * 1e3 / args.steps
    out["split_steps_cells_per_s"] = ref.size * args.steps / wall
    out["chemistry_ms"] = float(np.mean([x[0].elapsed_time(x[1]) for x in ev]))
    out["failed_cells"] = int(e.failed.sum())
    return out


def cpu_baseline_lts(f, budget_s=15.0):
    """The oracle's split step (its integrator at rtol 1e-6, then the
    reference transport) timed on a sample of the field's initial cells,
    stratified over the three streams; transport of the whole field is
    timed once and charged per cell.  The initial cells are the oracle's own
    input (it cannot spin the whole field up in minutes); they take about
    2.1 integrator steps per split step against 3.6 in the settled field."""
    from oracle.oracle import Oracle, max_threads
    from oracle.split import transport2d
    o = Oracle(f["mech"].to_text())
    threads = max_threads()
    rng = np.random.default_rng(6)
    sample = np.concatenate([rng.permutation(np.nonzero(f["stream"] == s)[0])[:4096] for s in (0, 1, 2)])
    sample = rng.permutation(sample)
    done, t_used, pos, per = 0, 0.0, 0, 8 * threads
    while t_used < budget_s and pos < sample.size:
        idx = sample[pos:pos + per]
        pos += idx.size
        t0 = time.perf_counter()
        r = o.integrate(f["T"][idx], f["p"][idx], f["Y"][idx], f["dt"][idx], rtol=1e-6, atol=1e-12,
                        nthreads=threads)
        t_used += time.perf_counter() - t0
        done += idx.size
        assert np.all(r["status"] == 0)
    q = np.vstack([f["Y"].T, f["T"][None, :]])
    inflow = np.vstack([f["inflow_Y"], f["inflow_T"][None, :]])
    t0 = time.perf_counter()
    transport2d(q, f["u"], f["dt"], f["dx"], f["D"], inflow, f["nx"], f["ny"])
    tr = (time.perf_counter() - t0) / q.shape[1]
    per_cell = t_used / done + tr
    return dict(value=1.0 / per_cell, unit="cells/s", cores=threads, kind="oracle",
                sample=f"chemistry of {done} initial cells of the field (not the settled field the GPU "
                       f"times), stratified over jet/pilot/coflow (seed 6), {t_used:.1f} s on {threads} "
                       "threads, rtol 1e-6 atol 1e-12; plus the reference transport of all 28,900 cells, "
                       "per cell")


if __name__ == "__main__":
    main()
