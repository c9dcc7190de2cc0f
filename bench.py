#!/usr/bin/env python3
"""Benchmark of the PAGANI hot path on one MI355X.

A step is one whole integration (Algorithm 2 to convergence) of the d=5
Gaussian exp(-sum a_i^2 (x_i - u_i)^2) on [0,1]^5 (a ~ U[10,25],
u ~ U[0.3,0.7], seed 2), 4^5 initial grid, rel_tol 1e-6, live list capped at
2^21 regions. Inputs (the integrand's parameters) are resident before the
timed region; each step allocates nothing (the workspace is set up once).

Prints one JSON line:
  value       integrand evaluations per second over the K timed steps
              (sum of regions evaluated x 93 points / wall time)
  roofline    the EVALUATE kernel (the method's arithmetic) against MI355X's
              FP64 vector peak, from HIP events recorded on its stream
  cpu_baseline  the CPU oracle on the same run to convergence: its parity
              build on one core and its OpenMP build on all the host's
              cores, with the host's CPU model and count
  configs     the product-peak (d=3) and oscillatory (d=8, relative-error
              filter on and off) workloads; headline_other_rules: the
              headline under the other threshold-search rules
  batched, adjoint  many integrals in one run against single runs, and
              the forward run with and without dI/dtheta (medians)

Other modes feed the profiles: --mode integrand (integrand values only, to
count one evaluation's FP64 operations with rocprofv3 counters) and
--mode copy (a plain device copy of known size, to scale FETCH_SIZE /
WRITE_SIZE). Experiments: --mode suite (the paper's f1..f8 over its
tolerance sweep, --error-rule raw or null4) and --mode errors (the two
region error estimates on peaked integrals with closed forms).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 operations of one evaluation of an integrand, counted with rocprofv3
# ((ADD + MUL + TRANS + 2 FMA)_F64 per evaluation) on the integrand-only
# kernel (--mode integrand); see profiles/integrand_flops.txt.
# Algorithmic FLOP per region = N points x (F + 1 orbit accumulation).
F_FLOP = {("gaussian", 5): 47.0, ("product_peak", 3): 20.0, ("oscillatory", 8): 73.0,
          ("corner_peak", 6): 25.0, ("gaussian", 6): 51.0}
# HBM bytes per evaluate launch of this workload from FETCH_SIZE / WRITE_SIZE
# (scaled by a plain copy), valid only for the kernel source they were taken
# on (first 16 hex digits of the sha256 of pg_eval_kernels.hpp followed by
# pg_eval_defs.hpp, comments and blank space removed); reported as null
# otherwise.
# The same counter runs give the FP64 operations the kernel executes per
# evaluation, 64 x (ADD + MUL + TRANS + 2 FMA)_F64 / evaluations: fewer than
# the algorithmic F + 1, because the kernel shares the unmoved coordinates'
# terms within a unit and the vertices' per-axis terms within a region.
EVAL_TRAFFIC = {"bytes_per_launch": 39379407.2, "kernel_sha256": "5e52acb6786c2b51",
                "fp64_flop_per_eval": 2.8541e10 / 784748322,
                "profile": "profiles/evaluate_gaussian_d5_counters.txt"}
# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
PEAK_FP64_TFLOPS = 78.6


def _kernel_sha():
    """sha256 (16 hex digits) of the evaluate kernel's source: its header and
    the definitions it is built from (rule, parameters, exponential), with
    comments and blank space removed, so that only code changes count."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("pg_eval_kernels.hpp", "pg_eval_defs.hpp"):
        src = open(os.path.join(ROOT, "paper_2104_06494_amd", "csrc", name)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def _host():
    """The host the CPU figures come from: CPU model, logical CPUs, and the
    CPUs this process may run on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _flop_per_eval(family, d):
    return F_FLOP.get((family, d))


def timed_runs(ctx, wl, steps, warmup, **kw):
    """`steps` whole integrations of `wl` after `warmup` untimed ones, each
    timed on the host (pg_integrate blocks until the result is known) with
    HIP events around its EVALUATE launches; then one more run with events
    around every phase. Returns the first timed run's result, the per-step
    wall times and the evaluate-kernel figures."""
    import torch
    for _ in range(warmup):
        ctx.integrate_workload(wl, timing=1, **kw)
    torch.cuda.synchronize()
    results, step_s = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        # HIP events around the EVALUATE launches only (the roofline's
        # duration); a full phase breakdown would add 3 events an iteration
        r = ctx.integrate_workload(wl, timing=1, **kw)
        step_s.append(time.perf_counter() - ts)
        results.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the phase breakdown, from one more run outside the timed region
    rp = ctx.integrate_workload(wl, timing=2, **kw)
    r0 = results[0]
    eval_ms = sum(r.phase_ms[0] for r in results)
    launches = sum(r.eval_launches for r in results)
    regions = sum(r.regions_evaluated for r in results)
    npts = wl.npoints
    out = {"result": r0, "wall_s": wall, "step_s": step_s,
           "fevals": sum(r.fevals for r in results),
           "eval_ms": eval_ms, "launches": launches, "regions": regions,
           "phases": list(rp.phase_ms)}
    F = _flop_per_eval(wl.family, wl.d)
    out["alg_flop"] = regions * npts * (F + 1.0) if F is not None else None
    return out


def _run_summary(wl, T, exact):
    """One workload's figures: time-to-tol (median and range over the timed
    runs), evaluations per second over the whole runs and over the EVALUATE
    launches, the evaluate kernel against the FP64 vector peak, the phases
    of one run, and the result against the closed form."""
    r = T["result"]
    out = {"time_to_tol_ms": 1e3 * statistics.median(T["step_s"]),
           "time_to_tol_ms_min": 1e3 * min(T["step_s"]),
           "time_to_tol_ms_max": 1e3 * max(T["step_s"]),
           "runs": len(T["step_s"]),
           "evals_per_s": T["fevals"] / T["wall_s"],
           "eval_evals_per_s": T["regions"] * wl.npoints / (T["eval_ms"] * 1e-3),
           "status": r.status_name, "estimate": r.estimate, "error": r.error,
           "true_rel_err": abs(r.estimate - exact) / abs(exact),
           "est_rel_err": r.error / abs(r.estimate),
           "iterations": r.iterations, "regions_evaluated": r.regions_evaluated,
           "peak_regions": r.peak_regions, "threshold_calls": r.threshold_calls,
           "threshold_trials": r.threshold_trials,
           "eval_launches_per_run": T["launches"] / len(T["step_s"]),
           "phase_ms_one_run": dict(zip(("evaluate", "post_process",
                                         "threshold_and_host", "filter_split"),
                                        T["phases"]))}
    if T["alg_flop"] is not None:
        achieved = T["alg_flop"] / (T["eval_ms"] * 1e-3) / 1e12
        out["evaluate_tflops"] = achieved
        out["evaluate_frac_fp64_peak"] = achieved / PEAK_FP64_TFLOPS
    return out


def headline(args):
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.gaussian_d5()
    npts = wl.npoints
    torch.cuda.set_device(0)
    exact = cf.exact(wl.family, wl.params, wl.d)
    with pg.Context(capacity=wl.max_regions, dim_max=wl.d) as ctx:
        T = timed_runs(ctx, wl, args.steps, args.warmup)
        # the same workload under the other threshold-search rules (the P_max
        # rule of Section 3.5.3 without a reserve for the active regions, and
        # the memory-only P_max rule, a departure from that section)
        rules = {}
        if not args.no_configs:
            for name, kw in (("paper_pmax_listing_budget",
                              dict(pmax_relax="paper", budget="listing")),
                             ("memory_only_pmax_reserve_budget",
                              dict(pmax_relax="memory", budget="reserve"))):
                rules[name] = _run_summary(wl, timed_runs(ctx, wl, 5, 1, **kw), exact)

    r0 = T["result"]
    value = T["fevals"] / T["wall_s"]
    launches = T["launches"]
    achieved = T["alg_flop"] / (T["eval_ms"] * 1e-3) / 1e12
    key_ok = _kernel_sha() == EVAL_TRAFFIC["kernel_sha256"]
    executed = (T["regions"] * npts * EVAL_TRAFFIC["fp64_flop_per_eval"]
                / (T["eval_ms"] * 1e-3) / 1e12) if key_ok else None
    summ = _run_summary(wl, T, exact)
    out = {
        "metric": "FP64 integrand evals/s + time-to-tol at 1e-6; batched & adjoint vs plain, 1 GPU",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gaussian_d5_tol1e-6", "family": "gaussian", "d": 5,
                   "rel_tol": wl.rel_tol, "init_grid": "4^5",
                   "max_regions": wl.max_regions, "points_per_region": npts,
                   "seed": 2, "pmax_relax": "paper", "budget": "reserve",
                   "error_rule": "raw"},
        "time_to_tol_ms": summ["time_to_tol_ms"],
        "result": {k: summ[k] for k in ("status", "estimate", "error", "true_rel_err",
                                        "iterations", "regions_evaluated",
                                        "peak_regions", "threshold_calls",
                                        "threshold_trials")},
        "phase_ms_one_run": {**summ["phase_ms_one_run"],
                             "note": "one run after the timed steps, 5 HIP events an iteration"},
        "roofline": {
            "kernel": "k_evaluate<gaussian,5>",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "frac_basis": "algorithmic: evaluations x (F_f + 1) FP64 FLOP",
            "executed_fp64_frac": (executed / PEAK_FP64_TFLOPS
                                   if executed is not None else None),
            "executed_fp64_basis": "FP64 operations the kernel executes per "
                                   "evaluation, from rocprofv3 counters of this "
                                   "kernel source",
            "traffic": EVAL_TRAFFIC["bytes_per_launch"] if key_ok else None,
            "traffic_unit": "HBM bytes per launch",
            "avg_launch_ms": T["eval_ms"] / launches,
            "alg_flop_per_launch": T["alg_flop"] / launches,
            "eval_evals_per_s": summ["eval_evals_per_s"],
        },
    }
    if rules:
        out["headline_other_rules"] = rules
    if not args.no_configs:
        out["configs"] = other_configs(args)
    if not args.no_batched:
        out["batched"] = batched(args)
    if not args.no_adjoint:
        out["adjoint"] = adjoint(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


def other_configs(args):
    """The small product peak (d=3 to 1e-3, 4^3 grid) and the oscillatory
    integrand (d=8 to 1e-5, 2^8 grid, with the relative-error filter on and
    off): median time-to-tol over 7 runs after 2 warm-up runs, evaluations
    per second, the evaluate kernel's fraction of the FP64 peak, phases."""
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    out = {}
    for name, wl in (("product_peak_d3_tol1e-3", W.product_peak_d3()),
                     ("oscillatory_d8_tol1e-5_relerr_on", W.oscillatory_d8(1)),
                     ("oscillatory_d8_tol1e-5_relerr_off", W.oscillatory_d8(0))):
        exact = cf.exact(wl.family, wl.params, wl.d)
        with pg.Context(capacity=wl.max_regions, dim_max=wl.d) as ctx:
            out[name] = _run_summary(wl, timed_runs(ctx, wl, 7, 2), exact)
        torch.cuda.empty_cache()
    return out


def _median_runs(fn, reps):
    """fn() `reps` times, each bracketed by device synchronisations; returns
    (last result, median seconds, all seconds)."""
    import torch
    ts, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return res, statistics.median(ts), ts


def batched(args):
    """The 1024 d=6 corner-peak integrals (per-integral a ~ U[0,2]^6 and
    rel_tol 10^U[-7,-4], seed 4, 2^6 initial grid, 2^21-region cap each)
    as one batched run and as 1024 single runs one after another, on the
    same context (median of --reps runs each, after one warm-up of the
    batched run). Both give the same results."""
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.corner_peak_batch_d6()
    B = min(wl.B, args.batch_count) if args.batch_count else wl.B
    slots = args.batch_slots
    with pg.Context(capacity=slots * wl.max_regions, dim_max=wl.d) as ctx:
        if args.eval_waves:
            ctx.set_eval_waves(args.eval_waves)
        if not args.no_batch_warmup:
            ctx.integrate_batch_workload(wl, count=min(B, 2 * slots))
        rb, tb, tbs = _median_runs(lambda: ctx.integrate_batch_workload(wl, count=B),
                                   args.reps)
        fe = sum(r.fevals for r in rb)
        met, misses = 0, []
        for b, r in enumerate(rb):
            exact = cf.exact(wl.family, wl.params[b], wl.d)
            rel = abs(r.estimate - exact) / (wl.rel_tol[b] * abs(exact))
            met += rel <= 1.0
            if rel > 1.0:
                # true error over tau, reported error over tau, status
                misses.append([b, round(rel, 3),
                               round(r.error / (wl.rel_tol[b] * abs(r.estimate)), 3),
                               r.status_name, float(wl.rel_tol[b])])
        out = {"workload": "corner_peak_batch_d6", "B": B, "slots_in_flight": slots,
               "evals_per_s": fe / tb, "wall_ms": 1e3 * tb,
               "wall_ms_runs": [1e3 * t for t in tbs], "fevals": fe,
               "status_ok": sum(r.status_name == "OK" for r in rb),
               "closed_form_met": int(met),
               "closed_form_misses": misses,
               "regions_evaluated": sum(r.regions_evaluated for r in rb),
               "max_iterations": max(r.iterations for r in rb)}
        if not args.no_plain:
            rp, tp, tps = _median_runs(
                lambda: [ctx.integrate_workload(wl.instance(b)) for b in range(B)],
                args.reps)
            out["plain_sequential"] = {"evals_per_s": fe / tp, "wall_ms": 1e3 * tp,
                                       "wall_ms_runs": [1e3 * t for t in tps]}
            out["speedup_vs_plain"] = tp / tb
            out["same_schedule_as_plain"] = sum(
                (a.status, a.iterations, a.regions_evaluated) ==
                (b.status, b.iterations, b.regions_evaluated) for a, b in zip(rb, rp))
    torch.cuda.empty_cache()
    return out


def _grad_scaled_error(G, ref, I, params, d):
    """Largest |dI/dtheta - closed form| over the parameters, in units of
    tau-free scale |ref_k| + |I| / s_k, s_k the parameter's natural scale
    (a_k for a width parameter a_k, the Gaussian's width 1 / a_k for a
    centre u_k): the run bounds the estimate's error by tau |I|, and on a
    fixed partition that error moves by about itself when a parameter moves
    by its scale."""
    import numpy as np
    a = np.abs(np.asarray(params[:d]))
    scale = np.concatenate([a, 1.0 / a])
    return float(np.max(np.abs(G - ref) / (np.abs(ref) + abs(I) / scale)))


def adjoint(args):
    """Gaussian parameter points, d=6 (a ~ U[5,20]^6, u ~ U[0.2,0.8]^6, seed
    5, 2^6 initial grid), batched: forward only, then forward plus the
    derivative over each final partition (same decisions, so the same
    regions), medians of --reps runs; and the forward as single runs. Also
    how many estimates meet the closed form and how far the gradients are
    from theirs (relative to the tolerance, on the scale of
    _grad_scaled_error)."""
    import numpy as np
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.gaussian_grad_d6(rel_tol=args.adjoint_tol)
    if args.adjoint_cap:
        wl.max_regions = args.adjoint_cap
    B = min(wl.B, args.adjoint_count) if args.adjoint_count else wl.B
    slots = max(1, min(args.batch_slots // 2, args.adjoint_capacity // wl.max_regions))
    kw = dict(error_rule=args.adjoint_error_rule)
    with pg.Context(capacity=slots * wl.max_regions, dim_max=wl.d) as ctx:
        if not args.no_batch_warmup:
            ctx.integrate_batch_workload(wl, count=min(B, slots), grad=True, **kw)
        rf, tf, tfs = _median_runs(
            lambda: ctx.integrate_batch_workload(wl, count=B, **kw), args.reps)
        (rg, G, _), tg, tgs = _median_runs(
            lambda: ctx.integrate_batch_workload(wl, count=B, grad=True, **kw),
            args.reps)
        fe = sum(r.fevals for r in rf)
        same = sum((a.status, a.regions_evaluated, a.estimate) ==
                   (b.status, b.regions_evaluated, b.estimate) for a, b in zip(rf, rg))
        est_ok, gerr = 0, []
        for b in range(B):
            I, dA, dU = cf.gaussian_grad(wl.params[b], wl.d)
            ref = np.concatenate([dA, dU])
            tau = wl.rel_tol[b]
            est_ok += abs(rg[b].estimate - I) <= tau * abs(I)
            gerr.append(_grad_scaled_error(G[b], ref, I, wl.params[b], wl.d) / tau)
        gerr = np.array(gerr)
        ok = np.array([r.status_name == "OK" for r in rg])
        # The derivative pass evaluates the integrand and its 2d parameter
        # derivatives at every point of each final partition. Every
        # evaluated region is either a leaf of that partition or was split
        # into two evaluated children, so leaves = (evaluated + initial)/2.
        # Work per point: F_f + 1 for the value and its weight, 4 per
        # parameter (derivative factor, product with f, weight, sum).
        init = wl.init_splits ** wl.d
        leaves = sum((r.regions_evaluated + init) // 2 for r in rg)
        pts = leaves * (2 ** wl.d + 2 * wl.d * wl.d + 2 * wl.d + 1)
        adj_flop = pts * (F_FLOP[("gaussian", wl.d)] + 1 + 4 * 2 * wl.d)
        adj_s = max(tg - tf, 1e-9)
        out = {"workload": "gaussian_grad_d6", "B": B, "slots_in_flight": slots,
               "rel_tol": float(wl.rel_tol[0]), "max_regions": wl.max_regions,
               "error_rule": args.adjoint_error_rule,
               "forward": {"evals_per_s": fe / tf, "wall_ms": 1e3 * tf,
                           "wall_ms_runs": [1e3 * t for t in tfs]},
               "forward_adjoint": {"evals_per_s": fe / tg, "wall_ms": 1e3 * tg,
                                   "wall_ms_runs": [1e3 * t for t in tgs]},
               "adjoint_overhead": tg / tf - 1.0, "fevals": fe,
               "same_run_with_adjoint": same,
               "status": {s: int(sum(r.status_name == s for r in rg))
                          for s in sorted({r.status_name for r in rg})},
               "estimate_meets_closed_form": int(est_ok),
               "gradient_scaled_err_over_tau": {
                   "median": float(np.median(gerr)), "max": float(gerr.max()),
                   "max_converged": float(gerr[ok].max()) if ok.any() else None,
                   "within_1": int((gerr <= 1).sum()),
                   "within_10": int((gerr <= 10).sum())},
               "adjoint_roofline": {
                   "bound": "alu", "achieved": adj_flop / adj_s / 1e12,
                   "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                   "frac": adj_flop / adj_s / 1e12 / PEAK_FP64_TFLOPS,
                   "leaves": int(leaves), "points": int(pts),
                   "flop_per_point": F_FLOP[("gaussian", wl.d)] + 1 + 8 * wl.d,
                   "time": "forward+derivative wall time minus forward wall "
                           "time (includes the derivative reduction and its copies)"}}
        if not args.no_plain:
            t0 = time.perf_counter()
            for b in range(B):
                ctx.integrate_workload(wl.instance(b), **kw)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            out["plain_sequential"] = {"evals_per_s": fe / tp, "wall_ms": 1e3 * tp}
    torch.cuda.empty_cache()
    return out


def adjoint_mode(args):
    """The adjoint comparison alone (for profiling)."""
    print(json.dumps({"mode": "adjoint", **adjoint(args)}), flush=True)


def suite_mode(args):
    """The paper's test suite (Section 4.1, f1..f8) over its tolerance sweep
    (1e-3 down to 1.024e-10, a fifth at a time), each integrand until its
    first run that does not converge, as the paper reports it; then the
    filtering ablation (threshold search off) on the same sweep for the
    5-d f4. One JSON line per run. Context of --suite-capacity regions
    (default 2^28, 80 GB at d=8)."""
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    torch.cuda.set_device(0)
    ctx = pg.Context(capacity=args.suite_capacity, dim_max=8)
    try:
        _suite_sweep(args, ctx)
    finally:
        ctx.close()


def _suite_sweep(args, ctx):
    import torch
    import workloads as W
    from workloads import closed_forms as cf
    tols = W.paper_tolerances()
    runs = [(name, wl, 1) for name, wl in W.paper_suite()]
    runs += [(name + "_no_threshold", wl, 0) for name, wl in W.paper_suite()
             if name == "f4_d5"]
    for name, wl, thr in runs:
        if args.suite_only and not name.startswith(args.suite_only):
            continue
        ex = cf.exact(wl.family, wl.params, wl.d)
        ctx.integrate_workload(wl, rel_tol=tols[0], max_regions=0, threshold_filter=thr,
                               error_rule=args.error_rule)
        for tol in tols:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.integrate_workload(wl, rel_tol=tol, max_regions=0, threshold_filter=thr,
                                       error_rule=args.error_rule)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            print(json.dumps({"mode": "suite", "integrand": name, "rel_tol": tol,
                              "error_rule": args.error_rule,
                              "status": r.status_name, "estimate": r.estimate,
                              "true_rel_err": abs(r.estimate - ex) / abs(ex),
                              "est_rel_err": r.error / abs(r.estimate),
                              "ms": ms, "iterations": r.iterations,
                              "regions_evaluated": r.regions_evaluated,
                              "peak_regions": r.peak_regions, "evals_per_s":
                              r.fevals / (ms * 1e-3)}), flush=True)
            if r.status_name != "OK":
                break


def errors_mode(args):
    """The two region error estimates (|R7 - R5| and the four null rules)
    on sharply peaked integrals with closed forms, through the batched
    driver: per family, dimension, tolerance and estimate, the share of
    runs that converge, of runs whose reported error bounds the true error
    (every run, whatever its status), of converged runs that meet the
    tolerance, and the regions and time spent. One JSON line each."""
    import numpy as np
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    torch.cuda.set_device(0)
    with pg.Context(capacity=args.batch_slots << 20, dim_max=8) as ctx:
        _errors_sweep(args, ctx)


def _errors_sweep(args, ctx):
    import numpy as np
    import torch
    import workloads as W
    from workloads import closed_forms as cf
    for family, d in (("gaussian", 5), ("gaussian", 8), ("product_peak", 5),
                      ("product_peak", 8)):
        wl = W.peaked_batch(family, d, B=args.errors_batch)
        exact = np.array([cf.exact(family, p, d) for p in wl.params])
        for tol in (1e-3, 1e-4, 1e-5, 1e-6):
            for rule in ("raw", "null4"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.integrate_batch(family, d, wl.params, tol, init_splits=2,
                                          max_regions=wl.max_regions, error_rule=rule)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0)
                est = np.array([r.estimate for r in res])
                err = np.array([r.error for r in res])
                ok = np.array([r.status_name == "OK" for r in res])
                true = np.abs(est - exact)
                print(json.dumps({
                    "mode": "errors", "workload": wl.name, "rel_tol": tol,
                    "error_rule": rule, "B": wl.B, "converged": int(ok.sum()),
                    "error_bounds_true": int((true <= err).sum()),
                    "converged_meet_tol": int((true[ok] <= tol * np.abs(exact[ok])).sum()),
                    "median_true_over_tol": float(np.median(true / (tol * np.abs(exact)))),
                    "regions_evaluated": int(sum(r.regions_evaluated for r in res)),
                    "ms": ms}), flush=True)


def autotune_mode(args):
    """The autotuner over the corner-peak batch: EVALUATE's wave target x
    integrals in flight, median of --reps runs each, and the fastest."""
    import torch
    import workloads as W
    from paper_2104_06494_amd import autotune
    torch.cuda.set_device(0)
    wl = W.corner_peak_batch_d6()
    out = autotune.tune_batched(wl, count=args.batch_count or None, reps=args.reps)
    print(json.dumps({"mode": "autotune", "workload": "corner_peak_batch_d6", **out}),
          flush=True)


def batched_mode(args):
    """The batched comparison alone (for profiling)."""
    print(json.dumps({"mode": "batched", **batched(args)}), flush=True)


def cpu_baseline(wl):
    """The CPU oracle on the whole headline run (to convergence, the same
    options and cap): the parity build on one core, then its OpenMP build
    (region evaluation shared out over the host's cores, the same results)
    on every core this process may use; the host they ran on."""
    import oracle
    r = oracle.integrate_workload(wl)
    out = {"value": r.fevals / r.seconds, "unit": "evals/s", "cores": 1,
           "kind": "oracle",
           "sample": f"the whole run to convergence ({r.status_name}, {r.iterations} "
                     f"iterations, {r.regions_evaluated} regions, {r.fevals} "
                     f"evaluations) in {r.seconds:.1f} s",
           "time_to_tol_ms": 1e3 * r.seconds, "status": r.status_name,
           "host": _host()}
    rp = oracle.integrate_workload(wl, parallel=True)
    out["all_cores"] = {"value": rp.fevals / rp.seconds, "unit": "evals/s",
                        "cores": oracle.threads(True), "kind": "oracle (OpenMP build)",
                        "time_to_tol_ms": 1e3 * rp.seconds,
                        "same_result": (rp.estimate, rp.error, rp.iterations) ==
                                       (r.estimate, r.error, r.iterations)}
    return out


def integrand_mode(args):
    """f alone at 2^22 points, for counting an evaluation's FP64 operations
    (--integrand: one of the workloads' integrands)."""
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    torch.cuda.set_device(0)
    wl = {"gaussian_d5": W.gaussian_d5, "product_peak_d3": W.product_peak_d3,
          "oscillatory_d8": lambda: W.oscillatory_d8(1),
          "corner_peak_d6": lambda: W.corner_peak_batch_d6().instance(0),
          "gaussian_d6": lambda: W.gaussian_grad_d6().instance(0)}[args.integrand]()
    n = 1 << 22
    x = torch.rand(wl.d, n, dtype=torch.float64, device="cuda")
    with pg.Context(capacity=1 << 10, dim_max=wl.d) as ctx:
        for _ in range(args.warmup + args.steps):
            y = ctx.integrand_values(wl.family, wl.params, x)
        torch.cuda.synchronize()
    print(json.dumps({"mode": "integrand", "integrand": args.integrand, "points": n,
                      "launches": args.warmup + args.steps,
                      "checksum": float(y.sum())}), flush=True)


def copy_mode(args):
    """A plain device copy of 2^28 bytes, for scaling the HBM byte counters."""
    import torch
    torch.cuda.set_device(0)
    nbytes = 1 << 28
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup + args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": nbytes,
                      "bytes_written_per_launch": nbytes,
                      "launches": args.warmup + args.steps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["headline", "batched", "adjoint", "suite",
                                       "errors", "integrand", "copy", "autotune"],
                    default="headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads and threshold-search rules")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward-vs-forward+adjoint comparison")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched run without the single-run comparison")
    ap.add_argument("--batch-count", type=int, default=0,
                    help="first integrals of the batch only (0 = all 1024)")
    ap.add_argument("--suite-capacity", type=int, default=1 << 28,
                    help="regions of the context the suite sweep runs in "
                         "(2^28: 80 GB at d=8)")
    ap.add_argument("--suite-only", default="",
                    help="suite integrands whose name starts with this only")
    ap.add_argument("--error-rule", default="raw", choices=["raw", "null4"],
                    help="region error estimate of the suite sweep")
    ap.add_argument("--errors-batch", type=int, default=128,
                    help="integrals per family and tolerance in --mode errors")
    ap.add_argument("--integrand", default="gaussian_d5",
                    choices=["gaussian_d5", "product_peak_d3", "oscillatory_d8",
                             "corner_peak_d6", "gaussian_d6"],
                    help="integrand of --mode integrand")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs of the batched and derivative comparisons "
                         "(medians reported)")
    ap.add_argument("--adjoint-tol", type=float, default=1e-5,
                    help="rel_tol of the derivative workload")
    ap.add_argument("--adjoint-cap", type=int, default=0,
                    help="region cap per integral of the derivative workload "
                         "(0: the workload's 2^22)")
    ap.add_argument("--adjoint-count", type=int, default=0,
                    help="first parameter points only (0 = all 256)")
    ap.add_argument("--adjoint-capacity", type=int, default=1 << 27,
                    help="regions of the derivative run's context (integrals "
                         "in flight: this / the cap, at most half of "
                         "--batch-slots)")
    ap.add_argument("--adjoint-error-rule", default="raw", choices=["raw", "null4"])
    ap.add_argument("--eval-waves", type=int, default=0,
                    help="EVALUATE's wave target in the batched run (0: the "
                         "library's default)")
    ap.add_argument("--no-batch-warmup", action="store_true",
                    help="skip the warm-up of the batched and derivative runs "
                         "(a kernel trace then covers only the reported runs)")
    ap.add_argument("--batch-slots", type=int, default=64,
                    help="integrals in flight in the batched run (each "
                         "reserves 2^21 regions of workspace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not "
              "supported (how the method would shard over several GPUs is described "
              "in the design notes, not implemented)", file=sys.stderr)
        sys.exit(2)
    {"headline": headline, "batched": batched_mode, "adjoint": adjoint_mode,
     "suite": suite_mode, "errors": errors_mode, "integrand": integrand_mode,
     "copy": copy_mode, "autotune": autotune_mode}[args.mode](args)


if __name__ == "__main__":
    main()
