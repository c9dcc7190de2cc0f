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
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the
              same workload: the first 12 iterations of the same run

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

# FP64 operations of one Gaussian evaluation in 5 dimensions, counted with
# rocprofv3 ((ADD + MUL + TRANS + 2 FMA)_F64 per evaluation) on the
# integrand-only kernel; see profiles/evaluate_gaussian_d5_counters.txt.
# Algorithmic FLOP per region = 93 points x (F + 1 orbit accumulation).
F_GAUSSIAN_D5 = 47.0
# HBM bytes per evaluate launch of this workload from FETCH_SIZE / WRITE_SIZE
# (scaled by a plain copy), valid only for the kernel source they were taken
# on (first 16 hex digits of the sha256 of pg_eval_kernels.hpp followed by
# pg_eval_defs.hpp, comments and blank space removed); reported as null
# otherwise.
EVAL_TRAFFIC = {"bytes_per_launch": 37759311.2, "kernel_sha256": "ca1f2b37fe775935",
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


def headline(args):
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.gaussian_d5()
    npts = wl.npoints
    torch.cuda.set_device(0)
    ctx = pg.Context(capacity=wl.max_regions, dim_max=wl.d)
    for _ in range(args.warmup):
        ctx.integrate_workload(wl, timing=1)
    torch.cuda.synchronize()
    results, step_s = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        # HIP events around the EVALUATE launches only (the roofline's
        # duration); a full phase breakdown would add 3 events an iteration
        r = ctx.integrate_workload(wl, timing=1)
        step_s.append(time.perf_counter() - ts)
        results.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the phase breakdown, from one more run outside the timed region
    rp = ctx.integrate_workload(wl, timing=2)

    fevals = sum(r.fevals for r in results)
    value = fevals / wall
    r0 = results[0]
    exact = cf.exact(wl.family, wl.params, wl.d)
    eval_ms = sum(r.phase_ms[0] for r in results)
    launches = sum(r.eval_launches for r in results)
    regions = sum(r.regions_evaluated for r in results)
    alg_flop = regions * npts * (F_GAUSSIAN_D5 + 1.0)
    achieved = alg_flop / (eval_ms * 1e-3) / 1e12
    phases = list(rp.phase_ms)
    out = {
        "metric": "FP64 integrand evals/s + time-to-tol at 1e-6; batched & adjoint vs plain, 1 GPU",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gaussian_d5_tol1e-6", "family": "gaussian", "d": 5,
                   "rel_tol": wl.rel_tol, "init_grid": "4^5",
                   "max_regions": wl.max_regions, "points_per_region": npts,
                   "seed": 2},
        "time_to_tol_ms": 1e3 * statistics.median(step_s),
        "result": {"status": r0.status_name, "estimate": r0.estimate,
                   "error": r0.error, "true_rel_err": abs(r0.estimate - exact) / abs(exact),
                   "iterations": r0.iterations, "regions_evaluated": r0.regions_evaluated,
                   "peak_regions": r0.peak_regions, "fevals": r0.fevals,
                   "threshold_calls": r0.threshold_calls,
                   "threshold_trials": r0.threshold_trials},
        "phase_ms_one_run": {"evaluate": phases[0], "post_process": phases[1],
                             "threshold_and_host": phases[2], "filter_split": phases[3],
                             "note": "one run after the timed steps, 5 HIP events an iteration"},
        "roofline": {
            "kernel": "k_evaluate<gaussian,5>",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": (EVAL_TRAFFIC["bytes_per_launch"]
                        if _kernel_sha() == EVAL_TRAFFIC["kernel_sha256"] else None),
            "traffic_unit": "HBM bytes per launch",
            "avg_launch_ms": eval_ms / launches,
            "alg_flop_per_launch": alg_flop / launches,
            "eval_evals_per_s": regions * npts / (eval_ms * 1e-3),
        },
    }
    if not args.no_batched:
        out["batched"] = batched(args)
    if not args.no_adjoint:
        out["adjoint"] = adjoint(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


def batched(args):
    """The 1024 d=6 corner-peak integrals (per-integral a ~ U[0,2]^6 and
    rel_tol 10^U[-7,-4], seed 4, 2^6 initial grid, 2^21-region cap each)
    as one batched run and as 1024 single runs one after another, on the
    same context. Both give the same results; evals/s and wall time of
    each (one untimed warm-up of the batched run first)."""
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.corner_peak_batch_d6()
    B = min(wl.B, args.batch_count) if args.batch_count else wl.B
    slots = args.batch_slots
    ctx = pg.Context(capacity=slots * wl.max_regions, dim_max=wl.d)
    ctx.integrate_batch_workload(wl, count=min(B, 2 * slots))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = ctx.integrate_batch_workload(wl, count=B)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    fe = sum(r.fevals for r in rb)
    met = 0
    for b, r in enumerate(rb):
        exact = cf.exact(wl.family, wl.params[b], wl.d)
        met += abs(r.estimate - exact) <= wl.rel_tol[b] * abs(exact)
    out = {"workload": "corner_peak_batch_d6", "B": B, "slots_in_flight": slots,
           "evals_per_s": fe / tb, "wall_ms": 1e3 * tb, "fevals": fe,
           "status_ok": sum(r.status_name == "OK" for r in rb),
           "closed_form_met": int(met),
           "regions_evaluated": sum(r.regions_evaluated for r in rb),
           "max_iterations": max(r.iterations for r in rb)}
    if not args.no_plain:
        t0 = time.perf_counter()
        rp = [ctx.integrate_workload(wl.instance(b)) for b in range(B)]
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["plain_sequential"] = {"evals_per_s": fe / tp, "wall_ms": 1e3 * tp}
        out["speedup_vs_plain"] = tp / tb
        out["same_schedule_as_plain"] = sum(
            (a.status, a.iterations, a.regions_evaluated) ==
            (b.status, b.iterations, b.regions_evaluated) for a, b in zip(rb, rp))
    ctx.close()
    torch.cuda.empty_cache()
    return out


def adjoint(args):
    """The 256 d=6 Gaussian parameter points (a ~ U[5,20]^6, u ~ U[0.2,0.8]^6,
    seed 5, rel_tol 1e-5, 2^6 initial grid, 2^22-region cap each), batched:
    forward only, then forward plus the derivative over each final
    partition (same decisions, so the same regions); and the forward as 256
    single runs. Also how many estimates and gradients meet the closed form."""
    import numpy as np
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    from workloads import closed_forms as cf

    wl = W.gaussian_grad_d6()
    B = min(wl.B, args.batch_count) if args.batch_count else wl.B
    slots = max(1, args.batch_slots // 2)
    ctx = pg.Context(capacity=slots * wl.max_regions, dim_max=wl.d)
    ctx.integrate_batch_workload(wl, count=min(B, slots), grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rf = ctx.integrate_batch_workload(wl, count=B)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    rg, G, _ = ctx.integrate_batch_workload(wl, count=B, grad=True)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    fe = sum(r.fevals for r in rf)
    same = sum((a.status, a.regions_evaluated, a.estimate) ==
               (b.status, b.regions_evaluated, b.estimate) for a, b in zip(rf, rg))
    est_ok = grad_ok = 0
    gerr = []
    for b in range(B):
        I, dA, dU = cf.gaussian_grad(wl.params[b], wl.d)
        ref = np.concatenate([dA, dU])
        tau = wl.rel_tol[b]
        est_ok += abs(rg[b].estimate - I) <= tau * abs(I)
        e = float(np.max(np.abs(G[b] - ref)) / np.max(np.abs(ref)))
        gerr.append(e)
        grad_ok += e <= 100 * tau
    out = {"workload": "gaussian_grad_d6", "B": B, "slots_in_flight": slots,
           "rel_tol": float(wl.rel_tol[0]),
           "forward": {"evals_per_s": fe / tf, "wall_ms": 1e3 * tf},
           "forward_adjoint": {"evals_per_s": fe / tg, "wall_ms": 1e3 * tg},
           "adjoint_overhead": tg / tf - 1.0, "fevals": fe,
           "same_run_with_adjoint": same,
           "status_ok": sum(r.status_name == "OK" for r in rg),
           "estimate_meets_closed_form": int(est_ok),
           "gradient_within_100tau_of_closed_form": int(grad_ok),
           "median_gradient_rel_err": float(np.median(gerr))}
    if not args.no_plain:
        t0 = time.perf_counter()
        for b in range(B):
            ctx.integrate_workload(wl.instance(b))
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["plain_sequential"] = {"evals_per_s": fe / tp, "wall_ms": 1e3 * tp}
    ctx.close()
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
    ctx.close()


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
    ctx = pg.Context(capacity=args.batch_slots << 20, dim_max=8)
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
    ctx.close()


def batched_mode(args):
    """The batched comparison alone (for profiling)."""
    print(json.dumps({"mode": "batched", **batched(args)}), flush=True)


def cpu_baseline(wl):
    """The CPU oracle, single-threaded, on the first 12 iterations of the same
    run (about 2e6 regions x 93 points)."""
    import oracle
    r = oracle.integrate_workload(wl, max_iters=12)
    return {"value": r.fevals / r.seconds, "unit": "evals/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first 12 iterations of the same run: {r.regions_evaluated} "
                      f"regions, {r.fevals} evaluations, {r.seconds:.1f} s"}


def integrand_mode(args):
    """f alone at 2^22 points, for counting an evaluation's FP64 operations."""
    import numpy as np
    import torch
    import paper_2104_06494_amd as pg
    import workloads as W
    torch.cuda.set_device(0)
    wl = W.gaussian_d5()
    n = 1 << 22
    x = torch.rand(wl.d, n, dtype=torch.float64, device="cuda")
    ctx = pg.Context(capacity=1 << 10, dim_max=wl.d)
    for _ in range(args.warmup + args.steps):
        y = ctx.integrand_values(wl.family, wl.params, x)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "integrand", "points": n, "launches": args.warmup + args.steps,
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
                                       "errors", "integrand", "copy"],
                    default="headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
     "copy": copy_mode}[args.mode](args)


if __name__ == "__main__":
    main()
