"""A small autotuner for the launch choices of the many-integral driver.

Two choices change how fast a batched run goes without changing what it
computes (every integral takes the same decisions; estimates move only by
the order of floating-point sums):

* the waves EVALUATE aims to keep in flight (blocks x waves per block; the
  library's default is 2048, the chip twice over), and
* the integrals in flight at once, set by the context's capacity (each
  integral in flight reserves its region cap of the workspace).

tune_batched() times every pair on the workload itself (the first `count`
integrals), median of `reps` runs after a warm-up, and returns the fastest.
The wave target changes the order in which a block's waves add their
partial sums, so an integral whose classification sits on a rounding tie
can take another schedule; each row counts the integrals whose schedule
(status, iterations, regions evaluated) differs from the first setting's.
The segment length of the list kernels is a compile-time constant and is
not tuned here.
"""
from __future__ import annotations

import statistics
import time

import torch

from .api import Context


def _schedule(results):
    return [(r.status, r.iterations, r.regions_evaluated) for r in results]


def tune_batched(wl, count=None, wave_targets=(1024, 2048, 4096, 8192),
                 slots=(16, 32, 64), reps=3, **kw):
    """Times wl.integrate_batch over the grid wave_targets x slots and
    returns {"best": {...}, "table": [...], "B": integrals}; keyword
    arguments go to the integrator."""
    B = wl.B if count is None else min(int(count), wl.B)
    table, ref = [], None
    for s in slots:
        with Context(capacity=int(s) * wl.max_regions, dim_max=wl.d) as ctx:
            for wt in wave_targets:
                ctx.set_eval_waves(int(wt))
                ctx.integrate_batch_workload(wl, count=min(B, 2 * int(s)), **kw)
                times = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = ctx.integrate_batch_workload(wl, count=B, **kw)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                sched = _schedule(res)
                if ref is None:
                    ref = sched
                table.append({"slots": int(s), "wave_target": int(wt),
                              "ms": 1e3 * statistics.median(times),
                              "ms_runs": [1e3 * t for t in times],
                              "schedule_diffs": sum(a != b for a, b in zip(sched, ref))})
        torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    return {"best": best, "table": table, "B": B}
