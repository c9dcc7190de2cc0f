"""Algorithm 2 driven from Python through the oracle's step functions, for
testing the oracle's replay mode on the CPU.

The driver takes the steps of the main loop (Section 3.1, Algorithm 2) in
the paper's order -- Evaluate, Two-Level-Error, Rel-Err-Classify, the sums,
the termination test, Threshold-Classify when one of the two triggers of
Section 3.5.2 holds, the finished sums, Filter + Split -- each through one
call of the oracle library (no arithmetic of the method is repeated here
beyond the scalar updates the listing itself spells out), and writes the
decision trace a GPU run writes (see the trace description in the library
header). Left alone it reproduces the oracle's free run bit for bit, and its
trace replays without a single override. A `plant` dict changes one
decision at one iteration, and the run continues from the changed decision
exactly as a GPU that had taken it would, so that the replay must report
the change as an uncertified difference:

  axis=(it, i, k)   region i's split axis becomes k
  flip=(it, i)      region i's final active flag is inverted
  trigger=it        the threshold search is invoked iff it was not
  search=it         an accepted search is recorded as failed (A = A_rel)
  trials=it         the search's trial count is recorded one higher
  tshift=it         the accepted threshold is recorded 1.5 times larger
  stop=it           the run is recorded as converged at iteration it
"""
from __future__ import annotations

import math
import struct

import numpy as np

import oracle

_REC = struct.Struct("<qqqiiiiddddd")
STATUS_OK, MAX_ITERS, MEMORY_EXHAUSTED, NO_ACTIVE = 0, 1, 2, 3


def run(family, d, params, *, rel_tol, abs_tol=1e-20, init_splits=4,
        max_iters=100, relerr_filter=1, threshold_filter=1,
        max_regions=1 << 22, error_rule="raw", pmax_relax="paper",
        budget="reserve", trace_path=None, plant=None, log=None):
    """Returns dict(estimate, error, status, iterations, regions_evaluated,
    threshold_calls, threshold_trials). `log`, if a list, receives one dict
    per iteration with the quantities the plants are chosen from."""
    plant = plant or {}
    params = np.ascontiguousarray(params, dtype=np.float64)
    tau = rel_tol
    cap = max_regions
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), init_splits)
    s = lo.shape[1]
    v_f = e_f = 0.0
    prev_vtot = math.nan
    Vp = None
    status = MAX_ITERS
    n_eval = calls = trials_tot = 0
    tr = open(trace_path, "wb") if trace_path else None
    if tr:
        tr.write(b"PGTRACE2")
        tr.write(struct.pack("<ii", d, oracle.FAMILY_ID[family]))
        tr.write(struct.pack("<qqq", oracle.PMAX_RELAX[pmax_relax],
                             oracle.ERROR_RULE[error_rule],
                             oracle.BUDGET[budget]))
    it = 0
    try:
        for it in range(1, max_iters + 1):
            ev = oracle.eval_regions(family, d, params, lo, w, error_rule)
            V, E, K = ev.V, ev.E, ev.K.copy()
            if plant.get("axis", (None,))[0] == it:
                _, i, k = plant["axis"]
                K[i] = k
            n_eval += s
            if it > 1:
                E = oracle.two_level(V, E, Vp)
            A_rel = oracle.classify(V, E, tau, relerr_filter)
            v = oracle.csum(V)
            e = oracle.csum(E)
            v_tot = v + v_f
            e_tot = e + e_f
            rec = dict(it=it, n=s, n_active=0, thr_invoked=0, thr_ok=0,
                       thr_trials=0, terminal=-1, t=math.nan, v=v, e=e,
                       v_f=v_f, e_f=e_f)
            terminated = e_tot <= tau * abs(v_tot) or e_tot <= abs_tol
            if plant.get("stop") == it:
                terminated = True
            n_rel = int(A_rel.sum())
            A = A_rel.copy()
            info = dict(it=it, v_tot=v_tot, e_tot=e_tot, prev_vtot=prev_vtot,
                        tau=tau, V=V, E=E, A_rel=A_rel, D=ev.D, w=w.copy(),
                        n_rel=n_rel)
            if log is not None:
                log.append(info)
            if terminated:
                status = STATUS_OK
                rec.update(terminal=STATUS_OK, n_active=n_rel)
                _write(tr, rec, K, A_rel)
                break
            trig_a = bool(threshold_filter) and it >= 2 and \
                abs(v_tot - prev_vtot) <= tau * abs(v_tot)
            trig_b = bool(threshold_filter) and 2 * n_rel > cap
            invoke = trig_a or trig_b
            if plant.get("trigger") == it:
                invoke = not invoke
            ok = False
            if invoke:
                calls += 1
                relax = pmax_relax == "paper" or trig_b
                if budget == "reserve" and not trig_b:
                    # the finished regions' own share (Lemma 1): earlier
                    # ones and those the rel-err test finishes now
                    fin = (1 - A_rel).astype(np.uint8)
                    allow = tau * abs(v_f + oracle.csum(V, fin)) - e_f
                else:
                    allow = tau * abs(v_tot) - e_f      # the listing's e_it - e_b
                ok, A_thr, t, ntr, _ = oracle.threshold_search(
                    E, A_rel, e, allow, relax)
                trials_tot += ntr
                info.update(searched=True, ok=ok, t=t, trials=ntr, trig_b=trig_b)
                if ok and plant.get("search") == it:
                    ok = False
                rec.update(thr_invoked=1, thr_ok=int(ok),
                           thr_trials=ntr + (plant.get("trials") == it))
                if ok:
                    A = A_thr
                    rec["t"] = t * (1.5 if plant.get("tshift") == it else 1.0)
            if not ok and 2 * n_rel > cap:
                status = MEMORY_EXHAUSTED
                rec.update(terminal=status, n_active=n_rel)
                _write(tr, rec, K, A_rel)
                break
            if plant.get("flip", (None,))[0] == it:
                i = plant["flip"][1]
                A[i] = 1 - A[i]
            prev_vtot = v_tot
            n_act = int(A.sum())
            rec["n_active"] = n_act
            if n_act == 0 or it == max_iters:
                status = NO_ACTIVE if n_act == 0 else MAX_ITERS
                rec["terminal"] = status
                _write(tr, rec, K, A)
                break
            _write(tr, rec, K, A)
            v_f = v - oracle.csum(V, A) + v_f
            e_f = e - oracle.csum(E, A) + e_f
            lo, w, Vp = oracle.filter_split(d, lo, w, K, V, A)
            s = 2 * n_act
    finally:
        if tr:
            tr.close()
    return dict(estimate=v_tot, error=e_tot, status=status, iterations=it,
                regions_evaluated=n_eval, threshold_calls=calls,
                threshold_trials=trials_tot)


def _write(tr, rec, K, A):
    if tr is None:
        return
    tr.write(_REC.pack(rec["it"], rec["n"], rec["n_active"], rec["thr_invoked"],
                       rec["thr_ok"], rec["thr_trials"], rec["terminal"],
                       rec["t"], rec["v"], rec["e"], rec["v_f"], rec["e_f"]))
    tr.write(np.ascontiguousarray(K, np.uint8).tobytes())
    tr.write(np.ascontiguousarray(A, np.uint8).tobytes())
