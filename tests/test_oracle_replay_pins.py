"""Pins for the oracle's replay mode, on the CPU.

Whole-run parity of the GPU rests on the oracle replaying a decision trace:
it recomputes every decision of Algorithm 2 and Algorithm 3 and follows the
trace only where its own margins certify a rounding tie, counting every
other difference as uncertified ("hard"). These tests write traces with an
independent driver of Algorithm 2 (tests/replay_driver.py, the oracle's step
functions called in the listing's order) and check that

* the driver reproduces the oracle's free run bit for bit under both P_max
  rules and both search budgets (so the run-level choices of when a search
  relaxes P_max and how much error it keeps back for the active regions
  are pinned against a second coding of Sections 3.5.2-3.5.3),
* an untouched trace replays with no override at all and the same result,
* one planted decision that is nowhere near a tie -- a split axis, an
  active flag, a trigger, a search outcome or trial count, a termination --
  raises the matching uncertified counter,
* a trace written under other rules is refused.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
import replay_driver as RD

CASES = {
    "product_peak_d3_1e-6": (W.product_peak_d3, dict(rel_tol=1e-6)),
    "gaussian_d5_1e-4": (W.gaussian_d5, dict(rel_tol=1e-4, max_regions=1 << 16)),
    "oscillatory_d8_relerr_on": (lambda: W.oscillatory_d8(1),
                                 dict(max_regions=1 << 16)),
    "gaussian_d5_memory_cap": (W.gaussian_d5, dict(rel_tol=1e-5,
                                                   max_regions=1 << 14)),
}


def _args(name, pmax, budget="reserve"):
    mk, kw = CASES[name]
    wl = mk()
    a = dict(rel_tol=wl.rel_tol, abs_tol=wl.abs_tol, init_splits=wl.init_splits,
             max_iters=wl.max_iters, relerr_filter=wl.relerr_filter,
             threshold_filter=wl.threshold_filter, max_regions=wl.max_regions,
             pmax_relax=pmax, budget=budget)
    a.update(kw)
    return wl, a


def _hard(o):
    return {k: v for k, v in o.replay.items() if k.endswith("_hard") and v}


@pytest.mark.parametrize("pmax,budget", [("paper", "reserve"), ("paper", "listing"),
                                         ("memory", "reserve")])
@pytest.mark.parametrize("name", sorted(CASES))
def test_driver_reproduces_free_run_and_replays_clean(name, pmax, budget, tmp_path):
    wl, a = _args(name, pmax, budget)
    trace = str(tmp_path / "t.bin")
    r = RD.run(wl.family, wl.d, wl.params, trace_path=trace, **a)
    o = oracle.integrate(wl.family, wl.d, wl.params, **a)
    assert (r["estimate"], r["error"], r["status"], r["iterations"],
            r["regions_evaluated"], r["threshold_calls"], r["threshold_trials"]) == \
        (o.estimate, o.error, o.status, o.iterations, o.regions_evaluated,
         o.threshold_calls, o.threshold_trials)
    rp = oracle.integrate(wl.family, wl.d, wl.params, replay_path=trace, **a)
    counts = {k: v for k, v in rp.replay.items()
              if k not in ("records", "max_t_rel", "max_v_rel", "max_e_rel") and v}
    assert not counts, counts                   # no override, nothing hard
    assert rp.replay["records"] == o.iterations
    assert rp.replay["max_t_rel"] == 0.0
    assert (rp.estimate, rp.error, rp.status, rp.iterations) == \
        (o.estimate, o.error, o.status, o.iterations)


def test_the_two_rules_differ_on_a_run_with_relaxed_searches():
    """Under the paper's rule a search started by the settled-digits
    trigger relaxes P_max; under the memory-only rule it does not. On the
    d=5 Gaussian to 1e-4 (2^16-region cap, the listing's budget) this
    changes the run, so the driver-equality test above pins which searches
    relax under each rule."""
    out = {}
    for pmax in ("paper", "memory"):
        wl, a = _args("gaussian_d5_1e-4", pmax, "listing")
        out[pmax] = RD.run(wl.family, wl.d, wl.params, **a)
    assert out["paper"]["threshold_trials"] != out["memory"]["threshold_trials"]


def test_the_two_budgets_differ_on_runs_with_searches():
    """Keeping back the active regions' error changes the searches started
    by the settled-digits trigger: the d=5 Gaussian to 1e-4 (2^16-region
    cap) converges with it and ends NO_ACTIVE without. Searches started
    because the list would overflow keep nothing back; the three searches
    of the 2^14-region case (d=5 Gaussian to 1e-5) are all of that kind.
    The driver-equality test above runs both cases under both budgets, so
    it pins both halves."""
    out = {}
    for budget in ("reserve", "listing"):
        wl, a = _args("gaussian_d5_1e-4", "paper", budget)
        out[budget] = RD.run(wl.family, wl.d, wl.params, **a)
    assert out["reserve"]["status"] == RD.STATUS_OK
    assert out["listing"]["status"] == RD.NO_ACTIVE


def _clean_log(name, pmax="paper", budget="reserve"):
    wl, a = _args(name, pmax, budget)
    log = []
    RD.run(wl.family, wl.d, wl.params, log=log, **a)
    return wl, a, log


def _replay_planted(tmp_path, wl, a, plant):
    trace = str(tmp_path / "planted.bin")
    RD.run(wl.family, wl.d, wl.params, trace_path=trace, plant=plant, **a)
    return oracle.integrate(wl.family, wl.d, wl.params, replay_path=trace, **a)


def test_planted_axis_is_uncertified(tmp_path):
    wl, a, log = _clean_log("product_peak_d3_1e-6")
    for L in log[1:]:
        D = L["D"]
        srt = np.sort(D, axis=1)
        clear = np.flatnonzero((srt[:, -1] > 4 * srt[:, -2]) & (srt[:, -1] > 0))
        if len(clear):
            i = int(clear[0])
            k = int(np.argmin(D[i]))
            o = _replay_planted(tmp_path, wl, a, dict(axis=(L["it"], i, k)))
            assert o.replay["axis_hard"] >= 1, o.replay
            assert o.replay["axis_override"] == 0
            return
    pytest.fail("no region with a clear split axis")


def test_planted_active_flag_is_uncertified(tmp_path):
    wl, a, log = _clean_log("product_peak_d3_1e-6")
    for L in log:
        if L.get("searched"):
            continue
        far = np.flatnonzero((L["A_rel"] == 1) &
                             (L["E"] > 2 * L["tau"] * np.abs(L["V"])))
        if len(far) and L["n_rel"] > 1:
            o = _replay_planted(tmp_path, wl, a, dict(flip=(L["it"], int(far[0]))))
            assert o.replay["class_hard"] >= 1, o.replay
            assert o.replay["class_override"] == 0
            return
    pytest.fail("no iteration without a search")


def test_planted_threshold_flag_is_uncertified(tmp_path):
    """A region the accepted threshold keeps active (E far above t) recorded
    as finished."""
    wl, a, log = _clean_log("product_peak_d3_1e-6")
    for L in log:
        if not (L.get("searched") and L["ok"]):
            continue
        far = np.flatnonzero((L["A_rel"] == 1) & (L["E"] > 2 * L["t"]))
        if len(far):
            o = _replay_planted(tmp_path, wl, a, dict(flip=(L["it"], int(far[0]))))
            assert o.replay["thr_hard"] + o.replay["class_hard"] >= 1, o.replay
            assert o.replay["thr_override"] == 0
            return
    pytest.fail("no accepted search")


def test_planted_trigger_is_uncertified(tmp_path):
    wl, a, log = _clean_log("gaussian_d5_1e-4")
    for L in log[1:]:
        if L.get("searched"):
            continue
        if abs(L["v_tot"] - L["prev_vtot"]) > 2 * L["tau"] * abs(L["v_tot"]):
            o = _replay_planted(tmp_path, wl, a, dict(trigger=L["it"]))
            assert o.replay["trig_hard"] >= 1, o.replay
            assert o.replay["trig_override"] == 0
            return
    pytest.fail("no iteration far from the settled-digits trigger")


@pytest.mark.parametrize("what", ["search", "trials"])
def test_planted_search_outcome_is_uncertified(tmp_path, what):
    # the listing's budget: its run accepts searches the settled-digits
    # trigger starts
    wl, a, log = _clean_log("gaussian_d5_1e-4", budget="listing")
    for L in log:
        if L.get("searched") and L["ok"] and not L["trig_b"]:
            o = _replay_planted(tmp_path, wl, a, {what: L["it"]})
            assert o.replay["search_hard"] >= 1, o.replay
            return
    pytest.fail("no accepted search under the settled-digits trigger")


def test_planted_threshold_value_is_uncertified(tmp_path):
    """An accepted threshold recorded half as large again (same outcome,
    same trial count) lies far outside the rounding band of the search's
    halvings and of the extreme errors they approach."""
    wl, a, log = _clean_log("gaussian_d5_1e-4")
    for L in log:
        if L.get("searched") and L.get("ok"):
            o = _replay_planted(tmp_path, wl, a, dict(tshift=L["it"]))
            assert o.replay["search_hard"] >= 1, o.replay
            return
    pytest.fail("no accepted search")


def test_planted_termination_is_uncertified(tmp_path):
    wl, a, log = _clean_log("gaussian_d5_1e-4")
    for L in log:
        if L["e_tot"] > 2 * L["tau"] * abs(L["v_tot"]):
            o = _replay_planted(tmp_path, wl, a, dict(stop=L["it"]))
            assert o.replay["term_hard"] >= 1, o.replay
            assert o.replay["term_override"] == 0
            return
    pytest.fail("no iteration far from termination")


def test_replay_refuses_a_trace_of_other_rules(tmp_path):
    wl, a = _args("product_peak_d3_1e-6", "paper")
    trace = str(tmp_path / "t.bin")
    RD.run(wl.family, wl.d, wl.params, trace_path=trace, **a)
    a["pmax_relax"] = "memory"
    with pytest.raises(RuntimeError):
        oracle.integrate(wl.family, wl.d, wl.params, replay_path=trace, **a)
    a["pmax_relax"] = "paper"
    with pytest.raises(RuntimeError):
        oracle.integrate(wl.family, wl.d, wl.params, replay_path=trace,
                         error_rule="null4", **a)
    a["budget"] = "listing"
    with pytest.raises(RuntimeError):
        oracle.integrate(wl.family, wl.d, wl.params, replay_path=trace, **a)


def test_trace_of_another_integrand_is_uncertified(tmp_path):
    """The decisions of another integrand (a steeper peak on one axis) are
    followed, since the trace drives the list, but counted as uncertified."""
    wl, a = _args("product_peak_d3_1e-6", "paper")
    trace = str(tmp_path / "t.bin")
    RD.run(wl.family, wl.d, wl.params, trace_path=trace, **a)
    p2 = wl.params.copy()
    p2[0] *= 1.7
    o = oracle.integrate(wl.family, wl.d, p2, replay_path=trace, **a)
    assert sum(_hard(o).values()) > 0, o.replay
