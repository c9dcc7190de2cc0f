"""GPU parity of the four-null-rule error estimate (PG_ERR_NULL4) through
the C-ABI: per region (pg_evaluate_rule) against the oracle, whole runs by
trace replay, the batched driver against single runs, and the argument
checks. The default estimate is unchanged by the option's existence.

Each test prints the case it runs before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import closed_forms as cf

from parity import assert_region_parity, rel_close, search_diff

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_06494_amd as pg
    torch.cuda.set_device(0)
    c = pg.Context(capacity=1 << 21, dim_max=10)
    yield c
    c.close()


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _params(family, d, seed):
    rng = np.random.default_rng(seed)
    if family in ("gaussian", "product_peak", "c0"):
        return np.concatenate([rng.uniform(3, 25, d), rng.uniform(0.2, 0.8, d)])
    if family == "oscillatory":
        return np.concatenate([rng.uniform(0, 4, d), rng.uniform(0, 1, 1)])
    if family == "discontinuous":
        return np.concatenate([rng.uniform(1, 6, d), rng.uniform(0.3, 1.5, d)])
    if family == "box":
        return np.array([rng.choice([2.5, 7.5, 11.0])])
    if family == "monomial":
        return rng.integers(0, 4, d).astype(float)
    return rng.uniform(0.2, 2.0, d)


EVAL_CASES = [(fam, d, n) for fam in ("gaussian", "product_peak", "oscillatory", "corner_peak")
              for d, n in ((2, 1), (3, 257), (5, 1000), (8, 513), (10, 130))] + \
             [(fam, d, n) for fam in ("monomial", "c0", "discontinuous", "box")
              for d, n in ((4, 300), (7, 129))]


@pytest.mark.parametrize("family,d,n", EVAL_CASES)
def test_evaluate_parity_null4(ctx, family, d, n):
    _say("evaluate-null4", family, d, n)
    p = _params(family, d, 80 + d + n)
    lo, w = W.random_boxes(d, n, seed=300 + d + n)
    V, E, K = ctx.evaluate(family, p, _dev(lo), _dev(w), error_rule="null4")
    torch.cuda.synchronize()
    ref = oracle.eval_regions(family, d, p, lo, w, error_rule="null4")
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


def test_default_error_is_the_raw_one(ctx):
    _say("evaluate-default")
    d, n = 5, 777
    p = _params("gaussian", d, 3)
    lo, w = W.random_boxes(d, n, seed=9)
    V0, E0, K0 = ctx.evaluate("gaussian", p, _dev(lo), _dev(w))
    V1, E1, K1 = ctx.evaluate("gaussian", p, _dev(lo), _dev(w), error_rule="raw")
    V2, E2, K2 = ctx.evaluate("gaussian", p, _dev(lo), _dev(w), error_rule="null4")
    assert torch.equal(V0, V1) and torch.equal(E0, E1) and torch.equal(K0, K1)
    assert torch.equal(V0, V2) and torch.equal(K0, K2)
    assert not torch.equal(E0, E2)


REPLAY = [
    ("gaussian_d3", "gaussian", 3, [12.0, 15.0, 9.0, 0.4, 0.55, 0.6], 1e-6, 2, 1),
    ("product_peak_d4", "product_peak", 4, [8.0, 6.0, 10.0, 7.0, 0.3, 0.5, 0.7, 0.45], 1e-5, 2, 1),
    ("oscillatory_d5", "oscillatory", 5, [1.5, 0.8, 2.1, 1.1, 0.6, 0.3], 1e-6, 2, 0),
    ("corner_peak_d6", "corner_peak", 6, [0.5, 1.2, 0.8, 1.6, 0.3, 0.9], 1e-5, 2, 1),
    ("box_d4_half", "box", 4, [7.5], 1e-7, 2, 1),
    ("gaussian_d5_peaked", "gaussian", 5, [25.0, 20.0, 22.0, 18.0, 24.0, 0.3, 0.6, 0.5, 0.45, 0.7],
     1e-4, 4, 1),
]


@pytest.mark.parametrize("name,family,d,p,tol,g,relerr", REPLAY, ids=[c[0] for c in REPLAY])
def test_integrate_replay_null4(ctx, tmp_path, name, family, d, p, tol, g, relerr):
    _say("replay-null4", name)
    trace = str(tmp_path / "trace.bin")
    r = ctx.integrate(family, d, p, rel_tol=tol, init_splits=g, relerr_filter=relerr,
                      trace_path=trace, error_rule="null4")
    o = oracle.integrate(family, d, p, rel_tol=tol, init_splits=g, relerr_filter=relerr,
                         max_regions=1 << 21, replay_path=trace, error_rule="null4")
    hard = {k: v for k, v in o.replay.items() if k.endswith("_hard") and v}
    assert not hard, (hard, search_diff(o.replay))
    assert (r.status, r.iterations, r.regions_evaluated) == \
        (o.status, o.iterations, o.regions_evaluated)
    assert rel_close(r.estimate, o.estimate, 1e-10)
    assert rel_close(r.error, o.error, 1e-9) or \
        abs(r.error - o.error) <= 1e-12 * abs(o.estimate), (r.error, o.error)
    if r.status_name == "OK":
        ex = cf.exact(family, p, d)
        assert abs(r.estimate - ex) <= tol * abs(ex)


def test_batched_null4_equals_single_runs(ctx):
    _say("batch-null4")
    wl = W.corner_peak_batch_d6(B=8)
    res = ctx.integrate_batch(wl.family, wl.d, wl.params, wl.rel_tol, wl.abs_tol,
                              init_splits=wl.init_splits, max_iters=wl.max_iters,
                              max_regions=1 << 17, error_rule="null4")
    for b in range(wl.B):
        r1 = ctx.integrate(wl.family, wl.d, wl.params[b], rel_tol=wl.rel_tol[b],
                           abs_tol=wl.abs_tol[b], init_splits=wl.init_splits,
                           max_iters=wl.max_iters, max_regions=1 << 17, error_rule="null4")
        assert (r1.status, r1.iterations, r1.regions_evaluated) == \
            (res[b].status, res[b].iterations, res[b].regions_evaluated)
        assert rel_close(r1.estimate, res[b].estimate, 1e-10)
        assert rel_close(r1.error, res[b].error, 1e-9)


def test_error_rule_is_checked(ctx):
    _say("null4-errors")
    import paper_2104_06494_amd as pg
    lo, w = W.random_boxes(3, 4, seed=1)
    with pytest.raises(pg.PaganiError):
        ctx.evaluate("gaussian", _params("gaussian", 3, 1), _dev(lo), _dev(w), error_rule=7)
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, _params("gaussian", 3, 1), error_rule=2)
    with pytest.raises(ValueError):
        ctx.integrate("gaussian", 3, _params("gaussian", 3, 1), error_rule="cuhre")
