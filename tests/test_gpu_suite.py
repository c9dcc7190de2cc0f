"""GPU parity for the paper's own test suite (Section 4.1): the extra
families (Genz C0, discontinuous, box integrals) through the C-ABI against
the oracle, per region and per run (trace replay), and the suite's
integrals f1..f8 against their closed forms.

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
    if family == "c0":
        return np.concatenate([rng.uniform(2, 12, d), rng.uniform(0.2, 0.8, d)])
    if family == "discontinuous":
        return np.concatenate([rng.uniform(1, 8, d), rng.uniform(0.3, 0.9, d)])
    return np.array([rng.choice([0.0, 3.0, 7.5, 11.0, 2.3])])


INTEGRAND_CASES = [("c0", 3, None), ("c0", 8, None), ("discontinuous", 6, None),
                   ("box", 8, [11.0]), ("box", 8, [7.5]), ("box", 5, [2.3]),
                   ("box", 4, [0.0])]


@pytest.mark.parametrize("family,d,p", INTEGRAND_CASES)
def test_integrand_values(ctx, family, d, p):
    _say("integrand", family, d, p)
    p = _params(family, d, 31) if p is None else np.array(p)
    x = np.random.default_rng(d).uniform(0, 1, size=(d, 3000))
    y = ctx.integrand_values(family, p, _dev(x)).cpu().numpy()
    ref = np.array([oracle.f(family, p, x[:, i]) for i in range(x.shape[1])])
    np.testing.assert_allclose(y, ref, rtol=2e-13, atol=0)


EVAL_CASES = [(fam, d, n, p) for fam in ("c0", "discontinuous")
              for d, n in ((2, 1), (3, 65), (5, 1000), (6, 3001), (8, 777), (9, 65),
                           (10, 129))
              for p in (None,)] + \
             [("box", d, n, [pw]) for d, n in ((2, 129), (3, 65), (5, 1000), (6, 300),
                                               (8, 777), (10, 129))
              for pw in (11.0, 7.5, 2.3)]


@pytest.mark.parametrize("family,d,n,p", EVAL_CASES)
def test_evaluate_parity(ctx, family, d, n, p):
    _say("evaluate", family, d, n, p)
    p = _params(family, d, 40 + d) if p is None else np.array(p)
    lo, w = W.random_boxes(d, n, seed=200 + d + n)
    V, E, K = ctx.evaluate(family, p, _dev(lo), _dev(w))
    torch.cuda.synchronize()
    ref = oracle.eval_regions(family, d, p, lo, w)
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


REPLAY = [
    ("c0_d3", "c0", 3, [10.0, 7.0, 4.0, 0.5, 0.5, 0.5], 1e-6, 2, 1),
    ("c0_d4_kink_inside", "c0", 4, [10.0, 10.0, 10.0, 10.0, 0.37, 0.5, 0.61, 0.5], 1e-4, 2, 1),
    ("discontinuous_d3", "discontinuous", 3, [5.0, 6.0, 7.0, 0.4, 0.5, 0.6], 1e-4, 2, 1),
    ("box_d4_half", "box", 4, [7.5], 1e-8, 2, 1),
    ("box_d8_int", "box", 8, [11.0], 1e-3, 2, 1),
    ("f6_d6", "discontinuous", 6, list(np.arange(1, 7) + 4.0) + list((3.0 + np.arange(1, 7)) / 10),
     1e-3, 2, 1),
]


@pytest.mark.parametrize("name,family,d,p,tol,g,relerr", REPLAY, ids=[c[0] for c in REPLAY])
def test_integrate_replay(ctx, tmp_path, name, family, d, p, tol, g, relerr):
    _say("replay", name)
    trace = str(tmp_path / "trace.bin")
    r = ctx.integrate(family, d, p, rel_tol=tol, init_splits=g, relerr_filter=relerr,
                      trace_path=trace)
    o = oracle.integrate(family, d, p, rel_tol=tol, init_splits=g,
                         relerr_filter=relerr, max_regions=1 << 21, replay_path=trace)
    hard = {k: v for k, v in o.replay.items() if k.endswith("_hard") and v}
    assert not hard, (hard, search_diff(o.replay))
    assert (r.status, r.iterations, r.regions_evaluated) == \
        (o.status, o.iterations, o.regions_evaluated)
    assert rel_close(r.estimate, o.estimate, 1e-10)
    # the error to 1e-10 of itself, unless it sits at the estimate's rounding
    # noise (near-polynomial regions: each E is a difference of two rules
    # that agree to a few ulps of V)
    assert rel_close(r.error, o.error, 1e-10) or \
        abs(r.error - o.error) <= 1e-12 * abs(o.estimate), (r.error, o.error)
    if r.status_name == "OK":
        ex = cf.exact(family, p, d)
        assert abs(r.estimate - ex) <= tol * abs(ex)


@pytest.fixture(scope="module")
def big_ctx():
    """2^24 regions (4.8 GB at d = 8): the suite's 8-d integrands need far
    longer lists than the 2^21 of the other tests."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_06494_amd as pg
    torch.cuda.set_device(0)
    c = pg.Context(capacity=1 << 24, dim_max=8)
    yield c
    c.close()


@pytest.mark.parametrize("name", [n for n, _ in W.paper_suite()])
def test_paper_suite_meets_closed_forms(big_ctx, name):
    """Each of f1..f8 at tau = 1e-3 and 2e-4 (the sweep's first two):
    converged runs meet the closed form and every run's reported error
    bounds its true error. At 1e-3, runs other than f1's (sign changes;
    the rel-err filter is off for it, as the paper runs it) end OK or
    NO_ACTIVE just above the tolerance (the regions left all pass the
    rel-err test while the error finished earlier already fills the
    budget); at 2e-4 some exhaust the 2^21-region list."""
    _say("suite", name)
    wl = dict(W.paper_suite())[name]
    ex = cf.exact(wl.family, wl.params, wl.d)
    for tol in W.paper_tolerances()[:2]:
        r = big_ctx.integrate_workload(wl, rel_tol=tol, max_regions=0)
        if name != "f1_d8" and tol == 1e-3:
            assert r.status_name == "OK" or (
                r.status_name == "NO_ACTIVE" and r.error <= 2 * tol * abs(r.estimate)), \
                (name, tol, r)
        if r.status_name == "OK":
            assert abs(r.estimate - ex) <= tol * abs(ex), (name, tol, r.estimate, ex)
        assert abs(r.estimate - ex) <= max(r.error, tol * abs(ex)), (name, tol, r, ex)


def test_batched_suite_family(ctx):
    """Box integrals with different powers in one batched run, against single
    runs."""
    _say("batch-box")
    import paper_2104_06494_amd as pg
    P = np.array([[2.5], [7.5], [11.0], [4.0], [0.5]])
    tol = np.array([1e-7, 1e-6, 1e-5, 1e-8, 1e-6])
    c = pg.Context(capacity=5 << 17, dim_max=6)
    res = c.integrate_batch("box", 6, P, tol, init_splits=2, max_regions=1 << 17)
    for b in range(len(P)):
        r1 = c.integrate("box", 6, P[b], rel_tol=tol[b], init_splits=2, max_regions=1 << 17)
        assert (r1.status, r1.iterations, r1.regions_evaluated) == \
            (res[b].status, res[b].iterations, res[b].regions_evaluated)
        assert rel_close(r1.estimate, res[b].estimate, 1e-10)
        if r1.status_name == "OK":
            ex = cf.box(P[b], 6)
            assert abs(r1.estimate - ex) <= tol[b] * ex
    c.close()
