"""GPU parity of the parameter derivative over the final partition.

The library's adjoint kernel (through the C-ABI entry points
pg_integrate_grad / pg_integrate_batch_grad) is compared with:

* the oracle's derivative over the very leaves the GPU run ended on (its
  partition copied out), to 1e-12 of the sum of absolute terms;
* central differences (h = 1e-5) of the summed estimates of those leaves,
  re-evaluated by the GPU at theta +- h (the frozen partition);
* the closed-form gradients (Gaussian, corner peak) at the run's accuracy;
* the batched form against single runs, and the forward with the adjoint
  against the forward without it (the adjoint must not change the run).

Each test prints the case it runs before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import closed_forms as cf

from parity import rel_close

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
    c = pg.Context(capacity=1 << 22, dim_max=10)
    yield c
    c.close()


def _params(family, d, seed):
    rng = np.random.default_rng(seed)
    if family == "gaussian":
        return np.concatenate([rng.uniform(5, 15, d), rng.uniform(0.2, 0.8, d)])
    if family == "product_peak":
        return np.concatenate([rng.uniform(3, 8, d), rng.uniform(0.2, 0.8, d)])
    if family == "oscillatory":
        return np.concatenate([rng.uniform(0, 1.5, d), rng.uniform(0, 1, 1)])
    return rng.uniform(0.2, 2.0, d)


CASES = [("gaussian", 3, 1e-6, 1), ("gaussian", 6, 1e-5, 1),
         ("product_peak", 3, 1e-6, 1), ("oscillatory", 4, 1e-5, 0),
         ("corner_peak", 6, 1e-6, 1), ("gaussian", 2, 1e-8, 1)]
# higher dimensions at loose tolerances (the Gaussian above d = 6 takes the
# point-by-point vertex walk instead of the unrolled one)
HIGH_D = [("gaussian", 7, 1e-2, 1), ("product_peak", 8, 1e-2, 1),
          ("oscillatory", 9, 1e-4, 0), ("corner_peak", 10, 1e-2, 1)]


def _leaf_sum(ctx, family, p, L):
    V, _, _ = ctx.evaluate(family, p, L["lo"], L["w"])
    return float(V.sum())


@pytest.mark.parametrize("family,d,tol,relerr", CASES + HIGH_D)
def test_grad_against_oracle_on_the_gpu_partition(ctx, family, d, tol, relerr):
    _say("grad-vs-oracle", family, d, tol)
    p = _params(family, d, 60 + d)
    r, g, L = ctx.integrate_grad(family, d, p, rel_tol=tol, relerr_filter=relerr,
                                 init_splits=2, max_regions=1 << 18,
                                 leaves_capacity=1 << 22)
    assert L["n"] > 0
    # the leaves tile the box: volumes add up to 1, estimates to the estimate
    w = L["w"].cpu().numpy()
    assert abs(np.prod(w, axis=0).sum() - 1.0) <= 1e-12
    assert rel_close(_leaf_sum(ctx, family, p, L), r.estimate, 1e-12)
    assert (L["owner"].cpu().numpy() == 0).all()
    G, Ga = oracle.grad_regions(family, d, p, L["lo"].cpu().numpy(), w)
    assert np.all(np.abs(g - G) <= 1e-12 * Ga + 1e-300), (g, G, Ga)


@pytest.mark.parametrize("family,d,tol,relerr", CASES[:5])
def test_grad_against_differences_on_the_frozen_partition(ctx, family, d, tol, relerr):
    _say("grad-vs-fd", family, d, tol)
    p = _params(family, d, 70 + d)
    r, g, L = ctx.integrate_grad(family, d, p, rel_tol=tol, relerr_filter=relerr,
                                 init_splits=2, max_regions=1 << 18,
                                 leaves_capacity=1 << 22)
    fd = np.empty_like(p)
    for q in range(len(p)):
        h = 1e-5 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd[q] = (_leaf_sum(ctx, family, pp, L) - _leaf_sum(ctx, family, pm, L)) / (2 * h)
    scale = np.max(np.abs(g))
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * scale)


def test_gaussian_d6_gradient_meets_the_closed_form(ctx):
    """The d=6 Gaussian parameter points at their tolerance (1e-5): the
    estimate meets it against the erf closed form, and each component of
    the derivative lies within tau of the closed form's on the component's
    own scale, |dI/dtheta_k| + |I| / s_k with s_k = a_k for a_k and 1 / a_k
    for u_k (the size a change of theta_k by its own width moves I by).
    The run controls the estimate's error, not the derivative's; on that
    scale the derivative's error measures at most 0.64 tau over all 256
    points of the workload at 1e-5 (and 0.095 tau for the converged ones
    at 1e-7), so tau is the bound asserted."""
    _say("grad-closed-form gaussian d6")
    wl = W.gaussian_grad_d6(B=6)
    n_ok = 0
    for b in range(wl.B):
        p = wl.params[b]
        r, g, _ = ctx.integrate_grad("gaussian", 6, p, rel_tol=wl.rel_tol[b],
                                     init_splits=2, max_regions=wl.max_regions)
        if r.status_name != "OK":
            continue
        n_ok += 1
        tau = wl.rel_tol[b]
        I, dA, dU = cf.gaussian_grad(p, 6)
        ref = np.concatenate([dA, dU])
        assert abs(r.estimate - I) <= tau * abs(I)
        a = p[:6]
        scale = np.abs(ref) + abs(I) / np.concatenate([a, 1.0 / a])
        assert np.all(np.abs(g - ref) <= tau * scale), np.max(np.abs(g - ref) / scale) / tau
    assert n_ok >= wl.B - 1


def test_corner_peak_gradient_meets_the_closed_form(ctx):
    _say("grad-closed-form corner d6")
    p = np.array([0.4, 1.1, 1.7, 0.9, 0.25, 1.3])
    r, g, _ = ctx.integrate_grad("corner_peak", 6, p, rel_tol=1e-7, init_splits=2)
    assert r.status_name == "OK"
    assert abs(r.estimate - cf.corner_peak(p, 6)) <= 1e-7 * abs(r.estimate)
    np.testing.assert_allclose(g, cf.corner_peak_grad(p, 6), rtol=1e-5)


def test_adjoint_leaves_the_forward_run_unchanged(ctx):
    _say("grad-forward-unchanged")
    wl = W.gaussian_grad_d6(B=6)
    wl.rel_tol[:] = 1e-6
    plain = ctx.integrate_batch_workload(wl)
    res, G, _ = ctx.integrate_batch_workload(wl, grad=True)
    for a, b in zip(plain, res):
        assert (a.status, a.iterations, a.regions_evaluated, a.estimate, a.error) == \
            (b.status, b.iterations, b.regions_evaluated, b.estimate, b.error)


def test_batched_grad_equals_single_runs(ctx):
    """Six Gaussian parameter points, three in flight at a time."""
    _say("grad-batch-vs-single")
    import paper_2104_06494_amd as pg
    wl = W.gaussian_grad_d6(B=6)
    wl.rel_tol[:] = 1e-4
    wl.max_regions = 1 << 16
    c = pg.Context(capacity=3 << 16, dim_max=6)
    res, G, L = c.integrate_batch_workload(wl, grad=True, leaves_capacity=1 << 22)
    owner = L["owner"].cpu().numpy()
    lo, w = L["lo"].cpu().numpy(), L["w"].cpu().numpy()
    for b in range(wl.B):
        r1, g1, _ = c.integrate_grad("gaussian", 6, wl.params[b], rel_tol=1e-4,
                                     init_splits=2, max_regions=wl.max_regions)
        assert (r1.status, r1.iterations, r1.regions_evaluated) == \
            (res[b].status, res[b].iterations, res[b].regions_evaluated)
        Gb, Gab = oracle.grad_regions("gaussian", 6, wl.params[b], lo[:, owner == b],
                                      w[:, owner == b])
        assert np.all(np.abs(G[b] - Gb) <= 1e-12 * Gab + 1e-300)
        assert np.all(np.abs(G[b] - g1) <= 1e-10 * Gab + 1e-300)
        assert abs(np.prod(w[:, owner == b], axis=0).sum() - 1.0) <= 1e-12
    c.close()


@pytest.mark.parametrize("kw,status", [
    (dict(rel_tol=1e-9, max_iters=3), "MAX_ITERS"),
    (dict(rel_tol=1e-9, max_regions=600, threshold_filter=0), "MEMORY_EXHAUSTED"),
])
def test_grad_when_the_run_stops_early(ctx, kw, status):
    """The partition is the finished regions plus the list left when the run
    stops, whatever the reason."""
    _say("grad-early-stop", status)
    p = np.array([5.0, 6.0, 7.0, 0.4, 0.5, 0.6])
    r, g, L = ctx.integrate_grad("gaussian", 3, p, init_splits=4,
                                 leaves_capacity=1 << 20, **kw)
    assert r.status_name == status
    assert rel_close(_leaf_sum(ctx, "gaussian", p, L), r.estimate, 1e-12)
    G, Ga = oracle.grad_regions("gaussian", 3, p, L["lo"].cpu().numpy(),
                                L["w"].cpu().numpy())
    assert np.all(np.abs(g - G) <= 1e-12 * Ga + 1e-300)
    o = oracle.integrate("gaussian", 3, p, init_splits=4, grad=True, **kw)
    assert o.status_name == status and o.regions_evaluated == r.regions_evaluated
    assert np.all(np.abs(g - o.grad) <= 1e-10 * o.grad_abs + 1e-300)


def test_autograd_function(ctx):
    _say("grad-autograd")
    import paper_2104_06494_amd as pg
    wl = W.gaussian_grad_d6(B=3)
    theta = torch.tensor(wl.params, dtype=torch.float64, requires_grad=True)
    I = pg.integral(theta, "gaussian", 6, rel_tol=1e-6, context=ctx, init_splits=2)
    wts = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    (gt,) = torch.autograd.grad((I * wts).sum(), theta)
    res, G, _ = ctx.integrate_batch_grad("gaussian", 6, wl.params, 1e-6, init_splits=2)
    np.testing.assert_array_equal(I.detach().numpy(), [r.estimate for r in res])
    np.testing.assert_allclose(gt.numpy(), wts.numpy()[:, None] * G, rtol=0, atol=0)
    with torch.no_grad():
        I2 = pg.integral(theta, "gaussian", 6, rel_tol=1e-6, context=ctx, init_splits=2)
    np.testing.assert_array_equal(I2.numpy(), I.detach().numpy())


def test_grad_errors(ctx):
    _say("grad-errors")
    import paper_2104_06494_amd as pg
    with pytest.raises(pg.PaganiError):
        ctx.integrate_grad("monomial", 3, [1, 2, 3])
    with pytest.raises(pg.PaganiError):        # more leaves than room for them
        ctx.integrate_grad("gaussian", 3, [5, 6, 7, .4, .5, .6], rel_tol=1e-6,
                           leaves_capacity=100)
