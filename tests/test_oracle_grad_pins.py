"""Pins of the oracle's parameter derivatives (the adjoint of the estimate
over a fixed partition) against what calculus fixes independently of them:

* the derivative of f against central differences of the oracle's own f;
* the derivative of a region list's summed degree-7 estimate against
  central differences of the (separately pinned) estimates themselves, which
  checks the points and weights the derivative uses;
* closed-form gradients of the Gaussian (erf/exp) and the corner peak
  (inclusion-exclusion, exact rationals) on fine partitions and after whole
  runs;
* a symmetry: a Gaussian centred in the cube has zero derivative in u on a
  symmetric partition;
* the leaves a run ends on: their estimates add up to the run's estimate
  whatever the status the run ends with.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import closed_forms as cf

FAMS = [("product_peak", 3), ("gaussian", 3), ("oscillatory", 4), ("corner_peak", 5)]


def _params(family, d, rng):
    if family == "product_peak":
        return np.concatenate([rng.uniform(2, 6, d), rng.uniform(0.2, 0.8, d)])
    if family == "gaussian":
        return np.concatenate([rng.uniform(2, 6, d), rng.uniform(0.2, 0.8, d)])
    if family == "oscillatory":
        return np.concatenate([rng.uniform(0, 2, d), rng.uniform(0, 1, 1)])
    return rng.uniform(0.2, 2.0, d)


def _steps(p):
    return 1e-5 * np.maximum(1.0, np.abs(p))


@pytest.mark.parametrize("family,d", FAMS)
def test_grad_f_matches_central_differences(family, d):
    rng = np.random.default_rng(100 + d)
    p = _params(family, d, rng)
    h = _steps(p)
    for _ in range(20):
        x = rng.uniform(0, 1, d)
        g = oracle.grad_f(family, p, x)
        assert g.shape == p.shape
        fd = np.empty_like(p)
        for q in range(len(p)):
            pp, pm = p.copy(), p.copy()
            pp[q] += h[q]
            pm[q] -= h[q]
            fd[q] = (oracle.f(family, pp, x) - oracle.f(family, pm, x)) / (2 * h[q])
        scale = np.max(np.abs(g)) + abs(oracle.f(family, p, x))
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * scale)


@pytest.mark.parametrize("family,d", FAMS)
def test_grad_regions_matches_central_differences_of_estimates(family, d):
    """d(sum V)/dtheta by the oracle's adjoint equals central differences of
    sum V: the same points with the same weights, box volume included."""
    rng = np.random.default_rng(200 + d)
    p = _params(family, d, rng)
    lo, w = W.random_boxes(d, 7, seed=d)
    G, Ga = oracle.grad_regions(family, d, p, lo, w)
    h = _steps(p)
    fd = np.empty_like(p)
    for q in range(len(p)):
        pp, pm = p.copy(), p.copy()
        pp[q] += h[q]
        pm[q] -= h[q]
        vp = oracle.eval_regions(family, d, pp, lo, w).V.sum()
        vm = oracle.eval_regions(family, d, pm, lo, w).V.sum()
        fd[q] = (vp - vm) / (2 * h[q])
    np.testing.assert_allclose(G, fd, rtol=1e-6, atol=1e-8 * np.max(Ga))
    assert np.all(Ga >= np.abs(G) * (1 - 1e-15))


def test_grad_regions_gaussian_closed_form_on_fine_grid():
    d = 3
    p = np.array([3.0, 4.0, 5.0, 0.35, 0.5, 0.62])
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), 8)
    G, _ = oracle.grad_regions("gaussian", d, p, lo, w)
    _, dA, dU = cf.gaussian_grad(p, d)
    ref = np.concatenate([dA, dU])
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-8 * np.max(np.abs(ref)))


def test_grad_regions_corner_peak_closed_form_on_fine_grid():
    d = 4
    p = np.array([0.4, 1.1, 1.7, 0.9])
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), 5)
    G, _ = oracle.grad_regions("corner_peak", d, p, lo, w)
    ref = cf.corner_peak_grad(p, d)
    np.testing.assert_allclose(G, ref, rtol=2e-5)   # the rule's error at 5^4 boxes


def test_corner_peak_closed_form_gradient_against_exact_differences():
    """The closed-form gradient itself, against central differences taken in
    exact rational arithmetic (error O(h^2) only)."""
    d = 4
    p = [0.4, 1.1, 1.7, 0.9]
    g = cf.corner_peak_grad(p, d)
    h = 1e-7

    def I(a):
        # same closed form, exact; a are Fractions
        from itertools import combinations
        from math import factorial
        tot = Fraction(0)
        for k in range(d + 1):
            for S in combinations(range(d), k):
                tot += Fraction((-1) ** k) / (1 + sum((a[i] for i in S), Fraction(0)))
        den = Fraction(factorial(d))
        for x in a:
            den *= x
        return tot / den

    a = [Fraction(x) for x in p]
    for j in range(d):
        ap = list(a)
        am = list(a)
        ap[j] += Fraction(h)
        am[j] -= Fraction(h)
        fd = float((I(ap) - I(am)) / (2 * Fraction(h)))
        assert abs(fd - g[j]) <= 1e-10 * abs(g[j])


def test_gaussian_closed_form_gradient_against_differences():
    d = 3
    p = np.array([3.0, 4.0, 5.0, 0.35, 0.5, 0.62])
    _, dA, dU = cf.gaussian_grad(p, d)
    g = np.concatenate([dA, dU])
    for q in range(2 * d):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (cf.gaussian(pp, d) - cf.gaussian(pm, d)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * np.max(np.abs(g))


def test_centred_gaussian_has_zero_u_derivative():
    d = 3
    p = np.array([3.0, 4.0, 5.0, 0.5, 0.5, 0.5])
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), 4)
    G, Ga = oracle.grad_regions("gaussian", d, p, lo, w)
    assert np.all(np.abs(G[d:]) <= 1e-14 * Ga[d:])
    assert np.all(G[:d] < 0)           # wider peaks (smaller a) hold more mass


def test_monomial_has_no_gradient():
    with pytest.raises(ValueError):
        oracle.grad_f("monomial", [1, 2], [0.5, 0.5])


@pytest.mark.parametrize("kw,status", [
    (dict(rel_tol=1e-7, pmax_relax="memory"), "OK"),
    (dict(rel_tol=1e-9, max_iters=3), "MAX_ITERS"),
    (dict(rel_tol=1e-9, max_regions=600, threshold_filter=0), "MEMORY_EXHAUSTED"),
])
def test_run_leaves_add_up_to_the_estimate(kw, status):
    d = 3
    p = np.array([5.0, 6.0, 7.0, 0.4, 0.5, 0.6])
    r = oracle.integrate("gaussian", d, p, grad=True, **kw)
    assert r.status_name == status
    assert abs(r.leaf_v - r.estimate) <= 1e-14 * abs(r.estimate)
    if status == "OK":
        _, dA, dU = cf.gaussian_grad(p, d)
        ref = np.concatenate([dA, dU])
        np.testing.assert_allclose(r.grad, ref, rtol=0,
                                   atol=1e-5 * np.max(np.abs(ref)))


def test_run_leaves_add_up_when_no_region_stays_active():
    """Oscillatory with the rel-err filter on ends NO_ACTIVE; the leaves are
    then the whole final list plus everything finished before."""
    wl = W.oscillatory_d8(1)
    r = oracle.integrate_workload(wl, grad=True, max_regions=1 << 14)
    assert r.status_name == "NO_ACTIVE"
    assert abs(r.leaf_v - r.estimate) <= 1e-13 * max(abs(r.estimate), r.error)


def test_corner_peak_run_gradient_against_closed_form():
    d = 5
    p = np.array([0.4, 1.1, 1.7, 0.9, 0.25])
    r = oracle.integrate("corner_peak", d, p, rel_tol=1e-8, init_splits=2, grad=True,
                         pmax_relax="memory")
    assert r.status_name == "OK"
    ref = cf.corner_peak_grad(p, d)
    np.testing.assert_allclose(r.grad, ref, rtol=1e-6)
