"""Pins for the CPU oracle: checks against what the mathematics fixes.

Every check here is independent of the oracle's own formulas: exact rational
integrals of monomials, closed-form integrals of the workloads, invariants
of the algorithm's steps (Lemma 1, volume conservation, the requirements of
the threshold search) and brute force on tiny inputs.
"""
from fractions import Fraction
from itertools import combinations_with_replacement, product
import math

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import closed_forms as cf
from parity import check_free_run

EPS = np.finfo(np.float64).eps


def _monomials(d, deg):
    """All exponent vectors of total degree exactly ``deg`` in d variables."""
    out = []
    for combo in combinations_with_replacement(range(d), deg):
        a = [0] * d
        for i in combo:
            a[i] += 1
        out.append(a)
    return out


def _dyadic_boxes(d, n, seed):
    rng = np.random.default_rng(seed)
    lo = rng.integers(-8, 8, size=(d, n)) / 8.0          # multiples of 1/8
    w = rng.integers(1, 9, size=(d, n)) / 8.0
    return lo, w


# ---------------------------------------------------------------------------
# Cubature rule (Sections 2.1 and 3.2: the Genz-Malik degree-7 rule)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,n", [(2, 17), (3, 33), (4, 57), (5, 93), (6, 149),
                                 (7, 241), (8, 401), (10, 1245)])
def test_point_count(d, n):
    # 2^d + Theta(d^3) points in the paper's count; the rule has 2^d+2d^2+2d+1
    assert oracle.npoints(d) == n == 2 ** d + 2 * d * d + 2 * d + 1


@pytest.mark.parametrize("d", range(2, 11))
def test_weights_integrate_constants(d):
    """The rule and its embedded rule integrate f = 1 to the box volume."""
    lo, w = _dyadic_boxes(d, 5, seed=d)
    r = oracle.eval_regions("monomial", d, np.zeros(d), lo, w)
    vol = np.prod(w, axis=0)
    np.testing.assert_allclose(r.V, vol, rtol=1e-14)
    assert np.all(r.E <= 1e-14 * vol)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 8])
def test_degree7_exact_on_every_monomial(d):
    """R7 is exact for every monomial of total degree <= 7 on any box."""
    lo, w = _dyadic_boxes(d, 2, seed=100 + d)
    degs = range(0, 8) if d <= 5 else [0, 1, 2, 3, 6, 7]
    worst = 0.0
    for deg in degs:
        for alpha in _monomials(d, deg):
            r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
            for j in range(lo.shape[1]):
                exact = cf.monomial(alpha, lo[:, j], lo[:, j] + w[:, j])
                err = abs(Fraction(r.V[j]) - exact)
                bound = Fraction(r.floorV[j]) + Fraction(1e-300)
                assert err <= bound, (alpha, j, float(err), float(bound))
                if exact != 0:
                    worst = max(worst, float(err / abs(exact)))
    assert worst < 1e-12


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_degree8_not_exact(d):
    """...but not for degree 8: x_1^8 on [-1,1]^d is integrated wrongly,
    which pins the degree (a rule of higher degree would be exact)."""
    lo, w = -np.ones((d, 1)), 2 * np.ones((d, 1))
    alpha = [8] + [0] * (d - 1)
    r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
    exact = float(cf.monomial(alpha, lo[:, 0], lo[:, 0] + w[:, 0]))
    assert abs(r.V[0] - exact) > 1e-3 * exact


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_null_rule_vanishes_to_degree5(d):
    """E = |R7 - R5| is zero (to rounding) on every monomial of degree <= 5,
    because both rules are exact there."""
    lo, w = _dyadic_boxes(d, 2, seed=200 + d)
    for deg in range(0, 6):
        for alpha in _monomials(d, deg):
            r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
            assert np.all(r.E <= r.floorE), (alpha, r.E, r.floorE)


@pytest.mark.parametrize("d", [2, 3, 5, 6, 8, 10])
def test_null_rule_value_on_x6(d):
    """On [-1,1]^d, R7(x_i^6) = 2^d / 7 (exact) and R5(x_i^6) = 2^d 117/700,
    so E / vol = 17/700 independently of d and of the axis."""
    lo, w = -np.ones((d, 1)), 2 * np.ones((d, 1))
    for i in range(d):
        alpha = [0] * d
        alpha[i] = 6
        r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
        assert r.E[0] / 2 ** d == pytest.approx(17 / 700, rel=1e-13)
        assert r.V[0] / 2 ** d == pytest.approx(1 / 7, rel=1e-13)


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_rule_is_fully_symmetric(d):
    """Permuting the axes of the integrand and of the box permutes nothing in
    V and E (the point set is invariant under axis permutations and
    reflections)."""
    rng = np.random.default_rng(d)
    lo, w = _dyadic_boxes(d, 3, seed=300 + d)
    p = W.gaussian_params(d, seed=7)
    perm = rng.permutation(d)
    r1 = oracle.eval_regions("gaussian", d, p, lo, w)
    p2 = np.concatenate([p[:d][perm], p[d:][perm]])
    r2 = oracle.eval_regions("gaussian", d, p2, lo[perm], w[perm])
    np.testing.assert_allclose(r1.V, r2.V, rtol=1e-13)
    np.testing.assert_allclose(r1.E, r2.E, rtol=1e-9, atol=1e-14 * np.abs(r1.V).max())


# ---------------------------------------------------------------------------
# Split axis: fourth divided differences (reading of the split rule)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_fourth_difference_of_x4(d):
    """For f = x_k^4 on [-1,1]^d: D_k = 2 l2^4 - (2/7) l3^4 = 243/1225, every
    other D_j = 0, so the split axis is k."""
    lo, w = -np.ones((d, 1)), 2 * np.ones((d, 1))
    for k in range(d):
        alpha = [0] * d
        alpha[k] = 4
        r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
        assert r.K[0] == k
        assert r.D[0, k] == pytest.approx(243 / 1225, rel=1e-14)
        others = np.delete(r.D[0], k)
        assert np.all(others <= 1e-15)


@pytest.mark.parametrize("d", [3, 5])
def test_fourth_difference_blind_to_cubics(d):
    """D_i = 0 for any polynomial of degree <= 3 in x_i; with every D zero
    the widest axis is split (lowest index among equal widths)."""
    w = np.ones((d, 1))
    w[2, 0] = 2.0
    lo = np.zeros((d, 1))
    for alpha in _monomials(d, 3) + _monomials(d, 2):
        r = oracle.eval_regions("monomial", d, np.array(alpha, float), lo, w)
        assert np.all(r.D[0] <= r.floorD[0] + 1e-15)
        assert r.K[0] == 2
    r = oracle.eval_regions("monomial", d, np.zeros(d), np.zeros((d, 1)),
                            np.ones((d, 1)))
    assert r.K[0] == 0


def test_split_axis_follows_the_steep_direction():
    """A Gaussian ridge steep along axis 1 only is split along axis 1."""
    d = 3
    p = np.array([1.0, 40.0, 1.0, 0.5, 0.37, 0.5])
    lo, w = np.zeros((d, 1)), np.ones((d, 1))
    r = oracle.eval_regions("gaussian", d, p, lo, w)
    assert r.K[0] == 1


# ---------------------------------------------------------------------------
# Uniform-Split, two-level error, classification, sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,g", [(2, 3), (3, 4), (5, 4), (8, 2)])
def test_uniform_split_tiles_the_domain(d, g):
    a = np.linspace(-1.0, 0.0, d)
    b = a + np.linspace(1.0, 2.0, d)
    lo, w = oracle.uniform_split(d, a, b, g)
    assert lo.shape == (d, g ** d)
    # axis 0 varies fastest
    np.testing.assert_allclose(lo[0, :g], a[0] + np.arange(g) * (b[0] - a[0]) / g)
    assert np.all(lo[1:, :g] == lo[1:, :1])
    # cells are distinct and tile the box
    cells = {tuple(np.round((lo[:, j] - a) / w[:, j]).astype(int)) for j in range(g ** d)}
    assert len(cells) == g ** d
    assert np.prod(w, axis=0).sum() == pytest.approx(np.prod(b - a), rel=1e-13)


def test_two_level_properties():
    rng = np.random.default_rng(11)
    m = 200
    V = rng.normal(size=2 * m)
    E = rng.uniform(0, 1e-3, size=2 * m)
    E[:5] = 0.0
    E[m:m + 5] = 0.0
    Vp = V[:m] + V[m:] + rng.normal(scale=1e-3, size=m)
    Vp[10:20] = V[10:20] + V[m + 10:m + 20]          # children agree with parent
    E2 = oracle.two_level(V, E, Vp)
    delta = np.abs(V[:m] + V[m:] - Vp) / 4
    # pair totals grow by exactly 4 delta (up to rounding) when S > 0
    S = E[:m] + E[m:]
    pos = S > 0
    np.testing.assert_allclose((E2[:m] + E2[m:])[pos], (S + 4 * delta)[pos],
                               rtol=1e-13, atol=1e-300)
    # refinement never lowers an error; agreement leaves it untouched
    assert np.all(E2 >= E)
    np.testing.assert_array_equal(E2[10:20], E[10:20])
    # S = 0: each sibling gets delta
    np.testing.assert_allclose(E2[:5], delta[:5], rtol=1e-15)
    # hand-worked pair: Va=1, Vb=2, Vp=3.4, Ea=0.1, Eb=0.3
    #   delta = 0.1, S = 0.4, factor = 1 + 2*0.1/0.4 = 1.5
    #   Ea' = 0.15 + 0.1 = 0.25, Eb' = 0.45 + 0.1 = 0.55
    e = oracle.two_level([1.0, 2.0], [0.1, 0.3], [3.4])
    np.testing.assert_allclose(e, [0.25, 0.55], rtol=1e-14)


def test_classify_semantics():
    V = np.array([1.0, -2.0, 0.0, 1.0, 5.0])
    E = np.array([1e-4, 2e-4, 0.0, 1.1e-4, 1.0])
    A = oracle.classify(V, E, 1e-4)
    # E <= tau |V| finishes (equality included, zero regions finish)
    np.testing.assert_array_equal(A, [0, 0, 0, 1, 1])
    np.testing.assert_array_equal(oracle.classify(V, E, 1e-4, 0), [1] * 5)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_lemma1(sign):
    """Lemma 1 (Section 3.5.1): same-sign V_i with E_i <= tau |V_i| give
    e <= tau |v|; regions the classifier finishes satisfy the premise."""
    rng = np.random.default_rng(3)
    tau = 1e-5
    V = sign * rng.lognormal(size=10000)
    E = tau * np.abs(V) * rng.uniform(0, 2, size=V.size)
    A = oracle.classify(V, E, tau)
    fin = A == 0
    assert fin.any() and (~fin).any()
    e = oracle.csum(E[fin])
    v = oracle.csum(V[fin])
    assert e <= tau * abs(v)


def test_compensated_sum():
    rng = np.random.default_rng(5)
    x = rng.normal(size=100000) * 10.0 ** rng.integers(-10, 10, size=100000)
    assert oracle.csum(x) == pytest.approx(math.fsum(x), rel=1e-15, abs=1e-300)
    m = (rng.uniform(size=x.size) < 0.3).astype(np.uint8)
    assert oracle.csum(x, m) == pytest.approx(math.fsum(x[m == 1]), rel=1e-15)


# ---------------------------------------------------------------------------
# Threshold-Classify (Algorithm 3)
# ---------------------------------------------------------------------------

def _check_search_result(E, A_rel, allow, mem, res):
    ok, A, t, trials, tried = res
    s = len(E)
    assert 1 <= trials <= 64
    if not ok:
        np.testing.assert_array_equal(A, A_rel)
        return
    np.testing.assert_array_equal(A, (A_rel.astype(bool) & (E > t)).astype(np.uint8))
    fin = A == 0
    # memory requirement: more than half finished
    assert fin.sum() > 0.5 * s
    # accuracy requirement with the largest P_max the search may reach
    p_cap = 0.95 if mem else 0.25
    assert math.fsum(E[fin]) <= p_cap * allow * (1 + 1e-12)
    # the accepted threshold was the last one tried
    assert tried[-1] == t
    # thresholds stay inside [min E, max E]
    assert np.all(tried >= E.min()) and np.all(tried <= E.max())


@pytest.mark.parametrize("seed", range(40))
def test_threshold_search_brute_force(seed):
    rng = np.random.default_rng(seed)
    s = int(rng.integers(4, 40))
    E = rng.lognormal(sigma=3.0, size=s) * 1e-6
    A_rel = (rng.uniform(size=s) < 0.85).astype(np.uint8)
    V = rng.uniform(0.5, 1.5, size=s)
    v = V.sum()
    e_it = math.fsum(E)
    tau = float(10.0 ** rng.uniform(-5, -2))
    e_f = float(rng.uniform(0, 0.5)) * tau * v
    e_tot = e_it + e_f
    mem = bool(rng.integers(0, 2))
    # the listing's allowance e_it - e_b, e_b = e_tot - tau |v_tot|
    allow = e_it - (e_tot - tau * v)
    res = oracle.threshold_search(E, A_rel, e_it, allow, mem)
    _check_search_result(E, A_rel, allow, mem, res)
    # brute force: if some candidate threshold satisfies both requirements at
    # P_max = 0.25 and the first trial (the mean) is feasible, it is accepted
    t0 = e_it / s
    A0 = A_rel.astype(bool) & (E > t0)
    first_ok = ((~A0).sum() > 0.5 * s and
                math.fsum(E[~A0]) <= 0.25 * allow)
    if first_ok:
        assert res[0] and res[3] == 1 and res[2] == t0


def test_threshold_search_worked_example():
    """Eight regions; hand-traced trajectory.

    E = [1,2,...,8] * 1e-3, all rel-err active, tau = 1e-3, v_tot = 20,
    e_f = 0 so e_it = e_tot = 0.036 and the allowance e_it - e_b = 0.02.
      trial 1: t = mean = 4.5e-3 -> finished {1..4} -> 4 of 8, memory fails
               -> raise: t = 4.5e-3 + (8e-3 - 4.5e-3)/2 = 6.25e-3
      trial 2: finished {1..6}: 6 > 4, error 0.021 > 0.25*0.02 -> lower:
               t = 6.25e-3 - (6.25e-3 - 1e-3)/2 = 3.625e-3 (direction change 1)
      trial 3: finished {1..3}: memory fails -> raise: t = 5.8125e-3 (2)
      ... the search alternates without a feasible threshold (5 of the 8
      regions carry 0.015 > 0.005) and fails after 10 direction changes.
    """
    E = np.arange(1, 9) * 1e-3
    A_rel = np.ones(8, np.uint8)
    ok, A, t, trials, tried = oracle.threshold_search(E, A_rel, 0.036, 0.02, False)
    assert not ok
    np.testing.assert_array_equal(A, A_rel)
    np.testing.assert_allclose(tried[:3], [4.5e-3, 6.25e-3, 3.625e-3], rtol=1e-15)
    assert tried[3] == pytest.approx(3.625e-3 + (8e-3 - 3.625e-3) / 2, rel=1e-15)
    assert trials == 11
    # relaxed (Section 3.5.3: +0.10 per direction change) the search
    # accepts once P_max * 0.02 covers the 0.015 of five finished regions


def test_threshold_search_worked_example_relaxed():
    """The same eight regions with P_max relaxed at every direction change
    (Section 3.5.3), traced by hand. Allowance 0.02; finished means E <= t.
      1: t = 4.5e-3      finished {1..4}: 4 of 8, memory fails     -> raise
      2: t = 6.25e-3     {1..6}: 0.021 > 0.25*0.02 accuracy fails  -> lower,
                         change 1, P_max 0.35
      3: t = 3.625e-3    {1..3}: memory fails -> raise, change 2, P_max 0.45
      4: t = 5.8125e-3   {1..5}: 0.015 > 0.45*0.02 = 0.009 -> lower,
                         change 3, P_max 0.55
      5: t = 3.40625e-3  {1..3}: memory fails -> raise, change 4, 0.65
      6: t = 5.703125e-3 {1..5}: 0.015 > 0.013 -> lower, change 5, 0.75
      7: t = 3.3515625e-3  {1..3}: memory fails -> raise, change 6, 0.85
      8: t = 5.67578125e-3 {1..5}: 0.015 <= 0.85*0.02 = 0.017: accepted.
    """
    E = np.arange(1, 9) * 1e-3
    A_rel = np.ones(8, np.uint8)
    ok, A, t, trials, tried = oracle.threshold_search(E, A_rel, 0.036, 0.02, True)
    hand = [4.5e-3, 6.25e-3, 3.625e-3, 5.8125e-3, 3.40625e-3, 5.703125e-3,
            3.3515625e-3, 5.67578125e-3]
    assert ok and trials == 8
    np.testing.assert_allclose(tried, hand, rtol=1e-14)
    assert t == tried[-1]
    np.testing.assert_array_equal(A, [0, 0, 0, 0, 0, 1, 1, 1])


def test_threshold_search_worked_example_with_reserve():
    """The relaxed example again with an allowance of 0.0175 instead of 0.02
    (as when part of the budget is kept back for the regions left active):
    the accuracy requirement becomes finished error <= P_max * 0.0175.
    Traced by hand (finished means E <= t):
      1-7: as without the reserve (0.015 fails 0.25, 0.45, 0.65 x 0.0175)
      8: t = 5.67578125e-3   {1..5}: 0.015 > 0.85*0.0175 = 0.014875
                             -> lower, change 7, P_max 0.95
      9: t = 3.337890625e-3  {1..3}: memory fails -> raise, change 8
     10: t = 5.6689453125e-3 {1..5}: 0.015 <= 0.95*0.0175 = 0.016625: accepted.
    """
    E = np.arange(1, 9) * 1e-3
    A_rel = np.ones(8, np.uint8)
    ok, A, t, trials, tried = oracle.threshold_search(E, A_rel, 0.036, 0.0175, True)
    hand = [4.5e-3, 6.25e-3, 3.625e-3, 5.8125e-3, 3.40625e-3, 5.703125e-3,
            3.3515625e-3, 5.67578125e-3, 3.337890625e-3, 5.6689453125e-3]
    assert ok and trials == 10
    np.testing.assert_allclose(tried, hand, rtol=1e-14)
    assert t == tried[-1]
    np.testing.assert_array_equal(A, [0, 0, 0, 0, 0, 1, 1, 1])
    # a negative allowance leaves no feasible threshold
    ok, A, t, trials, _ = oracle.threshold_search(E, A_rel, 0.036, -0.01, True)
    assert not ok
    np.testing.assert_array_equal(A, A_rel)


# ---------------------------------------------------------------------------
# Filter + Split
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 5, 8])
def test_filter_split_against_mask(d):
    rng = np.random.default_rng(d)
    n = 301
    lo, w = W.random_boxes(d, n, seed=d, dyadic_bits=10)
    K = rng.integers(0, d, size=n).astype(np.uint8)
    V = rng.normal(size=n)
    A = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    lo2, w2, Vp = oracle.filter_split(d, lo, w, K, V, A)
    idx = np.flatnonzero(A)
    na = len(idx)
    assert lo2.shape == (d, 2 * na)
    np.testing.assert_array_equal(Vp, V[idx])                   # stable order
    for half in (0, 1):
        seg = slice(half * na, (half + 1) * na)
        for k in range(d):
            split = K[idx] == k
            wk = np.where(split, w[k, idx] / 2, w[k, idx])
            lk = np.where(split & (half == 1), lo[k, idx] + w[k, idx] / 2, lo[k, idx])
            np.testing.assert_array_equal(w2[k, seg], wk)
            np.testing.assert_array_equal(lo2[k, seg], lk)
    # children tile their parent exactly (dyadic boxes: exact arithmetic)
    vol_par = np.prod(w[:, idx], axis=0)
    vol_ch = np.prod(w2[:, :na], axis=0) + np.prod(w2[:, na:], axis=0)
    np.testing.assert_array_equal(vol_ch, vol_par)


def test_filter_split_empty():
    d = 3
    lo, w = W.random_boxes(d, 10, seed=1)
    lo2, w2, Vp = oracle.filter_split(d, lo, w, np.zeros(10, np.uint8),
                                      np.ones(10), np.zeros(10, np.uint8))
    assert lo2.shape == (d, 0) and len(Vp) == 0


# ---------------------------------------------------------------------------
# Whole runs against the closed forms (Section 4.2's accuracy methodology:
# compare the true error, not only the estimated one)
# ---------------------------------------------------------------------------

def _check_run(wl, r, pmax="memory"):
    """Closed form met (status OK); under the paper's P_max rule a NO_ACTIVE
    end just above the tolerance is accepted if the estimate meets it."""
    exact = cf.exact(wl.family, wl.params, wl.d)
    check_free_run(r, exact, wl.rel_tol, allow_no_active=pmax == "paper")


PMAX = ["paper", "memory"]


@pytest.mark.parametrize("pmax", PMAX)
def test_free_run_product_peak_d3(pmax):
    wl = W.product_peak_d3()
    r = oracle.integrate_workload(wl, pmax_relax=pmax)
    _check_run(wl, r, pmax)
    assert r.fevals == r.regions_evaluated * 33


@pytest.mark.parametrize("pmax", PMAX)
@pytest.mark.parametrize("tau", [1e-3, 1e-5, 1e-7])
def test_free_run_product_peak_tolerance_sweep(tau, pmax):
    wl = W.product_peak_d3()
    wl.rel_tol = tau
    _check_run(wl, oracle.integrate_workload(wl, pmax_relax=pmax), pmax)


@pytest.mark.parametrize("pmax", PMAX)
def test_free_run_gaussian_d5_reduced(pmax):
    """The d=5 Gaussian at rel_tol 1e-4 with a 2^16-region cap (the full
    1e-6 run takes ~25 s)."""
    wl = W.gaussian_d5(max_regions=1 << 16)
    wl.rel_tol = 1e-4
    r = oracle.integrate_workload(wl, pmax_relax=pmax)
    _check_run(wl, r, pmax)
    assert r.threshold_calls > 0


def test_pmax_rules_differ_only_in_searches():
    """The two P_max rules take the same decisions up to the first threshold
    search whose trajectory changes direction; after it the paper's rule
    commits more error to finished regions. With no error kept back for the
    active regions (budget "listing"), on the d=5 Gaussian to 1e-4 with a
    2^16-region cap the paper's rule runs more searches and ends NO_ACTIVE,
    while the memory-only rule converges."""
    wl = W.gaussian_d5(max_regions=1 << 16)
    rp = oracle.integrate_workload(wl, rel_tol=1e-4, pmax_relax="paper",
                                   budget="listing")
    rm = oracle.integrate_workload(wl, rel_tol=1e-4, pmax_relax="memory",
                                   budget="listing")
    assert rm.status_name == "OK"
    assert rp.status_name == "NO_ACTIVE"
    assert rp.threshold_calls > rm.threshold_calls
    # no threshold search at all: the two rules cannot differ
    a = oracle.integrate_workload(wl, rel_tol=1e-4, threshold_filter=0,
                                  pmax_relax="paper")
    b = oracle.integrate_workload(wl, rel_tol=1e-4, threshold_filter=0,
                                  pmax_relax="memory")
    assert (a.estimate, a.error, a.iterations) == (b.estimate, b.error, b.iterations)


def test_reserve_keeps_the_run_convergent():
    """Under the paper's P_max rule, keeping back the error the active
    regions may still end with (Lemma 1) in searches started by the
    settled-digits trigger keeps the finished error below tau |v|: the d=5
    Gaussian to 1e-4 (2^16-region cap) converges with fewer searches than
    without it, and meets its closed form."""
    wl = W.gaussian_d5(max_regions=1 << 16)
    wl.rel_tol = 1e-4
    rr = oracle.integrate_workload(wl, budget="reserve")
    rl = oracle.integrate_workload(wl, budget="listing")
    assert rr.status_name == "OK" and rl.status_name == "NO_ACTIVE"
    assert rr.threshold_calls < rl.threshold_calls
    check_free_run(rr, cf.exact(wl.family, wl.params, wl.d), wl.rel_tol)
    # without a search the budget cannot matter
    a = oracle.integrate_workload(wl, threshold_filter=0, budget="reserve")
    b = oracle.integrate_workload(wl, threshold_filter=0, budget="listing")
    assert (a.estimate, a.error, a.iterations) == (b.estimate, b.error, b.iterations)


@pytest.mark.slow
@pytest.mark.parametrize("pmax", PMAX)
def test_free_run_gaussian_d5_full(pmax):
    wl = W.gaussian_d5()
    r = oracle.integrate_workload(wl, pmax_relax=pmax)
    _check_run(wl, r, pmax)
    assert r.peak_regions == wl.max_regions          # memory trigger fired


def test_free_run_oscillatory_d8():
    """Sign-changing integrand: with the rel-err filter off the run converges;
    with it on every region is finished before the total error is small
    enough (the failure Section 3.5.1 warns about), reported as NO_ACTIVE."""
    wl = W.oscillatory_d8(relerr_filter=0)
    _check_run(wl, oracle.integrate_workload(wl), "paper")
    r = oracle.integrate_workload(W.oscillatory_d8(relerr_filter=1))
    assert r.status_name == "NO_ACTIVE"
    assert r.error > 1e-5 * abs(r.estimate)


def test_free_run_corner_peak_d6():
    a = W.corner_peak_params(6, seed=9)
    exact = cf.corner_peak(a, 6)
    for pmax in PMAX:
        r = oracle.integrate("corner_peak", 6, a, rel_tol=1e-5, init_splits=2,
                             pmax_relax=pmax)
        check_free_run(r, exact, 1e-5, allow_no_active=pmax == "paper")


def test_status_paths():
    wl = W.gaussian_d5()
    r = oracle.integrate_workload(wl, max_iters=1)
    assert r.status_name == "MAX_ITERS" and r.iterations == 1
    r = oracle.integrate_workload(wl, max_regions=1500, threshold_filter=0)
    assert r.status_name == "MEMORY_EXHAUSTED"
    with pytest.raises(RuntimeError):
        oracle.integrate_workload(wl, max_regions=100)       # 4^5 > cap
    with pytest.raises(RuntimeError):
        oracle.integrate("gaussian", 5, wl.params, rel_tol=0.0, abs_tol=0.0)
