"""Pins of the oracle's extra integrand families (the paper's Section 4.1
suite: Genz C0, discontinuous, and the box integrals (sum x^2)^p) and of
their closed forms:

* box integrals of degree 2p <= 7 are integrated exactly by the degree-7
  rule (Section 2.1 reading R1) on arbitrary dyadic boxes, against exact
  rational integrals; degree 8 is not, and its null-rule error is non-zero;
* C0 and discontinuous integrands on grids whose planes hold the kinks and
  cut-offs are smooth in every region, so the summed estimates meet the
  closed forms closely; with a kink inside regions they do much worse;
* the box closed forms: the exact moment recursion against brute force, the
  half-integer value against an independent product-Gauss quadrature;
* whole oracle runs meet the closed forms.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_free_run
from workloads import closed_forms as cf


def _box_poly_integral(p, lo, w):
    """Exact int over the box [lo, lo + w] of (sum x_i^2)^p (multinomial)."""
    d = len(lo)
    L = [Fraction(float(x)) for x in lo]
    H = [Fraction(float(a)) + Fraction(float(b)) for a, b in zip(lo, w)]
    total = Fraction(0)

    def rec(i, left, coef, acc):
        nonlocal total
        if i == d - 1:
            k = left
            term = (H[i] ** (2 * k + 1) - L[i] ** (2 * k + 1)) / (2 * k + 1)
            total += coef / factorial(k) * acc * term
            return
        for k in range(left + 1):
            term = (H[i] ** (2 * k + 1) - L[i] ** (2 * k + 1)) / (2 * k + 1)
            rec(i + 1, left - k, coef / factorial(k), acc * term)

    rec(0, p, Fraction(factorial(p)), Fraction(1))
    return total


@pytest.mark.parametrize("d,p", [(2, 1), (3, 2), (3, 3), (5, 3), (2, 0)])
def test_box_polynomials_of_degree_at_most_7_are_exact(d, p):
    lo, w = W.random_boxes(d, 6, seed=10 * d + p, dyadic_bits=6)
    R = oracle.eval_regions("box", d, [float(p)], lo, w)
    for i in range(lo.shape[1]):
        ex = float(_box_poly_integral(p, lo[:, i], w[:, i]))
        assert abs(R.V[i] - ex) <= 1e-14 * abs(ex), (i, R.V[i], ex)
        if 2 * p <= 5:              # the embedded degree-5 rule is exact too
            assert R.E[i] <= 1e-13 * abs(ex)
        else:
            assert R.E[i] > 1e-13 * abs(ex)


def test_box_degree_8_is_not_exact():
    lo, w = W.random_boxes(3, 4, seed=5, dyadic_bits=6)
    R = oracle.eval_regions("box", 3, [4.0], lo, w)
    for i in range(lo.shape[1]):
        ex = float(_box_poly_integral(4, lo[:, i], w[:, i]))
        assert abs(R.V[i] - ex) > 1e-13 * abs(ex)
        assert R.E[i] > 1e-13 * abs(ex)


def test_box_moment_recursion_against_brute_force():
    # (x^2 + y^2 + z^2)^2 over the unit cube by direct expansion
    ex = _box_poly_integral(2, [0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    assert cf.box([2.0], 3) == float(ex)
    assert float(_box_poly_integral(11, [0.0] * 8, [1.0] * 8)) == cf.box([11.0], 8)


def test_box_half_integer_against_gauss_product_quadrature():
    """(x^2 + y^2)^(3/2) and (x^2+y^2+z^2)^(5/2) by tensor Gauss-Legendre on
    a 4^d grid of sub-boxes (the integrands are smooth away from the origin
    corner and C^3 / C^5 there): agreement to 1e-9."""
    for d, pw, m in ((2, 1.5, 24), (3, 2.5, 14)):
        x, wq = np.polynomial.legendre.leggauss(m)
        cells = 4
        pts, wts = [], []
        for c in range(cells):
            pts.append((x + 1) / 2 / cells + c / cells)
            wts.append(wq / 2 / cells)
        pts, wts = np.concatenate(pts), np.concatenate(wts)
        grids = np.meshgrid(*([pts] * d), indexing="ij")
        wgrid = np.ones_like(grids[0])
        for k, g in enumerate(np.meshgrid(*([wts] * d), indexing="ij")):
            wgrid = wgrid * g
        s = sum(g * g for g in grids)
        q = float(np.sum(wgrid * s ** pw))
        assert abs(q - cf.box([pw], d)) <= 1e-9 * q


def test_c0_aligned_grid_meets_the_closed_form():
    d = 3
    p = np.array([10.0, 7.0, 4.0, 0.5, 0.5, 0.5])
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), 8)
    R = oracle.eval_regions("c0", d, p, lo, w)
    ex = cf.c0(p, d)
    assert abs(R.V.sum() - ex) <= 5e-7 * ex      # the rule's error at 8^3 boxes
    # the same integrand with its kink inside the regions is far worse
    p2 = np.array([10.0, 7.0, 4.0, 0.4375 + 1 / 32, 0.5, 0.5])
    R2 = oracle.eval_regions("c0", d, p2, lo, w)
    assert abs(R2.V.sum() - cf.c0(p2, d)) > 100 * abs(R.V.sum() - ex)


def test_discontinuous_aligned_grid_meets_the_closed_form():
    d = 3
    p = np.array([5.0, 6.0, 7.0, 0.5, 0.75, 0.25])
    lo, w = oracle.uniform_split(d, np.zeros(d), np.ones(d), 8)
    R = oracle.eval_regions("discontinuous", d, p, lo, w)
    ex = cf.discontinuous(p, d)
    assert abs(R.V.sum() - ex) <= 2e-7 * ex      # the rule's error at 8^3 boxes
    # cut-offs beyond the cube: the plain exponential product
    p3 = np.array([1.0, 2.0, 3.0, 1.5, 2.0, 9.0])
    assert cf.discontinuous(p3, d) == pytest.approx(
        np.prod([(np.exp(a) - 1) / a for a in (1.0, 2.0, 3.0)]), rel=1e-15)


@pytest.mark.parametrize("family,d,params,tol,g", [
    ("box", 3, [11.0], 1e-8, 2),
    ("box", 4, [7.5], 1e-8, 2),
    ("c0", 3, [10.0, 10.0, 10.0, 0.5, 0.5, 0.5], 1e-6, 2),
    ("discontinuous", 3, [5.0, 6.0, 7.0, 0.4, 0.5, 0.6], 1e-4, 2),
])
@pytest.mark.parametrize("pmax", ["paper", "memory"])
def test_oracle_runs_meet_closed_forms(family, d, params, tol, g, pmax):
    r = oracle.integrate(family, d, params, rel_tol=tol, init_splits=g,
                         pmax_relax=pmax)
    ex = cf.exact(family, params, d)
    # the memory-only P_max rule converges; the paper's may end NO_ACTIVE
    # just above the tolerance with the estimate still within it
    check_free_run(r, ex, tol, allow_no_active=pmax == "paper")


def test_paper_suite_definitions():
    """Section 4.1's integrands at a few points, written out independently."""
    suite = dict(W.paper_suite())
    x8 = np.linspace(0.05, 0.9, 8)
    i8 = np.arange(1, 9)
    assert oracle.f("oscillatory", suite["f1_d8"].params, x8) == pytest.approx(np.cos(i8 @ x8), rel=1e-14)
    x6 = x8[:6]
    assert oracle.f("product_peak", suite["f2_d6"].params, x6) == pytest.approx(
        np.prod(1.0 / (1 / 50 ** 2 + (x6 - 0.5) ** 2)), rel=1e-14)
    assert oracle.f("corner_peak", suite["f3_d8"].params, x8) == pytest.approx(
        (1 + i8 @ x8) ** -9.0, rel=1e-14)
    assert oracle.f("gaussian", suite["f4_d8"].params, x8) == pytest.approx(
        np.exp(-625 * np.sum((x8 - 0.5) ** 2)), rel=1e-13)
    assert oracle.f("c0", suite["f5_d8"].params, x8) == pytest.approx(
        np.exp(-10 * np.sum(np.abs(x8 - 0.5))), rel=1e-14)
    xs = np.full(6, 0.3)
    i6 = np.arange(1, 7)
    assert oracle.f("discontinuous", suite["f6_d6"].params, xs) == pytest.approx(
        np.exp((i6 + 4) @ xs), rel=1e-14)
    xs[5] = 0.95                         # x_6 >= (3 + 6) / 10
    assert oracle.f("discontinuous", suite["f6_d6"].params, xs) == 0.0
    assert oracle.f("box", suite["f7_d8"].params, x8) == pytest.approx(np.sum(x8 ** 2) ** 11, rel=1e-13)
    assert oracle.f("box", suite["f8_d8"].params, x8) == pytest.approx(np.sum(x8 ** 2) ** 7.5, rel=1e-13)
