"""Seeded synthetic workloads for the PAGANI integrator.

This module only draws integrand parameters and tolerances from fixed seeds
and describes the five benchmark workloads. It contains none of the
integration method's arithmetic, so that both the GPU library's tests and
the CPU oracle can take their inputs from it without sharing code.

Parameter draws use ``numpy.random.default_rng(seed)`` and always draw the
steepness vector ``a`` (all axes) first, then the location vector ``u``.

Integrand families (all on the unit cube unless stated otherwise); the
paper's own test functions (Section 4.1) belong to the same Genz families:

* ``product_peak``  f(x) = prod_i 1 / (a_i^-2 + (x_i - u_i)^2)
* ``gaussian``      f(x) = exp(-sum_i a_i^2 (x_i - u_i)^2)
* ``oscillatory``   f(x) = cos(2 pi u_1 + sum_i a_i x_i)
* ``corner_peak``   f(x) = (1 + sum_i a_i x_i)^-(d+1)
* ``monomial``      f(x) = prod_i x_i^alpha_i   (test family, integer alpha)
* ``c0``            f(x) = exp(-sum_i a_i |x_i - u_i|)            (Genz C0)
* ``discontinuous`` f(x) = exp(sum_i a_i x_i) if x_i < c_i for all i, else 0
* ``box``           f(x) = (sum_i x_i^2)^p                        (box integrals)

Parameter vector layout per family (``params``):

* product_peak, gaussian: ``[a_1..a_d, u_1..u_d]``  (2d values)
* oscillatory:            ``[a_1..a_d, u_1]``        (d+1 values)
* corner_peak:            ``[a_1..a_d]``             (d values)
* monomial:               ``[alpha_1..alpha_d]``     (d values, integers)
* c0:                     ``[a_1..a_d, u_1..u_d]``   (2d values)
* discontinuous:          ``[a_1..a_d, c_1..c_d]``   (2d values)
* box:                    ``[p]``                    (1 value)
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

FAMILIES = {
    "product_peak": 0,
    "gaussian": 1,
    "oscillatory": 2,
    "corner_peak": 3,
    "monomial": 4,
    "c0": 5,
    "discontinuous": 6,
    "box": 7,
}


def n_params(family: str, d: int) -> int:
    """Length of the parameter vector of ``family`` in dimension ``d``."""
    if family in ("product_peak", "gaussian", "c0", "discontinuous"):
        return 2 * d
    if family == "box":
        return 1
    if family == "oscillatory":
        return d + 1
    if family in ("corner_peak", "monomial"):
        return d
    raise ValueError(f"unknown family {family!r}")


@dataclass
class Workload:
    """One plain (single-integral) run: integrand, domain and options."""
    name: str
    family: str
    d: int
    params: np.ndarray
    rel_tol: float
    abs_tol: float = 1e-20
    init_splits: int = 4
    max_regions: int = 1 << 21
    max_iters: int = 100
    relerr_filter: int = 1
    threshold_filter: int = 1
    lo: np.ndarray = field(default=None)
    hi: np.ndarray = field(default=None)

    def __post_init__(self):
        if self.lo is None:
            self.lo = np.zeros(self.d)
        if self.hi is None:
            self.hi = np.ones(self.d)
        self.params = np.ascontiguousarray(self.params, dtype=np.float64)
        self.lo = np.ascontiguousarray(self.lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(self.hi, dtype=np.float64)

    @property
    def npoints(self) -> int:
        """Cubature points per region, 2^d + 2d^2 + 2d + 1."""
        d = self.d
        return (1 << d) + 2 * d * d + 2 * d + 1


def product_peak_params(d: int, seed: int, a_range=(5.0, 15.0),
                        u_range=(0.2, 0.8)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.uniform(*a_range, size=d)
    u = rng.uniform(*u_range, size=d)
    return np.concatenate([a, u])


def gaussian_params(d: int, seed: int, a_range=(10.0, 25.0),
                    u_range=(0.3, 0.7)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.uniform(*a_range, size=d)
    u = rng.uniform(*u_range, size=d)
    return np.concatenate([a, u])


def oscillatory_params(d: int, seed: int, a_range=(0.0, 1.5),
                       a_sum=6.0) -> np.ndarray:
    """a_i ~ U[a_range] rescaled so that sum_i a_i = a_sum; u_1 ~ U[0, 1]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(*a_range, size=d)
    a = a * (a_sum / a.sum())
    u1 = rng.uniform(0.0, 1.0, size=1)
    return np.concatenate([a, u1])


def corner_peak_params(d: int, seed: int, a_range=(0.0, 2.0)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(*a_range, size=d)


def monomial_params(alpha) -> np.ndarray:
    return np.asarray(alpha, dtype=np.float64)


# --------------------------------------------------------------------------
# The five benchmark workloads (sizes and distributions as specified for the
# MI355X build; the paper's own suite uses the same families, Section 4.1).
# --------------------------------------------------------------------------

def product_peak_d3() -> Workload:
    """d=3 product peak, 4^3 initial grid, rel_tol 1e-3 (small case)."""
    return Workload("product_peak_d3", "product_peak", 3,
                    product_peak_params(3, seed=1), rel_tol=1e-3,
                    init_splits=4)


def gaussian_d5(max_regions: int = 1 << 21) -> Workload:
    """d=5 Gaussian, 4^5 initial grid, rel_tol 1e-6 (headline workload).

    The live list is capped at 2^21 regions, below the ~2.6e6 the run would
    otherwise reach, so that the memory trigger of the threshold search
    fires during the run."""
    return Workload("gaussian_d5", "gaussian", 5, gaussian_params(5, seed=2),
                    rel_tol=1e-6, init_splits=4, max_regions=max_regions)


def oscillatory_d8(relerr_filter: int = 1) -> Workload:
    """d=8 oscillatory (sum a = 6), 2^8 initial grid, rel_tol 1e-5."""
    return Workload("oscillatory_d8", "oscillatory", 8,
                    oscillatory_params(8, seed=3), rel_tol=1e-5,
                    init_splits=2, relerr_filter=relerr_filter)


# --------------------------------------------------------------------------
# The paper's own test suite (Section 4.1): fixed parameters, unit cube.
# Each entry: name, family, d, params, initial splits per axis.
# --------------------------------------------------------------------------

def _idx(d):
    return np.arange(1, d + 1, dtype=np.float64)


def paper_suite():
    """f1..f8 of Section 4.1 in the dimensions the paper reports (8-d f1,
    f3, f4, f5, f7, f8; 5-d f4; 6-d f6 and f2; 3-d f3), as (name, Workload)
    with rel_tol 1e-3 (the sweep sets its own tolerances). Initial grids:
    2^d splits (the halving planes fall on the kinks of f5 and on the
    cut-off of f6 at 1/2), 4^3 for 3-d and 4^5 for 5-d."""
    half = lambda d: np.full(d, 0.5)
    S = []
    d = 8
    S.append(("f1_d8", "oscillatory", d, np.concatenate([_idx(d), [0.0]]), 2, 0))
    S.append(("f2_d6", "product_peak", 6, np.concatenate([np.full(6, 50.0), half(6)]), 2, 1))
    S.append(("f3_d3", "corner_peak", 3, _idx(3), 4, 1))
    S.append(("f3_d8", "corner_peak", d, _idx(d), 2, 1))
    S.append(("f4_d5", "gaussian", 5, np.concatenate([np.full(5, 25.0), half(5)]), 4, 1))
    S.append(("f4_d8", "gaussian", d, np.concatenate([np.full(d, 25.0), half(d)]), 2, 1))
    S.append(("f5_d8", "c0", d, np.concatenate([np.full(d, 10.0), half(d)]), 2, 1))
    S.append(("f6_d6", "discontinuous", 6,
              np.concatenate([_idx(6) + 4.0, (3.0 + _idx(6)) / 10.0]), 2, 1))
    S.append(("f7_d8", "box", d, np.array([11.0]), 2, 1))
    S.append(("f8_d8", "box", d, np.array([7.5]), 2, 1))
    out = []
    for name, fam, dd, par, g, relerr in S:
        out.append((name, Workload(name, fam, dd, par, rel_tol=1e-3, init_splits=g,
                                   relerr_filter=relerr)))
    return out


def paper_tolerances():
    """The sweep of Section 4: 1e-3 down to 1.024e-10, each a fifth of the
    one before."""
    return [1e-3 * 0.2 ** k for k in range(11)]


@dataclass
class BatchWorkload:
    """Many independent integrals of one family with per-instance params."""
    name: str
    family: str
    d: int
    params: np.ndarray       # [B, n_params]
    rel_tol: np.ndarray      # [B]
    abs_tol: np.ndarray      # [B]
    init_splits: int = 2
    max_regions: int = 1 << 21   # cap of each integral's live list
    max_iters: int = 100
    relerr_filter: int = 1
    threshold_filter: int = 1
    lo: np.ndarray = field(default=None)
    hi: np.ndarray = field(default=None)

    def __post_init__(self):
        if self.lo is None:
            self.lo = np.zeros(self.d)
        if self.hi is None:
            self.hi = np.ones(self.d)

    @property
    def B(self) -> int:
        return int(self.params.shape[0])

    @property
    def npoints(self) -> int:
        return (1 << self.d) + 2 * self.d * self.d + 2 * self.d + 1

    def instance(self, b: int) -> "Workload":
        """Integral b as a single workload (same options)."""
        return Workload(f"{self.name}[{b}]", self.family, self.d,
                        np.array(self.params[b]), float(self.rel_tol[b]),
                        init_splits=self.init_splits, max_regions=self.max_regions,
                        max_iters=self.max_iters, abs_tol=float(self.abs_tol[b]),
                        relerr_filter=self.relerr_filter,
                        threshold_filter=self.threshold_filter,
                        lo=self.lo, hi=self.hi)


def corner_peak_batch_d6(B: int = 1024, seed: int = 4) -> BatchWorkload:
    """B corner-peak integrals, d=6, a ~ U[0,2] per instance and per-instance
    rel_tol log-uniform in [1e-7, 1e-4]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 2.0, size=(B, 6))
    tol = 10.0 ** rng.uniform(-7.0, -4.0, size=B)
    return BatchWorkload("corner_peak_batch_d6", "corner_peak", 6, a, tol,
                         np.full(B, 1e-20), init_splits=2)


def gaussian_grad_d6(B: int = 256, seed: int = 5,
                     rel_tol: float = 1e-5) -> BatchWorkload:
    """B Gaussian parameter points, d=6, theta = (a_1..a_6, u_1..u_6),
    a ~ U[5,20], u ~ U[0.2,0.8], 2^6 initial grid, cap
    2^22 regions per integral.

    rel_tol defaults to 1e-5: at 1e-7 every one of these peaked 6-d
    Gaussians exhausts even a 2^23-region cap with an estimated relative
    error near 1e-5 (the degree-7 rule's error estimate, not the true error,
    which is near 1e-7 there); at 1e-5 and 2^22 regions they converge."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(5.0, 20.0, size=(B, 6))
    u = rng.uniform(0.2, 0.8, size=(B, 6))
    return BatchWorkload("gaussian_grad_d6", "gaussian", 6,
                         np.concatenate([a, u], axis=1), np.full(B, rel_tol),
                         np.full(B, 1e-20), init_splits=2, max_regions=1 << 22)


def peaked_batch(family: str, d: int, B: int = 128, seed: int = 6,
                 rel_tol: float = 1e-4) -> BatchWorkload:
    """B sharply peaked integrals for comparing error estimates: Gaussians
    (a ~ U[10, 30]) or product peaks (a ~ U[5, 20]), peak centres
    u ~ U[0.2, 0.8] per axis, 2^d initial grid, cap 2^20 regions each."""
    rng = np.random.default_rng(seed)
    lo_a, hi_a = (10.0, 30.0) if family == "gaussian" else (5.0, 20.0)
    a = rng.uniform(lo_a, hi_a, size=(B, d))
    u = rng.uniform(0.2, 0.8, size=(B, d))
    return BatchWorkload(f"{family}_peaked_d{d}", family, d,
                         np.concatenate([a, u], axis=1), np.full(B, rel_tol),
                         np.full(B, 1e-20), init_splits=2, max_regions=1 << 20)


def random_boxes(d: int, n: int, seed: int, lo=0.0, hi=1.0,
                 dyadic_bits: int = 0):
    """n random axis-aligned boxes inside [lo, hi]^d, as SoA arrays
    (lower corners ``[d, n]`` and widths ``[d, n]``).

    With ``dyadic_bits > 0`` every corner and width is a multiple of
    2^-dyadic_bits, so that box arithmetic (halving, adding half widths) is
    exact in binary floating point.
    """
    rng = np.random.default_rng(seed)
    if dyadic_bits:
        m = 1 << dyadic_bits
        a = rng.integers(0, m, size=(d, n))
        b = rng.integers(0, m, size=(d, n))
        l = np.minimum(a, b)
        wd = np.abs(a - b) + 1
        wd = np.minimum(wd, m - l)
        span = hi - lo
        return lo + span * l / m, span * wd / m
    x0 = rng.uniform(lo, hi, size=(d, n))
    x1 = rng.uniform(lo, hi, size=(d, n))
    l = np.minimum(x0, x1)
    wd = np.maximum(np.abs(x1 - x0), 1e-3 * (hi - lo))
    wd = np.minimum(wd, hi - l)
    return l, wd
