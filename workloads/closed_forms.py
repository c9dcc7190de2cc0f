"""Exact values of the workload integrals (independent of any cubature).

Each integral over a box factorises or reduces to a finite sum, so it can be
evaluated to far more digits than double precision with ``mpmath`` (or
exactly with ``fractions``). These values are what the integrator's final
estimate is judged against; nothing here is used by the integrator itself.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations
from math import factorial

import mpmath as mp
import numpy as np

mp.mp.dps = 50


def _bounds(d, lo, hi):
    lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
    return [mp.mpf(float(x)) for x in lo], [mp.mpf(float(x)) for x in hi]


def product_peak(params, d, lo=None, hi=None) -> float:
    """prod_i  a_i (atan(a_i (hi_i - u_i)) - atan(a_i (lo_i - u_i)))."""
    a = [mp.mpf(float(x)) for x in params[:d]]
    u = [mp.mpf(float(x)) for x in params[d:2 * d]]
    L, H = _bounds(d, lo, hi)
    r = mp.mpf(1)
    for i in range(d):
        r *= a[i] * (mp.atan(a[i] * (H[i] - u[i])) - mp.atan(a[i] * (L[i] - u[i])))
    return float(r)


def gaussian(params, d, lo=None, hi=None) -> float:
    """prod_i  sqrt(pi)/(2 a_i) (erf(a_i (hi_i - u_i)) - erf(a_i (lo_i - u_i)))."""
    a = [mp.mpf(float(x)) for x in params[:d]]
    u = [mp.mpf(float(x)) for x in params[d:2 * d]]
    L, H = _bounds(d, lo, hi)
    r = mp.mpf(1)
    for i in range(d):
        r *= mp.sqrt(mp.pi) / (2 * a[i]) * (mp.erf(a[i] * (H[i] - u[i]))
                                             - mp.erf(a[i] * (L[i] - u[i])))
    return float(r)


def oscillatory(params, d, lo=None, hi=None) -> float:
    """Re[ exp(i 2 pi u_1) prod_i (exp(i a_i hi_i) - exp(i a_i lo_i)) / (i a_i) ]."""
    a = [mp.mpf(float(x)) for x in params[:d]]
    u1 = mp.mpf(float(params[d]))
    L, H = _bounds(d, lo, hi)
    z = mp.expj(2 * mp.pi * u1)
    for i in range(d):
        if a[i] == 0:
            z *= (H[i] - L[i])
        else:
            z *= (mp.expj(a[i] * H[i]) - mp.expj(a[i] * L[i])) / (1j * a[i])
    return float(mp.re(z))


def corner_peak(params, d) -> float:
    """Unit cube only: (1/(d! prod a_i)) sum_{S subset [d]} (-1)^|S| / (1 + sum_{i in S} a_i),
    evaluated in exact rational arithmetic over the double-precision a_i (the
    alternating sum cancels badly when some a_i are small)."""
    a = [Fraction(float(x)) for x in params[:d]]
    if any(x == 0 for x in a):
        raise ValueError("corner_peak closed form needs every a_i != 0")
    total = Fraction(0)
    for k in range(d + 1):
        for S in combinations(range(d), k):
            total += Fraction((-1) ** k) / (1 + sum((a[i] for i in S), Fraction(0)))
    den = Fraction(factorial(d))
    for x in a:
        den *= x
    return float(total / den)


def corner_peak_grad(params, d):
    """Unit cube: dI/da_j of the corner-peak closed form, differentiated term
    by term: with P = d! prod a_i and T = sum_S (-1)^|S| / (1 + sum_S a),
    dI/da_j = -I / a_j - (1/P) sum_{S containing j} (-1)^|S| / (1 + sum_S a)^2.
    Exact rational arithmetic over the double-precision a_i."""
    a = [Fraction(float(x)) for x in params[:d]]
    if any(x == 0 for x in a):
        raise ValueError("corner_peak closed form needs every a_i != 0")
    P = Fraction(factorial(d))
    for x in a:
        P *= x
    T = Fraction(0)
    dT = [Fraction(0)] * d
    for k in range(d + 1):
        for S in combinations(range(d), k):
            den = 1 + sum((a[i] for i in S), Fraction(0))
            T += Fraction((-1) ** k) / den
            for j in S:
                dT[j] -= Fraction((-1) ** k) / (den * den)
    I = T / P
    return np.array([float(-I / a[j] + dT[j] / P) for j in range(d)])


def monomial(alpha, lo, hi) -> Fraction:
    """Exact prod_i (hi_i^(k+1) - lo_i^(k+1)) / (k+1) over a box with float corners."""
    r = Fraction(1)
    for k, l, h in zip(alpha, lo, hi):
        k = int(k)
        r *= (Fraction(float(h)) ** (k + 1) - Fraction(float(l)) ** (k + 1)) / (k + 1)
    return r


def c0(params, d, lo=None, hi=None) -> float:
    """prod_i int exp(-a_i |x - u_i|) dx over [lo_i, hi_i]:
    (2 - e^{-a(u - lo)} - e^{-a(hi - u)}) / a for lo <= u <= hi."""
    a = [mp.mpf(float(x)) for x in params[:d]]
    u = [mp.mpf(float(x)) for x in params[d:2 * d]]
    L, H = _bounds(d, lo, hi)
    r = mp.mpf(1)
    for i in range(d):
        if not (L[i] <= u[i] <= H[i]):
            raise ValueError("c0 closed form needs lo <= u <= hi")
        r *= (2 - mp.exp(-a[i] * (u[i] - L[i])) - mp.exp(-a[i] * (H[i] - u[i]))) / a[i]
    return float(r)


def discontinuous(params, d, lo=None, hi=None) -> float:
    """prod_i int_{lo_i}^{min(c_i, hi_i)} e^{a_i x} dx (zero if c_i <= lo_i)."""
    a = [mp.mpf(float(x)) for x in params[:d]]
    c = [mp.mpf(float(x)) for x in params[d:2 * d]]
    L, H = _bounds(d, lo, hi)
    r = mp.mpf(1)
    for i in range(d):
        top = min(c[i], H[i])
        if top <= L[i]:
            return 0.0
        r *= (top - L[i]) if a[i] == 0 else (mp.exp(a[i] * top) - mp.exp(a[i] * L[i])) / a[i]
    return float(r)


def _square_sum_moments(p: int, d: int):
    """E[S^k], k = 0..p, S the sum of d squares of independent U(0,1):
    exact rationals, adding one axis at a time by the binomial theorem
    (E[X^(2j)] = 1/(2j+1))."""
    from math import comb
    M = [Fraction(1 if k == 0 else 0) for k in range(p + 1)]
    for _ in range(d):
        M = [sum(Fraction(comb(k, j)) * M[j] / (2 * (k - j) + 1) for j in range(k + 1))
             for k in range(p + 1)]
    return M


def box(params, d) -> float:
    """int_{[0,1]^d} (sum x_i^2)^p dx. Integer p: the exact rational moment.
    Otherwise E[S^p] from the Laplace-transform identity, for n < p < n+1,
    S^p = (1/Gamma(-p)) int_0^inf (e^{-tS} - sum_{k<=n} (-tS)^k/k!) t^{-p-1} dt,
    with E[e^{-tS}] = (sqrt(pi)/(2 sqrt t) erf(sqrt t))^d: the part over
    [0, 1/2] termwise from the moment series, the rest by quadrature, at
    40 significant digits."""
    pw = float(params[0])
    if pw == int(pw) and pw >= 0:
        return float(_square_sum_moments(int(pw), d)[int(pw)])
    with mp.workdps(40):
        alpha = mp.mpf(pw)
        n = int(mp.floor(alpha))
        K = 90
        mk = [mp.mpf(x.numerator) / x.denominator for x in _square_sum_moments(K, d)]
        t0 = mp.mpf("0.5")
        head = mp.fsum((-1) ** k * mk[k] / mp.factorial(k) * t0 ** (k - alpha) / (k - alpha)
                       for k in range(n + 1, K + 1))

        def integrand(t):
            m = (mp.sqrt(mp.pi) / (2 * mp.sqrt(t)) * mp.erf(mp.sqrt(t))) ** d
            poly = mp.fsum((-t) ** k * mk[k] / mp.factorial(k) for k in range(n + 1))
            return (m - poly) * t ** (-alpha - 1)

        tail = mp.quad(integrand, [t0, 2, 10, 100, mp.inf])
        return float((head + tail) / mp.gamma(-alpha))


def exact(family: str, params, d, lo=None, hi=None) -> float:
    if family == "product_peak":
        return product_peak(params, d, lo, hi)
    if family == "gaussian":
        return gaussian(params, d, lo, hi)
    if family == "oscillatory":
        return oscillatory(params, d, lo, hi)
    if family == "corner_peak":
        if lo is not None and (np.any(np.asarray(lo) != 0) or np.any(np.asarray(hi) != 1)):
            raise ValueError("corner_peak closed form is for the unit cube")
        return corner_peak(params, d)
    if family == "monomial":
        lo = np.zeros(d) if lo is None else lo
        hi = np.ones(d) if hi is None else hi
        return float(monomial(params, lo, hi))
    if family == "c0":
        return c0(params, d, lo, hi)
    if family == "discontinuous":
        return discontinuous(params, d, lo, hi)
    if family == "box":
        if lo is not None and (np.any(np.asarray(lo) != 0) or np.any(np.asarray(hi) != 1)):
            raise ValueError("box closed form is for the unit cube")
        return box(params, d)
    raise ValueError(family)


def gaussian_grad(params, d):
    """Closed-form gradient of the unit-cube Gaussian integral with respect to
    theta = (a_1..a_d, u_1..u_d): returns (I, dI/da[d], dI/du[d]) as floats.

    With G_i(a, u) = int_0^1 exp(-a^2 (x-u)^2) dx:
      dG/du = exp(-a^2 u^2) - exp(-a^2 (1-u)^2)
      dG/da = -G/a + ((1-u) exp(-a^2 (1-u)^2) + u exp(-a^2 u^2)) / a
    and dI/dtheta_i = (I / G_i) dG_i/dtheta_i.
    """
    a = [mp.mpf(float(x)) for x in params[:d]]
    u = [mp.mpf(float(x)) for x in params[d:2 * d]]
    G = [mp.sqrt(mp.pi) / (2 * a[i]) * (mp.erf(a[i] * (1 - u[i])) + mp.erf(a[i] * u[i]))
         for i in range(d)]
    I = mp.mpf(1)
    for g in G:
        I *= g
    dA, dU = [], []
    for i in range(d):
        e0 = mp.exp(-a[i] ** 2 * u[i] ** 2)
        e1 = mp.exp(-a[i] ** 2 * (1 - u[i]) ** 2)
        dGu = e0 - e1
        dGa = -G[i] / a[i] + ((1 - u[i]) * e1 + u[i] * e0) / a[i]
        dA.append(float(I / G[i] * dGa))
        dU.append(float(I / G[i] * dGu))
    return float(I), np.array(dA), np.array(dU)
