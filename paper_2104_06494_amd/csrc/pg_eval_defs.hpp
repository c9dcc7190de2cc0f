// pg_eval_defs.hpp -- what the EVALUATE kernel is built from besides
// pg_eval_kernels.hpp: the integrand parameters and rule constants it takes
// by value, its exponential and its launch bound (gfx950). Not part of the
// public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pagani.h"

namespace pg {

// Waves (at most) sharing the 64 regions of an EVALUATE block.
constexpr int EVAL_MAX_WAVES = 8;

// e^x for x <= 0 (the Gaussian's and the C0 integrand's exponent), no
// special cases: Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, with ln 2
// split into two doubles and the reduction done by two FMAs; e^r by the
// degree-11 polynomial interpolating e^r at the 12 Chebyshev points of
// [-ln2/2, ln2/2] (coefficients from 60-digit arithmetic rounded to double;
// the polynomial's relative error is 1.7e-17), Horner's rule; then 2^n by
// ldexp, which underflows gradually and reaches 0 below -745 without a
// test. Largest error 0.91 ulp on 2e5 points of [-745, 0] against a
// 40-digit reference. Domain: -1.4e9 < x <= 0 (below, n leaves int's range;
// the Gaussian's exponent stays in it unless some a_k^2 exceeds 1e9).
// NaN in, NaN out.
__device__ __forceinline__ double exp_nonpos(double x) {
    constexpr double LOG2E = 1.4426950408889634;      // RN(1 / ln 2)
    constexpr double LN2_HI = 0.6931471805599453;     // RN(ln 2)
    constexpr double LN2_LO = 2.3190468138462996e-17; // RN(ln 2 - LN2_HI)
    const double n = rint(x * LOG2E);
    double r = fma(-n, LN2_HI, x);
    r = fma(-n, LN2_LO, r);
    double q = 2.5110037605963777e-08;
    q = fma(q, r, 2.763263963904103e-07);
    q = fma(q, r, 2.755724091857897e-06);
    q = fma(q, r, 2.4801485482328494e-05);
    q = fma(q, r, 0.00019841269890047113);
    q = fma(q, r, 0.0013888888952314775);
    q = fma(q, r, 0.008333333333319601);
    q = fma(q, r, 0.0416666666664881);
    q = fma(q, r, 0.1666666666666668);
    q = fma(q, r, 0.5000000000000019);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    return ldexp(q, (int)n);
}

// a * b rounded to double by itself. HIP code is compiled with floating-
// point contraction across statements, which would fuse a product such as
// lambda h into the addition that uses it (c + lambda h with one rounding
// instead of two); a cubature point's coordinate is defined as the centre
// plus the rounded offset, so the offset's product is kept out of that.
__device__ __forceinline__ double mul_rounded(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// x^N for a compile-time N >= 1 by squaring: about log2 N multiplications
// instead of N - 1 (s^7 in 4, s^9 in 4), each rounded like any product.
template <int N>
__device__ __forceinline__ double pow_int(double x) {
    static_assert(N >= 1, "positive power");
    if constexpr (N == 1) {
        return x;
    } else {
        const double h = pow_int<N / 2>(x);
        if constexpr (N % 2 == 0) return h * h;
        else return (h * h) * x;
    }
}

// 1/x for a positive x whose reciprocal is a normal number (the product
// peak's and the corner peak's denominators, products of terms >= a^-2 and
// >= 1): the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r), each of which squares the relative error, so
// the result is within an ulp of 1/x; five instructions where the
// correctly rounded division with its scaling and special cases takes
// about ten. Outside that range (x <= 0, denormal, or 1/x beyond the
// largest double) the result is unspecified.
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Integrand parameters as the kernels take them (by value, in SGPRs):
//  product peak: p[k] = a_k^-2, p[d+k] = u_k
//  gaussian:     p[k] = a_k^2,  p[d+k] = u_k
//  oscillatory:  p[k] = a_k,    p[d]   = 2 pi u_1
//  corner peak:  p[k] = a_k
//  monomial:     p[k] = alpha_k
//  c0:           p[k] = a_k,    p[d+k] = u_k
//  discontinuous: p[k] = a_k,   p[d+k] = c_k
//  box:          p[0] = p, p[1] = 0 (integer p, p[2] = p), 1 (p = p[2] +
//                1/2), 2 (other p: pow)
struct FParams {
    double p[2 * PG_DIM_MAX + 2];
};

// Per-dimension rule constants: generators lambda2..5 and the weights of
// the degree-7 rule (w7) and of the null rule (wn = w7 - w5) per orbit.
// With err_rule = PG_ERR_NULL4 the error comes from the four null rules of
// the same points, nul[0] (degree 5), nul[1], nul[2] (degree 3) and nul[3]
// (degree 1), per-orbit weights with the degree-7 rule's norm.
struct Rule {
    double lam2, lam3, lam4, lam5;
    double w7[5];
    double wn[5];
    double nul[4][5];
    double kappa;
    int err_rule;
};

// Four-null-rule error (Section 3.2's comparison with four further
// rules): from e5 = |N1|, e3 = rms(N2, N3), e1 = |N4|, which for a smooth
// integrand shrink by a factor r ~ (h f-scale)^2 per two degrees while the
// degree-7 rule errs by ~h^8 (about r^2 e3 by the same decay), the
// estimate is kappa_d r^2 e3 when r = max(e3 / e1, e5 / e3) <= NULL_RC,
// else the largest of the three. kappa_d (Rule::kappa) is twice the larger
// of 1 and the worst limit ratio of true error to r^2 e3 over
// f = exp(a.x), rounded up to two digits.
constexpr double NULL_RC = 0.5;

}  // namespace pg
