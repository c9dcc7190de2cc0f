// pg_eval_kernels.hpp -- gfx950 EVALUATE kernels of PAGANI (Section 3.2).
//
// EVALUATE is FP64-VALU bound: one lane owns one region for the whole
// cubature rule (64 regions per block), so the rule's weighted sums need no
// cross-lane reduction. The point set is cut into work units of four points
// (one axis: +-lambda2, +-lambda3; one pair of axes: four sign choices of
// lambda4; four sign vectors of lambda5); W waves of a block share the same
// 64 regions and take every W-th unit, so small lists still fill the chip.
// Axis and pair units are unrolled with the moving axes as compile-time
// indices: a point differs from the centre only in those coordinates, each
// one FMA, x_k = c_k + s_k (lambda h_k), which rounds exactly like
// c_k + s_k * (lambda * h_k); the untouched coordinates stay the centre's
// registers, and the integrand's arithmetic on them is shared by the four
// points of a unit where the compiler can see it is the same. Which unit a
// wave takes is decided in scalar registers (wave-uniform branches).
#pragma once

#include "pg_internal.hpp"

#include <hip/hip_runtime.h>

namespace pg {

// ---------------------------------------------------------------------------
// Integrands (parameter layout: see FParams). Inlined into the evaluation.
// ---------------------------------------------------------------------------
template <int FAM, int D>
__device__ __forceinline__ double integrand(const double *x, const FParams &P) {
    if constexpr (FAM == PG_PRODUCT_PEAK) {
        double den = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = x[k] - P.p[D + k];
            den *= fma(t, t, P.p[k]);
        }
        return rcp_pos(den);
    } else if constexpr (FAM == PG_GAUSSIAN) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = x[k] - P.p[D + k];
            s = fma(P.p[k] * t, t, s);
        }
        return exp_nonpos(-s);
    } else if constexpr (FAM == PG_OSCILLATORY) {
        double s = P.p[D];
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], x[k], s);
        return cos(s);
    } else if constexpr (FAM == PG_CORNER_PEAK) {
        double s = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], x[k], s);
        return rcp_pos(pow_int<D + 1>(s));
    } else if constexpr (FAM == PG_MONOMIAL) {   // test family
        double r = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int e = (int)P.p[k];
            for (int j = 0; j < e; ++j) r *= x[k];
        }
        return r;
    } else if constexpr (FAM == PG_C0) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], fabs(x[k] - P.p[D + k]), s);
        return exp_nonpos(-s);
    } else if constexpr (FAM == PG_DISCONTINUOUS) {
        double s = 0.0;
        bool in = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            in = in && (x[k] < P.p[D + k]);
            s = fma(P.p[k], x[k], s);
        }
        const double e = exp(s);
        return in ? e : 0.0;
    } else {                                     // box: (sum x^2)^p
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(x[k], x[k], s);
        // p[1] = 0: integer power p[2] by squaring; 1: s^p[2] sqrt(s);
        // 2: pow
        if (P.p[1] == 2.0) return pow(s, P.p[0]);
        int e = (int)P.p[2];
        double r = P.p[1] == 1.0 ? sqrt(s) : 1.0, b = s;
        while (e) {
            if (e & 1) r *= b;
            b *= b;
            e >>= 1;
        }
        return r;
    }
}

// Error of a region from its null-rule magnitudes (PG_ERR_NULL4; see
// NULL_KAPPA): a ratio is 0 when its numerator is 0, infinite when only
// its denominator is.
__device__ __forceinline__ double null4_error(double kappa, double e5,
                                              double e3, double e1) {
    const double inf = __builtin_inf();
    const double r31 = e3 == 0.0 ? 0.0 : (e1 == 0.0 ? inf : e3 / e1);
    const double r53 = e5 == 0.0 ? 0.0 : (e3 == 0.0 ? inf : e5 / e3);
    const double r = fmax(r31, r53);
    if (r <= NULL_RC) return kappa * r * r * e3;
    return fmax(fmax(e5, e3), e1);
}

// ---------------------------------------------------------------------------
// EVALUATE
// ---------------------------------------------------------------------------
// BATCH: the integrand's parameters are per region, table[inst[i]] (many
// integrals in one list); otherwise P for every region.
template <int FAM, int D, bool BATCH>
__global__ void __launch_bounds__(64 * EVAL_MAX_WAVES)
k_evaluate(const FParams P, const Rule R, int64_t n,
           const double *__restrict__ lo, const double *__restrict__ wid,
           int64_t ld, double *__restrict__ V, double *__restrict__ E,
           uint8_t *__restrict__ K, const uint32_t *__restrict__ inst,
           const FParams *__restrict__ table) {
    constexpr int NPAIR = D * (D - 1) / 2;
    constexpr int N5 = (1 << D) / 4;         // units of four orbit-5 points
    extern __shared__ double lds[];          // Dbuf[D][64], part[W][5][64]

    const int lane = threadIdx.x & 63;
    // the wave index is the same on every lane: say so, so that the unit
    // loop, the point signs and the pair decoding stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;           // 1, 2, 4 or 8 (launch_evaluate)
    const int wmask = W - 1;                 // unit u goes to wave u mod W
    const int64_t r0 = (int64_t)blockIdx.x * 64 + lane;
    const int64_t r = r0 < n ? r0 : n - 1;   // tail lanes recompute the last

    FParams lp;
    if constexpr (BATCH) {
        const FParams *src = table + inst[r];
#pragma unroll
        for (int k = 0; k < 2 * D + 1; ++k) lp.p[k] = src->p[k];
    }
    const FParams &PP = BATCH ? lp : P;

    double c[D], h[D], l4[D], l5[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        h[k] = wid[k * ld + r] * 0.5;
        c[k] = lo[k * ld + r] + h[k];
        l4[k] = mul_rounded(R.lam4, h[k]);
        l5[k] = mul_rounded(R.lam5, h[k]);
    }

    double fc = 0.0;
    if (wave < D) fc = integrand<FAM, D>(c, PP);   // axis units need f(c)

    double S2 = 0.0, S3 = 0.0, S4 = 0.0, S5 = 0.0, nmax = 0.0;
    double *Dbuf = lds;

    // axis units: the axis is a compile-time index, so only the moving
    // coordinate is recomputed (unit u = i goes to wave u mod W)
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if ((i & wmask) != wave) continue;
        double f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x[D];
#pragma unroll
            for (int k = 0; k < D; ++k) x[k] = c[k];
            const double lam = q < 2 ? R.lam2 : R.lam3;
            x[i] = fma((q & 1) ? -1.0 : 1.0, mul_rounded(lam, h[i]), c[i]);
            f[q] = integrand<FAM, D>(x, PP);
        }
        const double P2 = f[0] + f[1], P3 = f[2] + f[3];
        S2 += P2;
        S3 += P3;
        // lambda2^2 / lambda3^2 = 1/7, as a product by RN(1/7): a division
        // costs ten instructions, and the split axis is chosen with a
        // relative tie margin far above this rounding
        constexpr double SEVENTH = 1.0 / 7.0;
        Dbuf[i * 64 + lane] = fabs((P2 - 2.0 * fc) - (P3 - 2.0 * fc) * SEVENTH);
        const double nm = (fabs(f[0]) + fabs(f[1])) +
                          (fabs(f[2]) + fabs(f[3])) * SEVENTH +
                          (12.0 / 7.0) * fabs(fc);
        nmax = fmax(nmax, nm);
    }
    // pair units, pairs in row order, unit u = D + pair index
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
            const int u = D + i * (2 * D - i - 1) / 2 + (j - i - 1);
            if ((u & wmask) != wave) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double x[D];
#pragma unroll
                for (int k = 0; k < D; ++k) x[k] = c[k];
                x[i] = fma((q & 2) ? -1.0 : 1.0, l4[i], c[i]);
                x[j] = fma((q & 1) ? -1.0 : 1.0, l4[j], c[j]);
                S4 += integrand<FAM, D>(x, PP);
            }
        }
    }
    // vertex units
    {
        int u0 = D + NPAIR;
        int m = wave - (u0 & wmask);
        if (m < 0) m += W;
        // The families below are functions of per-axis terms combined by
        // one operation: the Gaussian of the sum of a_k^2 (x_k - u_k)^2,
        // the corner peak and the oscillatory of the sum of a_k x_k, the
        // product peak of the product of a_k^-2 + (x_k - u_k)^2. A vertex's
        // coordinates are, axis by axis, one of the two rounded values
        // c_k + l5_k and c_k - l5_k (the points every other family
        // evaluates), so its terms are computed once per axis and sign; a
        // unit of four vertices then combines D - 2 terms it shares and two
        // of its own per vertex. The rounding differs from the point-by-
        // point form only in the order the terms are combined (a few ulps;
        // the Gaussian's and the peaks' terms are positive, so nothing
        // cancels).
        constexpr bool SEP = FAM == PG_GAUSSIAN || FAM == PG_CORNER_PEAK ||
                             FAM == PG_OSCILLATORY || FAM == PG_PRODUCT_PEAK;
        constexpr bool PROD = FAM == PG_PRODUCT_PEAK;
        if constexpr (SEP) {
            double qp[D], qm[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double xp = fma(1.0, l5[k], c[k]);
                const double xm = fma(-1.0, l5[k], c[k]);
                if constexpr (FAM == PG_GAUSSIAN) {
                    const double tp = xp - PP.p[D + k], tm = xm - PP.p[D + k];
                    qp[k] = (PP.p[k] * tp) * tp;
                    qm[k] = (PP.p[k] * tm) * tm;
                } else if constexpr (FAM == PG_PRODUCT_PEAK) {
                    const double tp = xp - PP.p[D + k], tm = xm - PP.p[D + k];
                    qp[k] = fma(tp, tp, PP.p[k]);
                    qm[k] = fma(tm, tm, PP.p[k]);
                } else {
                    qp[k] = PP.p[k] * xp;
                    qm[k] = PP.p[k] * xm;
                }
            }
            auto join = [](double x, double y) { return PROD ? x * y : x + y; };
            auto value = [&](double t) {
                if constexpr (FAM == PG_GAUSSIAN) return exp_nonpos(-t);
                else if constexpr (FAM == PG_CORNER_PEAK)
                    return rcp_pos(pow_int<D + 1>(1.0 + t));
                else if constexpr (FAM == PG_OSCILLATORY) return cos(PP.p[D] + t);
                else return rcp_pos(t);
            };
            auto unit = [&](int mm) {
                double base = PROD ? 1.0 : 0.0;
#pragma unroll
                for (int k = 2; k < D; ++k) {
                    const double q = (((4 * mm) >> k) & 1) ? qm[k] : qp[k];
                    base = k == 2 ? q : join(base, q);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double s01 = join((q & 1) ? qm[0] : qp[0],
                                            (q & 2) ? qm[1] : qp[1]);
                    S5 += value(D > 2 ? join(s01, base) : s01);
                }
            };
            if constexpr (N5 <= 16) {
                // unrolled: the unit's signs are compile-time, so its terms
                // are picked without selects (up to d = 6)
#pragma unroll
                for (int mm = 0; mm < N5; ++mm)
                    if (((u0 + mm) & wmask) == wave) unit(mm);
            } else {
                for (; m < N5; m += W) unit(m);
            }
        } else {
            for (; m < N5; m += W) {
                double x[D];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = 4 * m + q;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        x[k] = fma(((b >> k) & 1) ? -1.0 : 1.0, l5[k], c[k]);
                    S5 += integrand<FAM, D>(x, PP);
                }
            }
        }
    }

    if (W > 1) {
        double *part = lds + D * 64;
        part[(wave * 5 + 0) * 64 + lane] = S2;
        part[(wave * 5 + 1) * 64 + lane] = S3;
        part[(wave * 5 + 2) * 64 + lane] = S4;
        part[(wave * 5 + 3) * 64 + lane] = S5;
        part[(wave * 5 + 4) * 64 + lane] = nmax;
        __syncthreads();
        if (wave == 0) {
            for (int q = 1; q < W; ++q) {
                S2 += part[(q * 5 + 0) * 64 + lane];
                S3 += part[(q * 5 + 1) * 64 + lane];
                S4 += part[(q * 5 + 2) * 64 + lane];
                S5 += part[(q * 5 + 3) * 64 + lane];
                nmax = fmax(nmax, part[(q * 5 + 4) * 64 + lane]);
            }
        }
    } else {
        __syncthreads();
    }

    if (wave == 0 && r0 < n) {
        double vol = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) vol *= 2.0 * h[k];
        const double s7 = R.w7[0] * fc + R.w7[1] * S2 + R.w7[2] * S3 +
                          R.w7[3] * S4 + R.w7[4] * S5;
        const double sn = R.wn[0] * fc + R.wn[1] * S2 + R.wn[2] * S3 +
                          R.wn[3] * S4 + R.wn[4] * S5;
        V[r0] = vol * s7;
        if (R.err_rule == PG_ERR_NULL4) {
            double nv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                nv[q] = vol * (R.nul[q][0] * fc + R.nul[q][1] * S2 +
                               R.nul[q][2] * S3 + R.nul[q][3] * S4 +
                               R.nul[q][4] * S5);
            E[r0] = null4_error(R.kappa, fabs(nv[0]),
                                sqrt(0.5 * (nv[1] * nv[1] + nv[2] * nv[2])),
                                fabs(nv[3]));
        } else {
            E[r0] = fabs(vol * sn);
        }
        double dk[D], dmax = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dk[k] = Dbuf[k * 64 + lane];
            dmax = fmax(dmax, dk[k]);
        }
        const double thr = dmax - 1e-10 * dmax - 1e-12 * nmax;
        int best = 0;
        double bw = -1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (dk[k] >= thr && h[k] > bw) { best = k; bw = h[k]; }
        }
        K[r0] = (uint8_t)best;
    }
}

// ---------------------------------------------------------------------------
// Integrand values at n points x[k * ld + i] (one lane per point)
// ---------------------------------------------------------------------------
template <int FAM, int D>
__global__ void __launch_bounds__(256)
k_fvalues(const FParams P, int64_t n, const double *__restrict__ x,
          int64_t ld, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = x[k * ld + i];
    y[i] = integrand<FAM, D>(xi, P);
}

// ---------------------------------------------------------------------------
// Kernel tables of one family (instantiated one family per object file,
// pg_eval_family.hip, so that the families compile in parallel)
// ---------------------------------------------------------------------------
typedef void (*EvalKernel)(const FParams, const Rule, int64_t, const double *,
                           const double *, int64_t, double *, double *,
                           uint8_t *, const uint32_t *, const FParams *);
typedef void (*FvalKernel)(const FParams, int64_t, const double *, int64_t,
                           double *);

template <int FAM, bool BATCH>
EvalKernel eval_dims(int d) {
    switch (d) {
    case 2: return k_evaluate<FAM, 2, BATCH>;
    case 3: return k_evaluate<FAM, 3, BATCH>;
    case 4: return k_evaluate<FAM, 4, BATCH>;
    case 5: return k_evaluate<FAM, 5, BATCH>;
    case 6: return k_evaluate<FAM, 6, BATCH>;
    case 7: return k_evaluate<FAM, 7, BATCH>;
    case 8: return k_evaluate<FAM, 8, BATCH>;
    case 9: return k_evaluate<FAM, 9, BATCH>;
    case 10: return k_evaluate<FAM, 10, BATCH>;
    default: return nullptr;
    }
}

template <int FAM>
EvalKernel eval_family(int d, bool batch) {
    return batch ? eval_dims<FAM, true>(d) : eval_dims<FAM, false>(d);
}

template <int FAM>
FvalKernel fval_family(int d) {
    switch (d) {
    case 2: return k_fvalues<FAM, 2>;
    case 3: return k_fvalues<FAM, 3>;
    case 4: return k_fvalues<FAM, 4>;
    case 5: return k_fvalues<FAM, 5>;
    case 6: return k_fvalues<FAM, 6>;
    case 7: return k_fvalues<FAM, 7>;
    case 8: return k_fvalues<FAM, 8>;
    case 9: return k_fvalues<FAM, 9>;
    case 10: return k_fvalues<FAM, 10>;
    default: return nullptr;
    }
}

}  // namespace pg
