// pg_adjoint.hip -- gfx950 kernels for the parameter derivative of the
// estimate over the partition a run converges on.
//
// The estimate is the sum of the degree-7 rule values of the partition's
// leaves (every region finished on the way, and the live list when the run
// ends). Each rule value is a weighted sum of f at points that do not move
// with the parameters, so dI/dtheta is the same weighted sum of df/dtheta
// over the leaves' points. The leaves of an iteration are still in the
// current list when its decisions are known, so the derivative is
// accumulated there, one launch per iteration, and no leaf is stored
// (unless the caller asks for the partition itself).
//
// Layout: one block per (segment, quarter): the block finds the segment's
// leaves (ballot prefix into LDS), then one lane per leaf walks the leaf's
// points; partial sums per block in a fixed order, then per integral.
#include "pg_device.hpp"

#include <hip/hip_runtime.h>

#include <utility>

namespace pg {

namespace {

// Waves each SIMD must be able to hold (caps the registers of a lane at
// 512 / ADJ_WAVES_PER_SIMD): the point walk is a chain of dependent FP64
// operations, and more resident waves hide their latency.
constexpr int ADJ_WAVES_PER_SIMD = 2;

// Parameters as the derivative kernels read them: p as FParams would hold
// them for the integrand, and gs[q] the constant factor of parameter q's
// derivative (see point_grad):
//   product peak: p[k] = a_k^-2, p[d+k] = u_k;  gs = 2 a_k^-3, 2
//   gaussian:     p[k] = a_k,    p[d+k] = u_k;  gs = -2 a_k, 2 a_k^2
//   oscillatory:  p[k] = a_k,    p[d] = 2 pi u_1;  gs = -1, -2 pi
//   corner peak:  p[k] = a_k;  gs = -(d+1)
template <int FAM, int D>
constexpr int n_grad() {
    return (FAM == PG_PRODUCT_PEAK || FAM == PG_GAUSSIAN) ? 2 * D
           : FAM == PG_OSCILLATORY ? D + 1 : D;
}

// g += wgt * (df/dtheta at x) / gs: each family's parameter derivatives
// share a constant factor per parameter, applied once per integral after
// the sums (k_batch_grad_reduce):
//   gaussian  f = exp(-sum a^2 t^2), t = x - u:
//             df/da_k = -2 a_k (t_k^2 f),   df/du_k = 2 a_k^2 (t_k f)
//   product   f = prod r_k, r_k = 1 / (a_k^-2 + t_k^2):
//             df/da_k = 2 a_k^-3 (f r_k),   df/du_k = 2 (f t_k r_k)
//   oscillatory f = cos(phi), phi = 2 pi u_1 + sum a x:
//             df/da_k = -(x_k sin phi),     df/du_1 = -2 pi (sin phi)
//   corner    f = s^-(d+1), s = 1 + sum a x:
//             df/da_k = -(d+1) (x_k s^-(d+2))
// The Gaussian's point term from t_k = x_k - u_k: f = e^-s, s the sum of
// (a_k t_k)^2; d/du_k = 2 a_k^2 t_k f and d/da_k = -2 a_k t_k^2 f, whose
// constant factors gs are applied once per integral.
template <int D>
__device__ __forceinline__ void gauss_grad_t(const double (&t)[D],
                                             const GParams &P, double wgt,
                                             double *g) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double at = P.p[k] * t[k];
        s = fma(at, at, s);
    }
    const double wf = wgt * exp_nonpos(-s);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double wt = wf * t[k];
        g[D + k] += wt;
        g[k] = fma(wt, t[k], g[k]);
    }
}

template <int FAM, int D>
__device__ __forceinline__ void point_grad(const double (&x)[D],
                                           const GParams &P, double wgt,
                                           double *g) {
    if constexpr (FAM == PG_GAUSSIAN) {
        double t[D];
#pragma unroll
        for (int k = 0; k < D; ++k) t[k] = x[k] - P.p[D + k];
        gauss_grad_t<D>(t, P, wgt, g);
    } else if constexpr (FAM == PG_PRODUCT_PEAK) {
        double t[D], r[D], f = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            t[k] = x[k] - P.p[D + k];
            r[k] = rcp_pos(fma(t[k], t[k], P.p[k]));
            f *= r[k];
        }
        const double wf = wgt * f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double wr = wf * r[k];
            g[k] += wr;
            g[D + k] = fma(wr, t[k], g[D + k]);
        }
    } else if constexpr (FAM == PG_OSCILLATORY) {
        double phi = P.p[D];
#pragma unroll
        for (int k = 0; k < D; ++k) phi = fma(P.p[k], x[k], phi);
        const double ws = wgt * sin(phi);
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] = fma(x[k], ws, g[k]);
        g[D] += ws;
    } else {
        double s = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], x[k], s);
        const double wf = wgt * pow_int<D + 2>(rcp_pos(s));
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] = fma(x[k], wf, g[k]);
    }
}

// Derivative of one region's rule value (orbit weights times the volume,
// wv, added into g), over
// the points of the degree-7 rule: the centre; the axis units (+-lambda2,
// +-lambda3 on one axis) and pair units (the four sign choices of lambda4
// on two axes), unrolled with the moving axes as compile-time indices so a
// point moves one or two coordinates off the centre with one FMA each,
// x_k = c_k + s_k (lambda h_k) as the evaluation rounds it; and the 2^d
// vertices at lambda5, four per loop step.
template <int FAM, int D>
__device__ __forceinline__ void region_grad(const double (&c)[D],
                                            const double (&h)[D],
                                            const GParams &P, const Rule &R,
                                            const double (&wv)[5], double *g) {
    point_grad<FAM, D>(c, P, wv[0], g);
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            double x[D];
#pragma unroll
            for (int k = 0; k < D; ++k) x[k] = c[k];
            const double lam = q < 2 ? R.lam2 : R.lam3;
            x[i] = fma((q & 1) ? -1.0 : 1.0, mul_rounded(lam, h[i]), c[i]);
            point_grad<FAM, D>(x, P, q < 2 ? wv[1] : wv[2], g);
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                double x[D];
#pragma unroll
                for (int k = 0; k < D; ++k) x[k] = c[k];
                x[i] = fma((q & 2) ? -1.0 : 1.0, mul_rounded(R.lam4, h[i]), c[i]);
                x[j] = fma((q & 1) ? -1.0 : 1.0, mul_rounded(R.lam4, h[j]), c[j]);
                point_grad<FAM, D>(x, P, wv[3], g);
            }
        }
    }
    if constexpr (FAM == PG_GAUSSIAN && D <= 6) {
        // t_k at the two vertex coordinates of each axis, once per region;
        // the vertices, unrolled, pick theirs at compile time (same values
        // and order of sums as the point-by-point walk below)
        double tp[D], tm[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double l5 = mul_rounded(R.lam5, h[k]);
            tp[k] = fma(1.0, l5, c[k]) - P.p[D + k];
            tm[k] = fma(-1.0, l5, c[k]) - P.p[D + k];
        }
#pragma unroll
        for (int b = 0; b < (1 << D); ++b) {
            double t[D];
#pragma unroll
            for (int k = 0; k < D; ++k) t[k] = ((b >> k) & 1) ? tm[k] : tp[k];
            gauss_grad_t<D>(t, P, wv[4], g);
        }
    } else {
        for (int m = 0; m < (1 << D) / 4; ++m) {
#pragma unroll 2
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * m + q;
                double x[D];
#pragma unroll
                for (int k = 0; k < D; ++k)
                    x[k] = fma(((b >> k) & 1) ? -1.0 : 1.0,
                               mul_rounded(R.lam5, h[k]), c[k]);
                point_grad<FAM, D>(x, P, wv[4], g);
            }
        }
    }
}

// Leaves of one segment: every region of an integral that ends this
// iteration; otherwise the regions that are not active (active: A_rel, and
// E > t_acc after an accepted threshold -- the count pass's test).
template <int FAM, int D>
__global__ void __launch_bounds__(LIST_THREADS, ADJ_WAVES_PER_SIMD)
k_batch_adjoint(const BSeg *__restrict__ segs, const BInst *__restrict__ inst,
                const SearchState *__restrict__ states,
                const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
                const double *__restrict__ lo, const double *__restrict__ w,
                int64_t ld, const GParams *__restrict__ gtab, const Rule R,
                double *__restrict__ gpart, int64_t ncol,
                const uint32_t *__restrict__ offsets, LeafOut out) {
    constexpr int NP = n_grad<FAM, D>();
    constexpr int NW = LIST_THREADS / 64;
    __shared__ uint16_t idx[BSEG];
    __shared__ uint32_t wtot[NW];
    __shared__ double red[NW][NP];
    const int64_t s = blockIdx.x / ADJ_SPLIT;
    const int part = blockIdx.x % ADJ_SPLIT;
    const BSeg sg = segs[s];
    const BInst &I = inst[sg.slot];
    const SearchState &S = states[sg.slot];
    const int mode = !I.live ? 0 : ((I.searching && S.ok) ? 2 : 1);
    const double t = S.t_acc;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t nleaf = 0;
    for (int64_t c0 = sg.start; c0 < sg.end; c0 += LIST_THREADS) {
        const int64_t i = c0 + threadIdx.x;
        bool leaf = false;
        if (i < sg.end) {
            if (mode == 0) {
                leaf = true;
            } else {
                const bool act = A_rel[i] && (mode == 1 || E[i] > t);
                leaf = !act;
            }
        }
        const uint64_t b = __ballot(leaf);
        const uint32_t pre = (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wave] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t base = nleaf, tot = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q < wave) base += wtot[q];
            tot += wtot[q];
        }
        if (leaf) idx[base + pre] = (uint16_t)(i - sg.start);
        nleaf += tot;
        __syncthreads();
    }
    const GParams P = gtab[sg.slot];
    // leaves of this segment before it in its integral's leaf order
    const int64_t leaf0 = I.fin_base + (sg.start - I.start) -
                          (mode == 0 ? 0 : (int64_t)offsets[s]);
    double G[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) G[q] = 0.0;
    for (uint32_t j = part * LIST_THREADS + threadIdx.x; j < nleaf;
         j += ADJ_SPLIT * LIST_THREADS) {
        const int64_t i = sg.start + idx[j];
        double c[D], h[D], vol = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double wk = w[k * ld + i], lk = lo[k * ld + i];
            h[k] = wk * 0.5;
            c[k] = lk + h[k];
            vol *= wk;
            if (out.lo) {
                const int64_t pos = out.base + leaf0 + j;
                out.lo[k * out.ld + pos] = lk;
                out.w[k * out.ld + pos] = wk;
            }
        }
        if (out.owner) out.owner[out.base + leaf0 + j] = I.owner;
        double wv[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) wv[o] = vol * R.w7[o];
        region_grad<FAM, D>(c, h, P, R, wv, G);
    }
    // fixed-order block sum: butterfly within waves, then waves in order
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        double v = G[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NP) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) v += red[q][threadIdx.x];
        gpart[(int64_t)threadIdx.x * ncol + blockIdx.x] = v;
    }
}

// Per integral: its columns of gpart added in a fixed order, times the
// parameter's constant factor.
__global__ void __launch_bounds__(LIST_THREADS)
k_batch_grad_reduce(const int32_t *__restrict__ order,
                    const BInst *__restrict__ inst,
                    const GParams *__restrict__ gtab, int np,
                    const double *__restrict__ gpart, int64_t ncol,
                    double *__restrict__ git) {
    __shared__ double red[LIST_THREADS];
    const int slot = order[blockIdx.x];
    const BInst &I = inst[slot];
    const int64_t c0 = I.seg0 * ADJ_SPLIT, c1 = (I.seg0 + I.nseg) * ADJ_SPLIT;
    for (int q = 0; q < np; ++q) {
        double v = 0.0;
        for (int64_t c = c0 + threadIdx.x; c < c1; c += LIST_THREADS)
            v += gpart[(int64_t)q * ncol + c];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int o = LIST_THREADS / 2; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            git[(int64_t)slot * GRAD_MAX + q] = red[0] * gtab[slot].gs[q];
        __syncthreads();
    }
}

using AdjFn = void (*)(const BSeg *, const BInst *, const SearchState *,
                       const uint8_t *, const double *, const double *,
                       const double *, int64_t, const GParams *, const Rule,
                       double *, int64_t, const uint32_t *, LeafOut);

template <int FAM, int... Ds>
constexpr AdjFn pick(int d, std::integer_sequence<int, Ds...>) {
    AdjFn f = nullptr;
    ((f = (d == Ds ? &k_batch_adjoint<FAM, Ds> : f)), ...);
    return f;
}

AdjFn adjoint_kernel(int family, int d) {
    using Dims = std::integer_sequence<int, 2, 3, 4, 5, 6, 7, 8, 9, 10>;
    switch (family) {
    case PG_PRODUCT_PEAK: return pick<PG_PRODUCT_PEAK>(d, Dims{});
    case PG_GAUSSIAN: return pick<PG_GAUSSIAN>(d, Dims{});
    case PG_OSCILLATORY: return pick<PG_OSCILLATORY>(d, Dims{});
    case PG_CORNER_PEAK: return pick<PG_CORNER_PEAK>(d, Dims{});
    default: return nullptr;
    }
}

}  // namespace

int grad_nparams(int family, int d) {
    switch (family) {
    case PG_PRODUCT_PEAK: case PG_GAUSSIAN: return 2 * d;
    case PG_OSCILLATORY: return d + 1;
    case PG_CORNER_PEAK: return d;
    default: return -1;
    }
}

bool adjoint_supported(int family, int d) {
    return d >= PG_DIM_MIN && d <= PG_DIM_MAX && adjoint_kernel(family, d);
}

hipError_t launch_batch_adjoint(hipStream_t st, int family, int d,
                                int64_t nseg, const BSeg *segs,
                                const BInst *inst, const SearchState *states,
                                const uint8_t *A_rel, const double *E,
                                const double *lo, const double *w, int64_t ld,
                                const GParams *gtab, const Rule &R,
                                double *gpart, const uint32_t *offsets,
                                const LeafOut &out) {
    if (nseg <= 0) return hipSuccess;
    AdjFn k = adjoint_kernel(family, d);
    if (!k) return hipErrorInvalidValue;
    const int64_t ncol = nseg * ADJ_SPLIT;
    hipLaunchKernelGGL(k, dim3((unsigned)ncol), dim3(LIST_THREADS), 0, st,
                       segs, inst, states, A_rel, E, lo, w, ld, gtab, R, gpart,
                       ncol, offsets, out);
    return hipGetLastError();
}

hipError_t launch_batch_grad_reduce(hipStream_t st, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const GParams *gtab, int np,
                                    const double *gpart, int64_t nseg,
                                    double *git) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_grad_reduce, dim3(nslots), dim3(LIST_THREADS), 0,
                       st, order, inst, gtab, np, gpart, nseg * ADJ_SPLIT, git);
    return hipGetLastError();
}

}  // namespace pg
