// pg_kernels.hip -- gfx950 kernels of one PAGANI iteration (Algorithm 2).
//
// EVALUATE is FP64-VALU bound: one lane owns one region for the whole
// cubature rule (64 regions per block), so the rule's weighted sums need no
// cross-lane reduction. The point set is cut into work units of four points
// (one axis: +-lambda2, +-lambda3; one pair of axes: four sign choices of
// lambda4; four sign vectors of lambda5); W waves of a block share the same
// 64 regions and take every W-th unit, so small lists still fill the chip.
// The unit index is wave-uniform: which coordinates move, and with what
// sign, is decided in scalar registers, and every lane builds its point with
// one FMA per coordinate, x_k = c_k + s_k (lambda h_k), s_k in {-1, 0, 1},
// which rounds exactly like c_k + s_k * (lambda * h_k).
//
// The list kernels (classify, threshold trials, count, compact + split) are
// HBM bound; they stream SoA arrays with coalesced accesses and reduce in a
// fixed order (no floating-point atomics), so runs are bit-reproducible.
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
        return 1.0 / den;
    } else if constexpr (FAM == PG_GAUSSIAN) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double t = x[k] - P.p[D + k];
            s = fma(P.p[k] * t, t, s);
        }
        return exp(-s);
    } else if constexpr (FAM == PG_OSCILLATORY) {
        double s = P.p[D];
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], x[k], s);
        return cos(s);
    } else if constexpr (FAM == PG_CORNER_PEAK) {
        double s = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(P.p[k], x[k], s);
        double pw = s;
#pragma unroll
        for (int e = 0; e < D; ++e) pw *= s;   // s^(D+1)
        return 1.0 / pw;
    } else {                                     // monomial (test family)
        double r = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int e = (int)P.p[k];
            for (int j = 0; j < e; ++j) r *= x[k];
        }
        return r;
    }
}

// ---------------------------------------------------------------------------
// EVALUATE
// ---------------------------------------------------------------------------
constexpr int EVAL_MAX_WAVES = 8;

template <int FAM, int D>
__global__ void __launch_bounds__(64 * EVAL_MAX_WAVES)
k_evaluate(const FParams P, const Rule R, int64_t n,
           const double *__restrict__ lo, const double *__restrict__ wid,
           int64_t ld, double *__restrict__ V, double *__restrict__ E,
           uint8_t *__restrict__ K) {
    constexpr int NPAIR = D * (D - 1) / 2;
    constexpr int N5 = (1 << D) / 4;         // units of four orbit-5 points
    constexpr int U = D + NPAIR + N5;
    extern __shared__ double lds[];          // Dbuf[D][64], part[W][5][64]

    const int lane = threadIdx.x & 63;
    // the wave index is the same on every lane: say so, so that the unit
    // loop, the point signs and the pair decoding stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + lane;
    const int64_t r = r0 < n ? r0 : n - 1;   // tail lanes recompute the last

    double c[D], h[D], l4[D], l5[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        h[k] = wid[k * ld + r] * 0.5;
        c[k] = lo[k * ld + r] + h[k];
        l4[k] = R.lam4 * h[k];
        l5[k] = R.lam5 * h[k];
    }

    double fc = 0.0;
    if (wave < D) fc = integrand<FAM, D>(c, P);   // axis units need f(c)

    double S2 = 0.0, S3 = 0.0, S4 = 0.0, S5 = 0.0, nmax = 0.0;
    double *Dbuf = lds;

    for (int u = wave; u < U; u += W) {
        double x[D];
        if (u < D) {
            // orbits 2 and 3 along axis i, and its fourth difference
            const int i = u;
            double f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double lam = q < 2 ? R.lam2 : R.lam3;
                const double sg = (q & 1) ? -1.0 : 1.0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    x[k] = fma(k == i ? sg : 0.0, lam * h[k], c[k]);
                f[q] = integrand<FAM, D>(x, P);
            }
            const double P2 = f[0] + f[1], P3 = f[2] + f[3];
            S2 += P2;
            S3 += P3;
            Dbuf[i * 64 + lane] = fabs((P2 - 2.0 * fc) - (P3 - 2.0 * fc) / 7.0);
            const double nm = (fabs(f[0]) + fabs(f[1])) +
                              (fabs(f[2]) + fabs(f[3])) / 7.0 +
                              (12.0 / 7.0) * fabs(fc);
            nmax = fmax(nmax, nm);
        } else if (u < D + NPAIR) {
            // orbit 4: pair (i, j) with i < j, pairs in row order
            int i = 0, rem = u - D;
            while (rem >= D - 1 - i) { rem -= D - 1 - i; ++i; }
            const int j = i + 1 + rem;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double si = (q & 2) ? -1.0 : 1.0;
                const double sj = (q & 1) ? -1.0 : 1.0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    x[k] = fma(k == i ? si : (k == j ? sj : 0.0), l4[k], c[k]);
                S4 += integrand<FAM, D>(x, P);
            }
        } else {
            // orbit 5: sign vectors 4m..4m+3, bit k set = minus on axis k
            const int m = u - D - NPAIR;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * m + q;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    x[k] = fma(((b >> k) & 1) ? -1.0 : 1.0, l5[k], c[k]);
                S5 += integrand<FAM, D>(x, P);
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
        E[r0] = fabs(vol * sn);
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
// Deterministic block reductions (fixed shuffle tree, then waves in order)
// ---------------------------------------------------------------------------
struct Acc {
    double v, e, av, ae, mn, mx;
    uint32_t cnt;
    __device__ void init() {
        v = e = av = ae = 0.0;
        mn = __builtin_huge_val();
        mx = -__builtin_huge_val();
        cnt = 0;
    }
    __device__ void add(double V, double E, int a) {
        v += V;
        e += E;
        if (a) { av += V; ae += E; ++cnt; }
        mn = fmin(mn, E);
        mx = fmax(mx, E);
    }
    __device__ void merge(const Acc &o) {
        v += o.v; e += o.e; av += o.av; ae += o.ae;
        mn = fmin(mn, o.mn); mx = fmax(mx, o.mx);
        cnt += o.cnt;
    }
    __device__ void shfl_merge(int off) {
        Acc o;
        o.v = __shfl_xor(v, off);
        o.e = __shfl_xor(e, off);
        o.av = __shfl_xor(av, off);
        o.ae = __shfl_xor(ae, off);
        o.mn = __shfl_xor(mn, off);
        o.mx = __shfl_xor(mx, off);
        o.cnt = __shfl_xor(cnt, off);
        merge(o);
    }
};

// Reduces `a` over the block (LIST_THREADS threads); thread 0 writes slot s.
__device__ void block_reduce_store(Acc a, SegPartials part, int64_t s) {
    __shared__ Acc wacc[LIST_THREADS / 64];
    for (int off = 32; off >= 1; off >>= 1) a.shfl_merge(off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) wacc[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = wacc[0];
        for (int q = 1; q < LIST_THREADS / 64; ++q) t.merge(wacc[q]);
        part.v[s] = t.v;
        part.e[s] = t.e;
        part.av[s] = t.av;
        part.ae[s] = t.ae;
        part.emin[s] = t.mn;
        part.emax[s] = t.mx;
        part.cnt[s] = t.cnt;
    }
}

// ---------------------------------------------------------------------------
// TWO-LEVEL-ERROR + REL-ERR-CLASSIFY + per-segment sums
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(LIST_THREADS)
k_classify(int64_t n, int paired, const double *__restrict__ V,
           double *__restrict__ E, const double *__restrict__ Vp, double tau,
           int relerr, uint8_t *__restrict__ A, SegPartials part) {
    const int64_t b = blockIdx.x;
    Acc lo_acc, hi_acc;
    lo_acc.init();
    hi_acc.init();
    if (!paired) {
        const int64_t s0 = b * SEG, s1 = s0 + SEG < n ? s0 + SEG : n;
        for (int64_t i = s0 + threadIdx.x; i < s1; i += LIST_THREADS) {
            const double v = V[i], e = E[i];
            const int a = relerr ? (e > tau * fabs(v)) : 1;
            A[i] = (uint8_t)a;
            lo_acc.add(v, e, a);
        }
        block_reduce_store(lo_acc, part, b);
        return;
    }
    const int64_t half = n / 2;
    const int64_t nh = (half + SEG - 1) / SEG;
    const int64_t q0 = b * SEG, q1 = q0 + SEG < half ? q0 + SEG : half;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += LIST_THREADS) {
        const int64_t ia = q, ib = q + half;
        const double va = V[ia], vb = V[ib];
        double ea = E[ia], eb = E[ib];
        const double delta = fabs(va + vb - Vp[q]) / 4.0;
        const double S = ea + eb;
        if (S > 0.0) {
            const double g = 1.0 + 2.0 * delta / S;
            ea = ea * g + delta;
            eb = eb * g + delta;
        } else {
            ea = ea + delta;
            eb = eb + delta;
        }
        E[ia] = ea;
        E[ib] = eb;
        const int aa = relerr ? (ea > tau * fabs(va)) : 1;
        const int ab = relerr ? (eb > tau * fabs(vb)) : 1;
        A[ia] = (uint8_t)aa;
        A[ib] = (uint8_t)ab;
        lo_acc.add(va, ea, aa);
        hi_acc.add(vb, eb, ab);
    }
    block_reduce_store(lo_acc, part, b);
    block_reduce_store(hi_acc, part, nh + b);
}

// Per-segment count and sums of A = A_rel AND (E > t); E == nullptr: A_rel.
// With a search state, t is the accepted threshold (or none if it failed).
__global__ void __launch_bounds__(LIST_THREADS)
k_seg_count(int64_t n, int paired, double t, const double *__restrict__ V,
            const double *__restrict__ E, const uint8_t *__restrict__ A_rel,
            const SearchState *__restrict__ S, SegPartials part) {
    if (S) t = S->ok ? S->t_acc : -__builtin_huge_val();
    int64_t s0, s1;
    seg_range(blockIdx.x, n, paired, &s0, &s1);
    Acc acc;
    acc.init();
    for (int64_t i = s0 + threadIdx.x; i < s1; i += LIST_THREADS) {
        const double v = V[i], e = E ? E[i] : 0.0;
        acc.add(v, e, A_rel[i] && (!E || e > t));
    }
    block_reduce_store(acc, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Single-block totals of the segment partials + exclusive scan of the counts
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(SCAN_THREADS)
k_reduce_scan(int64_t nseg, SegPartials part, uint32_t *__restrict__ offsets,
              Totals *__restrict__ tot) {
    __shared__ uint64_t wsum[SCAN_THREADS / 64];
    __shared__ Acc wacc[SCAN_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (nseg + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t s0 = tid * per, s1 = s0 + per < nseg ? s0 + per : nseg;
    Acc a;
    a.init();
    uint64_t local = 0;
    for (int64_t s = s0; s < s1; ++s) {
        a.v += part.v[s];
        a.e += part.e[s];
        a.av += part.av[s];
        a.ae += part.ae[s];
        a.mn = fmin(a.mn, part.emin[s]);
        a.mx = fmax(a.mx, part.emax[s]);
        local += part.cnt[s];
    }
    // exclusive scan of `local` over the block
    uint64_t incl = local;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t wbase = 0;
    for (int q = 0; q < wave; ++q) wbase += wsum[q];
    uint64_t run = wbase + incl - local;
    for (int64_t s = s0; s < s1; ++s) {
        offsets[s] = (uint32_t)run;
        run += part.cnt[s];
    }
    // totals
    a.cnt = 0;
    for (int off = 32; off >= 1; off >>= 1) a.shfl_merge(off);
    if (lane == 0) wacc[wave] = a;
    __syncthreads();
    if (tid == 0) {
        Acc t = wacc[0];
        for (int q = 1; q < SCAN_THREADS / 64; ++q) t.merge(wacc[q]);
        uint64_t total = 0;
        for (int q = 0; q < SCAN_THREADS / 64; ++q) total += wsum[q];
        tot->v = t.v;
        tot->e = t.e;
        tot->av = t.av;
        tot->ae = t.ae;
        tot->emin = t.mn;
        tot->emax = t.mx;
        tot->cnt = (double)total;
        tot->pad = 0.0;
    }
}

// ---------------------------------------------------------------------------
// THRESHOLD-CLASSIFY (Algorithm 3) with its state on the device.
//
// The search is sequential -- each trial picks the next threshold from the
// previous outcome -- but the thresholds it can reach in its next
// TRIAL_DEPTH trials form a complete binary tree that depends only on the
// current threshold and on min/max E (raise: t + (max - t)/2, lower:
// t - (t - min)/2). One pass over the list counts, for all TRIAL_M nodes of
// that tree, the regions that stay active (A_rel AND E > t) and the sum of
// their errors; the tree is then walked exactly as the sequential search
// would walk it, which leaves the next root in the state.
// ---------------------------------------------------------------------------
__device__ inline void build_tree(const SearchState &S, double *thr) {
    thr[0] = S.t;
#pragma unroll
    for (int i = 0; 2 * i + 2 < TRIAL_M; ++i) {
        thr[2 * i + 1] = thr[i] + (S.mx - thr[i]) / 2.0;    // raise
        thr[2 * i + 2] = thr[i] - (thr[i] - S.mn) / 2.0;    // lower
    }
}

__global__ void k_search_init(SearchState *__restrict__ S, int64_t n,
                              double e_it, double allowance, int mem,
                              const Totals *__restrict__ minmax) {
    if (threadIdx.x != 0) return;
    SearchState s{};
    s.n = n;
    s.e_it = e_it;
    s.allowance = allowance;
    s.mem = mem;
    s.mn = minmax->emin;
    s.mx = minmax->emax;
    s.t = e_it / (double)n;
    s.P_max = 0.25;
    s.t_acc = -__builtin_huge_val();
    *S = s;
}

// Walks up to TRIAL_DEPTH levels of the tree (Algorithm 3's loop) given the
// totals of a pass: tot[m] regions stay active under node m's threshold and
// tot[TRIAL_M + m] is the sum of their errors.
__device__ void walk_tree(SearchState &st, const double *tot) {
    double thr[TRIAL_M];
    build_tree(st, thr);
    int node = 0;
    for (int level = 0; level < TRIAL_DEPTH; ++level) {
        if (st.trials >= THR_MAX_TRIALS) { st.done = 1; return; }
        const double tt = thr[node];
        ++st.trials;
        const double s_abar = (double)st.n - tot[node];
        const double e_abar = st.e_it - tot[TRIAL_M + node];
        int dir;
        if (s_abar > 0.5 * (double)st.n) {
            if (e_abar <= st.P_max * st.allowance) {
                st.done = 1;
                st.ok = 1;
                st.t_acc = tt;
                return;
            }
            dir = -1;                           // accuracy failed: lower t
        } else {
            dir = +1;                           // memory failed: raise t
        }
        if (st.last_dir != 0 && dir != st.last_dir) {
            ++st.dir_changes;
            if (st.mem) st.P_max = fmin(st.P_max + 0.10, 0.95);
            if (st.dir_changes >= THR_MAX_DIRCHG) { st.done = 1; return; }
        }
        st.last_dir = dir;
        st.t = dir > 0 ? tt + (st.mx - tt) / 2.0 : tt - (tt - st.mn) / 2.0;
        node = dir > 0 ? 2 * node + 1 : 2 * node + 2;
    }
}

// One pass over the list for the TRIAL_M thresholds of the current tree.
// Counts come from wave ballots (already wave totals, in scalar registers);
// the error sums are reduced through LDS (each wave writes its lanes' sums
// and TRIAL_M lanes add one row each) and then over the waves in order.
// The list is walked in wave-sized chunks so the loop is wave-uniform. The
// block sums go to k_trial_walk; the kernel boundary between the two makes
// them visible without any device-wide fence inside a kernel.
__global__ void __launch_bounds__(TRIAL_THREADS)
k_trials(int64_t n, const double *__restrict__ E,
         const uint8_t *__restrict__ A_rel, const SearchState *__restrict__ S,
         double *__restrict__ blk_part) {
    constexpr int NW = TRIAL_THREADS / 64;
    __shared__ double rows[NW][TRIAL_M][65];    // padded: no bank conflicts
    __shared__ double wsum[NW][2 * TRIAL_M];
    if (S->done) return;                        // same for every block
    double thr[TRIAL_M];
    build_tree(*S, thr);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t cnt[TRIAL_M];
    double ae[TRIAL_M];
#pragma unroll
    for (int m = 0; m < TRIAL_M; ++m) { cnt[m] = 0; ae[m] = 0.0; }
    const int64_t stride = (int64_t)gridDim.x * TRIAL_THREADS;
    for (int64_t i0 = (int64_t)blockIdx.x * TRIAL_THREADS + wave * 64; i0 < n;
         i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < n;
        const double e = valid ? E[i] : 0.0;
        const bool a = valid && A_rel[i] != 0;
#pragma unroll
        for (int m = 0; m < TRIAL_M; ++m) {
            const bool act = a && e > thr[m];
            cnt[m] += (uint32_t)__popcll(__ballot(act));
            ae[m] += act ? e : 0.0;
        }
    }
#pragma unroll
    for (int m = 0; m < TRIAL_M; ++m) rows[wave][m][lane] = ae[m];
    __syncthreads();
    if (lane < TRIAL_M) {
        double t = 0.0;
        for (int l = 0; l < 64; ++l) t += rows[wave][lane][l];
        wsum[wave][TRIAL_M + lane] = t;
        wsum[wave][lane] = (double)cnt[0];
#pragma unroll
        for (int m = 1; m < TRIAL_M; ++m)
            if (lane == m) wsum[wave][lane] = (double)cnt[m];
    }
    __syncthreads();
    if (threadIdx.x < 2 * TRIAL_M) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += wsum[q][threadIdx.x];
        blk_part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// Adds the block sums of one pass in a fixed order and walks the tree.
__global__ void __launch_bounds__(SCAN_THREADS)
k_trial_walk(int nblk, const double *__restrict__ blk_part,
             SearchState *__restrict__ S) {
    __shared__ double tot[2 * TRIAL_M];
    if (S->done) return;
    {
        // 16 threads per sum over a fixed stride of blocks (loads unrolled),
        // then a fixed shuffle tree over the 16
        const int v = threadIdx.x >> 4, g = threadIdx.x & 15;
        double t = 0.0;
        if (v < 2 * TRIAL_M) {
            const double *src = blk_part + (int64_t)v * nblk;
#pragma unroll 16
            for (int b = g; b < nblk; b += 16) t += src[b];
        }
        for (int off = 8; off >= 1; off >>= 1) t += __shfl_xor(t, off);
        if (v < 2 * TRIAL_M && g == 0) tot[v] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        SearchState st = *S;
        walk_tree(st, tot);
        *S = st;
    }
}

// ---------------------------------------------------------------------------
// FILTER + parent update + SPLIT: stable compaction of a segment of up to SEG
// regions by one block. The flags of all SEG / LIST_THREADS rounds are read
// first (region s0 + r * LIST_THREADS + tid in round r, coalesced), their
// wave ballots give the prefix in (round, wave) order after one barrier, and
// the survivors are then copied and bisected; the segment's base comes from
// the exclusive scan of the segment counts.
// ---------------------------------------------------------------------------
constexpr int CS_ROUNDS = SEG / LIST_THREADS;

__global__ void __launch_bounds__(LIST_THREADS)
k_compact_split(int d, int64_t n, int paired, double t,
                const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
                const double *__restrict__ V, const uint8_t *__restrict__ K,
                const double *__restrict__ lo, const double *__restrict__ w,
                int64_t ld_in, const uint32_t *__restrict__ offsets,
                int64_t na, double *__restrict__ lo_out,
                double *__restrict__ w_out, int64_t ld_out,
                double *__restrict__ Vp) {
    constexpr int NW = LIST_THREADS / 64;
    __shared__ uint32_t wcnt[CS_ROUNDS * NW];
    int64_t s0, s1;
    seg_range(blockIdx.x, n, paired, &s0, &s1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t act = 0, pre[CS_ROUNDS];
#pragma unroll
    for (int r = 0; r < CS_ROUNDS; ++r) {
        const int64_t i = s0 + r * LIST_THREADS + threadIdx.x;
        const bool a = i < s1 && A_rel[i] && (!E || E[i] > t);
        const uint64_t mask = __ballot(a);
        pre[r] = __popcll(mask & below);
        act |= (a ? 1u : 0u) << r;
        if (lane == 0) wcnt[r * NW + wave] = __popcll(mask);
    }
    __syncthreads();
    const int64_t base = offsets[blockIdx.x];
    uint32_t run = 0;                       // survivors before round r
#pragma unroll
    for (int r = 0; r < CS_ROUNDS; ++r) {
        uint32_t rbase = run;
        for (int q = 0; q < NW; ++q) {
            if (q < wave) rbase += wcnt[r * NW + q];
            run += wcnt[r * NW + q];
        }
        if (!((act >> r) & 1u)) continue;
        const int64_t i = s0 + r * LIST_THREADS + threadIdx.x;
        const int64_t j = base + rbase + pre[r];
        const int ax = K[i];
        for (int k = 0; k < d; ++k) {
            const double l = lo[k * ld_in + i], ww = w[k * ld_in + i];
            const double half = ww * 0.5;
            const bool sp = k == ax;
            lo_out[k * ld_out + j] = l;
            w_out[k * ld_out + j] = sp ? half : ww;
            lo_out[k * ld_out + j + na] = sp ? l + half : l;
            w_out[k * ld_out + j + na] = sp ? half : ww;
        }
        Vp[j] = V[i];
    }
}

__global__ void k_apply_threshold(int64_t n, double t,
                                  const uint8_t *__restrict__ A_rel,
                                  const double *__restrict__ E,
                                  uint8_t *__restrict__ A_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A_out[i] = (uint8_t)(A_rel[i] && E[i] > t);
}

// ---------------------------------------------------------------------------
// UNIFORM-SPLIT: g^d boxes, axis 0 varying fastest. Corners are a_k plus
// digit * width_k rounded twice, exactly as written (no contraction).
// ---------------------------------------------------------------------------
struct Box {
    double a[PG_DIM_MAX], width[PG_DIM_MAX];
};

__global__ void k_init(int d, int g, int64_t n, const Box B,
                       double *__restrict__ lo, double *__restrict__ w,
                       int64_t ld) {
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t q = r;
    for (int k = 0; k < d; ++k) {
        const int64_t digit = q % g;
        q /= g;
        const double off = (double)digit * B.width[k];
        lo[k * ld + r] = B.a[k] + off;
        w[k * ld + r] = B.width[k];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
typedef void (*EvalKernel)(const FParams, const Rule, int64_t, const double *,
                           const double *, int64_t, double *, double *,
                           uint8_t *);

template <int FAM>
static EvalKernel eval_table(int d) {
    switch (d) {
    case 2: return k_evaluate<FAM, 2>;
    case 3: return k_evaluate<FAM, 3>;
    case 4: return k_evaluate<FAM, 4>;
    case 5: return k_evaluate<FAM, 5>;
    case 6: return k_evaluate<FAM, 6>;
    case 7: return k_evaluate<FAM, 7>;
    case 8: return k_evaluate<FAM, 8>;
    case 9: return k_evaluate<FAM, 9>;
    case 10: return k_evaluate<FAM, 10>;
    default: return nullptr;
    }
}

static EvalKernel eval_kernel(int family, int d) {
    switch (family) {
    case PG_PRODUCT_PEAK: return eval_table<PG_PRODUCT_PEAK>(d);
    case PG_GAUSSIAN: return eval_table<PG_GAUSSIAN>(d);
    case PG_OSCILLATORY: return eval_table<PG_OSCILLATORY>(d);
    case PG_CORNER_PEAK: return eval_table<PG_CORNER_PEAK>(d);
    case PG_MONOMIAL: return eval_table<PG_MONOMIAL>(d);
    default: return nullptr;
    }
}

typedef void (*FvalKernel)(const FParams, int64_t, const double *, int64_t,
                           double *);

template <int FAM>
static FvalKernel fval_table(int d) {
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

hipError_t launch_fvalues(hipStream_t st, int family, int d, const FParams &P,
                          int64_t n, const double *x, int64_t ld, double *y) {
    FvalKernel k = nullptr;
    switch (family) {
    case PG_PRODUCT_PEAK: k = fval_table<PG_PRODUCT_PEAK>(d); break;
    case PG_GAUSSIAN: k = fval_table<PG_GAUSSIAN>(d); break;
    case PG_OSCILLATORY: k = fval_table<PG_OSCILLATORY>(d); break;
    case PG_CORNER_PEAK: k = fval_table<PG_CORNER_PEAK>(d); break;
    case PG_MONOMIAL: k = fval_table<PG_MONOMIAL>(d); break;
    default: break;
    }
    if (!k) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       P, n, x, ld, y);
    return hipGetLastError();
}

bool evaluate_supported(int family, int d) {
    return eval_kernel(family, d) != nullptr;
}

int evaluate_max_waves(int d) {
    const int units = d + d * (d - 1) / 2 + (1 << d) / 4;
    int w = 1;
    while (w * 2 <= EVAL_MAX_WAVES && w * 2 <= units) w *= 2;
    return w;
}

hipError_t launch_evaluate(hipStream_t st, int family, int d,
                           const FParams &P, const Rule &R, int64_t n,
                           const double *lo, const double *w, int64_t ld,
                           double *V, double *E, uint8_t *K, int waves) {
    EvalKernel k = eval_kernel(family, d);
    if (!k) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 63) / 64;
    const size_t lds = sizeof(double) * 64 * (size_t)(d + (waves > 1 ? 5 * waves : 0));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * waves), lds, st, P,
                       R, n, lo, w, ld, V, E, K);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t st, int d, int g, const double *a,
                       const double *width, double *lo, double *w,
                       int64_t ld) {
    Box B;
    int64_t n = 1;
    for (int k = 0; k < d; ++k) {
        B.a[k] = a[k];
        B.width[k] = width[k];
        n *= g;
    }
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, st, d, g,
                       n, B, lo, w, ld);
    return hipGetLastError();
}

hipError_t launch_classify(hipStream_t st, int64_t n, int paired,
                           const double *V, double *E, const double *Vp,
                           double tau, int relerr, uint8_t *A,
                           SegPartials part) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = paired ? seg_count(n, 1) / 2 : seg_count(n, 0);
    hipLaunchKernelGGL(k_classify, dim3((unsigned)blocks), dim3(LIST_THREADS),
                       0, st, n, paired, V, E, Vp, tau, relerr, A, part);
    return hipGetLastError();
}

hipError_t launch_seg_count(hipStream_t st, int64_t n, int paired, double t,
                            const double *V, const double *E,
                            const uint8_t *A_rel, const SearchState *S,
                            SegPartials part) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)seg_count(n, paired)),
                       dim3(LIST_THREADS), 0, st, n, paired, t, V, E, A_rel, S,
                       part);
    return hipGetLastError();
}

hipError_t launch_reduce_scan(hipStream_t st, int64_t nseg, SegPartials part,
                              uint32_t *offsets, Totals *tot) {
    hipLaunchKernelGGL(k_reduce_scan, dim3(1), dim3(SCAN_THREADS), 0, st, nseg,
                       part, offsets, tot);
    return hipGetLastError();
}

hipError_t launch_search_init(hipStream_t st, SearchState *S, int64_t n,
                              double e_it, double allowance, int mem,
                              const Totals *minmax) {
    hipLaunchKernelGGL(k_search_init, dim3(1), dim3(64), 0, st, S, n, e_it,
                       allowance, mem, minmax);
    return hipGetLastError();
}

int trial_blocks(int64_t n) {
    int64_t blocks = (n + TRIAL_THREADS - 1) / TRIAL_THREADS;
    if (blocks > TRIAL_BLOCKS) blocks = TRIAL_BLOCKS;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

hipError_t launch_search_pass(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              double *blk_part) {
    const int blocks = trial_blocks(n);
    hipLaunchKernelGGL(k_trials, dim3((unsigned)blocks), dim3(TRIAL_THREADS), 0,
                       st, n, E, A_rel, S, blk_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trial_walk, dim3(1), dim3(SCAN_THREADS), 0, st,
                       blocks, blk_part, S);
    return hipGetLastError();
}

hipError_t launch_compact_split(hipStream_t st, int d, int64_t n, int paired,
                                double t, const uint8_t *A_rel,
                                const double *E, const double *V,
                                const uint8_t *K, const double *lo,
                                const double *w, int64_t ld_in,
                                const uint32_t *offsets, int64_t n_active,
                                double *lo_out, double *w_out, int64_t ld_out,
                                double *Vp) {
    if (n <= 0 || n_active <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_split, dim3((unsigned)seg_count(n, paired)),
                       dim3(LIST_THREADS), 0, st, d, n, paired, t, A_rel, E, V,
                       K, lo, w, ld_in, offsets, n_active, lo_out, w_out,
                       ld_out, Vp);
    return hipGetLastError();
}

hipError_t launch_apply_threshold(hipStream_t st, int64_t n, double t,
                                  const uint8_t *A_rel, const double *E,
                                  uint8_t *A_out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_threshold, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, st, n, t, A_rel, E, A_out);
    return hipGetLastError();
}

}  // namespace pg
