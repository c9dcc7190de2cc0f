// pg_device.hpp -- device-side building blocks of the list kernels, shared by
// the single-integral kernels (pg_list.hip) and the many-integral kernels
// (pg_batch.hip) so that an integral sees the same arithmetic, in the same
// order, whichever driver runs it.
#pragma once

#include <hip/hip_runtime.h>

#include "pg_internal.hpp"

namespace pg {

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
__device__ inline void block_reduce_store(Acc a, SegPartials part, int64_t s) {
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
// TWO-LEVEL-ERROR + REL-ERR-CLASSIFY of one segment (LIST_THREADS threads).
// Paired: pairs q in [q0, q1) are regions a0 + q and b0 + q, children of the
// parent whose estimate is Vp[p0 + q]; partials go to slots s_lo and s_hi.
// Unpaired: regions [q0, q1), partials to slot s_lo.
// ---------------------------------------------------------------------------
__device__ inline void classify_segment(int paired, int64_t q0, int64_t q1,
                                        int64_t a0, int64_t b0, int64_t p0,
                                        const double *__restrict__ V,
                                        double *__restrict__ E,
                                        const double *__restrict__ Vp,
                                        double tau, int relerr,
                                        uint8_t *__restrict__ A,
                                        SegPartials part, int64_t s_lo,
                                        int64_t s_hi) {
    Acc lo_acc, hi_acc;
    lo_acc.init();
    hi_acc.init();
    if (!paired) {
        for (int64_t i = q0 + threadIdx.x; i < q1; i += LIST_THREADS) {
            const double v = V[i], e = E[i];
            const int a = relerr ? (e > tau * fabs(v)) : 1;
            A[i] = (uint8_t)a;
            lo_acc.add(v, e, a);
        }
        block_reduce_store(lo_acc, part, s_lo);
        return;
    }
    for (int64_t q = q0 + threadIdx.x; q < q1; q += LIST_THREADS) {
        const int64_t ia = a0 + q, ib = b0 + q;
        const double va = V[ia], vb = V[ib];
        double ea = E[ia], eb = E[ib];
        const double delta = fabs(va + vb - Vp[p0 + q]) / 4.0;
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
    block_reduce_store(lo_acc, part, s_lo);
    block_reduce_store(hi_acc, part, s_hi);
}

// Count and sums of one segment [s0, s1) of A = A_rel AND (E > t) (every
// region active-tested with `mode`: 0 none active, 1 A_rel, 2 A_rel and
// E > t); partials to slot s.
__device__ inline void count_segment(int64_t s0, int64_t s1, int mode,
                                     double t, const double *__restrict__ V,
                                     const double *__restrict__ E,
                                     const uint8_t *__restrict__ A_rel,
                                     SegPartials part, int64_t s) {
    Acc acc;
    acc.init();
    for (int64_t i = s0 + threadIdx.x; i < s1; i += LIST_THREADS) {
        const double v = V[i], e = E ? E[i] : 0.0;
        const int a = mode == 0 ? 0 : (A_rel[i] && (mode == 1 || e > t));
        acc.add(v, e, a);
    }
    block_reduce_store(acc, part, s);
}

// ---------------------------------------------------------------------------
// Totals of the segment partials [seg0, seg0 + nseg) and the exclusive scan
// of their counts (one block of SCAN_THREADS threads).
// ---------------------------------------------------------------------------
__device__ inline void reduce_scan_segments(int64_t seg0, int64_t nseg,
                                            SegPartials part,
                                            uint32_t *__restrict__ offsets,
                                            Totals *__restrict__ tot) {
    __shared__ uint64_t wsum[SCAN_THREADS / 64];
    __shared__ Acc wacc[SCAN_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (nseg + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t s0 = seg0 + tid * per;
    const int64_t s1 = s0 + per < seg0 + nseg ? s0 + per : seg0 + nseg;
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

// Walks up to TRIAL_DEPTH levels of the tree given the totals of a pass:
// tot[m] regions stay active under node m's threshold and tot[TRIAL_M + m]
// is the sum of their errors.
__device__ inline void walk_tree(SearchState &st, const double *tot) {
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

// Fixed-order sum of the 2 TRIAL_M block sums of a pass, blocks strided by
// `stride` starting at src (16 threads per sum, then a shuffle tree of 16).
// Needs >= 32 * TRIAL_M threads; tot[] in shared memory.
__device__ inline void sum_trial_parts(const double *__restrict__ src,
                                       int64_t nblk, int64_t stride,
                                       double *tot) {
    const int v = threadIdx.x >> 4, g = threadIdx.x & 15;
    double t = 0.0;
    if (v < 2 * TRIAL_M) {
        const double *p = src + (int64_t)v * stride;
#pragma unroll 16
        for (int64_t b = g; b < nblk; b += 16) t += p[b];
    }
    for (int off = 8; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if (v < 2 * TRIAL_M && g == 0) tot[v] = t;
}

// ---------------------------------------------------------------------------
// FILTER + parent update + SPLIT of one segment [s0, s1) by one block: the
// flags of all SEG / LIST_THREADS rounds are read first (region
// s0 + r * LIST_THREADS + tid in round r, coalesced), their wave ballots give
// the prefix in (round, wave) order after one barrier, and the survivors are
// then copied and bisected: the survivor at output index j = base + prefix
// goes to j (lower half) and j + na (upper half), with Vp[j - vp_shift] = V.
// With a non-null inst_out, the children are tagged with `tag`.
// ---------------------------------------------------------------------------
constexpr int CS_ROUNDS = SEG / LIST_THREADS;

__device__ inline void compact_segment(
    int d, int64_t s0, int64_t s1, int mode, double t,
    const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
    const double *__restrict__ V, const uint8_t *__restrict__ K,
    const double *__restrict__ lo, const double *__restrict__ w,
    int64_t ld_in, int64_t base, int64_t na, double *__restrict__ lo_out,
    double *__restrict__ w_out, int64_t ld_out, double *__restrict__ Vp,
    int64_t vp_shift, uint32_t *__restrict__ inst_out, uint32_t tag) {
    constexpr int NW = LIST_THREADS / 64;
    __shared__ uint32_t wcnt[CS_ROUNDS * NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t act = 0, pre[CS_ROUNDS];
#pragma unroll
    for (int r = 0; r < CS_ROUNDS; ++r) {
        const int64_t i = s0 + r * LIST_THREADS + threadIdx.x;
        const bool a = i < s1 && mode != 0 && A_rel[i] &&
                       (mode == 1 || E[i] > t);
        const uint64_t mask = __ballot(a);
        pre[r] = __popcll(mask & below);
        act |= (a ? 1u : 0u) << r;
        if (lane == 0) wcnt[r * NW + wave] = __popcll(mask);
    }
    __syncthreads();
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
        Vp[j - vp_shift] = V[i];
        if (inst_out) {
            inst_out[j] = tag;
            inst_out[j + na] = tag;
        }
    }
}

}  // namespace pg
