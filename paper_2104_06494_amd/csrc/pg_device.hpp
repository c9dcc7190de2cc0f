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
    double v, e, av, ae, fv, mn, mx;      // fv: V of the regions with a = 0
    uint32_t cnt;
    __device__ void init() {
        v = e = av = ae = fv = 0.0;
        mn = __builtin_huge_val();
        mx = -__builtin_huge_val();
        cnt = 0;
    }
    __device__ void add(double V, double E, int a) {
        v += V;
        e += E;
        if (a) { av += V; ae += E; ++cnt; } else { fv += V; }
        mn = fmin(mn, E);
        mx = fmax(mx, E);
    }
    __device__ void merge(const Acc &o) {
        v += o.v; e += o.e; av += o.av; ae += o.ae; fv += o.fv;
        mn = fmin(mn, o.mn); mx = fmax(mx, o.mx);
        cnt += o.cnt;
    }
    __device__ void shfl_merge(int off) {
        Acc o;
        o.v = __shfl_xor(v, off);
        o.e = __shfl_xor(e, off);
        o.av = __shfl_xor(av, off);
        o.ae = __shfl_xor(ae, off);
        o.fv = __shfl_xor(fv, off);
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
        part.fv[s] = t.fv;
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
    // in chunks of SEG pairs (a segment is one chunk), PER per thread: every
    // load of a chunk is issued before the first use; the sums keep the
    // order of a plain strided loop
    constexpr int PER = SEG / LIST_THREADS;
    for (int64_t c0 = q0; c0 < q1; c0 += SEG) {
        double va[PER], vb[PER], ea[PER], eb[PER], vp[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t q = c0 + threadIdx.x + (int64_t)k * LIST_THREADS;
            if (q < q1) {
                va[k] = V[a0 + q];
                vb[k] = V[b0 + q];
                ea[k] = E[a0 + q];
                eb[k] = E[b0 + q];
                vp[k] = Vp[p0 + q];
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t q = c0 + threadIdx.x + (int64_t)k * LIST_THREADS;
            if (q >= q1) break;
            const int64_t ia = a0 + q, ib = b0 + q;
            const double delta = fabs(va[k] + vb[k] - vp[k]) / 4.0;
            const double S = ea[k] + eb[k];
            double xa = ea[k], xb = eb[k];
            if (S > 0.0) {
                const double g = 1.0 + 2.0 * delta / S;
                xa = xa * g + delta;
                xb = xb * g + delta;
            } else {
                xa = xa + delta;
                xb = xb + delta;
            }
            E[ia] = xa;
            E[ib] = xb;
            const int aa = relerr ? (xa > tau * fabs(va[k])) : 1;
            const int ab = relerr ? (xb > tau * fabs(vb[k])) : 1;
            A[ia] = (uint8_t)aa;
            A[ib] = (uint8_t)ab;
            lo_acc.add(va[k], xa, aa);
            hi_acc.add(vb[k], xb, ab);
        }
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
    // chunks of SEG regions, every load of a chunk issued before its first
    // use (the sums keep the order of a plain strided loop)
    constexpr int PER = SEG / LIST_THREADS;
    for (int64_t c0 = s0; c0 < s1; c0 += SEG) {
        double v[PER], e[PER];
        uint8_t ar[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = c0 + threadIdx.x + (int64_t)k * LIST_THREADS;
            if (i < s1) {
                v[k] = V[i];
                e[k] = E ? E[i] : 0.0;
                ar[k] = mode == 0 ? 0 : A_rel[i];
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = c0 + threadIdx.x + (int64_t)k * LIST_THREADS;
            if (i >= s1) break;
            const int a = mode == 0 ? 0 : (ar[k] && (mode == 1 || e[k] > t));
            acc.add(v[k], e[k], a);
        }
    }
    block_reduce_store(acc, part, s);
}

// ---------------------------------------------------------------------------
// Totals of the segment partials [seg0, seg0 + nseg) and the exclusive scan
// of their counts (one block of NT threads).
// ---------------------------------------------------------------------------
template <int NT = REDUCE_THREADS>
__device__ inline Totals reduce_scan_segments(int64_t seg0, int64_t nseg,
                                              SegPartials part,
                                              uint32_t *__restrict__ offsets,
                                              Totals *__restrict__ tot) {
    __shared__ uint64_t wsum[NT / 64];
    __shared__ Acc wacc[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (nseg + NT - 1) / NT;
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
        a.fv += part.fv[s];
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
    Totals r{};
    if (tid == 0) {
        Acc t = wacc[0];
        for (int q = 1; q < NT / 64; ++q) t.merge(wacc[q]);
        uint64_t total = 0;
        for (int q = 0; q < NT / 64; ++q) total += wsum[q];
        r.v = t.v;
        r.e = t.e;
        r.av = t.av;
        r.ae = t.ae;
        r.emin = t.mn;
        r.emax = t.mx;
        r.cnt = (double)total;
        r.fv = t.fv;
        *tot = r;
    }
    return r;          // the totals (thread 0 only)
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

// One trial of Algorithm 3 at threshold tt, given whether the memory and the
// accuracy requirements hold there: accept, or move t (raise it when memory
// fails, lower it when accuracy fails), counting direction changes. With
// st.relax set, P_max grows by 0.10 at each direction change, up to 0.95
// (Section 3.5.3); the host sets it for every search, or (the memory-only
// option) only for searches run because the list would overflow its cap.
// Returns 1 when the search has ended. The caller checks the trial limit
// first.
__device__ inline int search_step(SearchState &st, double tt, bool mem_ok,
                                  bool acc_ok) {
    ++st.trials;
    int dir;
    if (mem_ok) {
        if (acc_ok) {
            st.done = 1;
            st.ok = 1;
            st.t_acc = tt;
            return 1;
        }
        dir = -1;                               // accuracy failed: lower t
    } else {
        dir = +1;                               // memory failed: raise t
    }
    if (st.last_dir != 0 && dir != st.last_dir) {
        ++st.dir_changes;
        if (st.relax) st.P_max = fmin(st.P_max + 0.10, 0.95);
        if (st.dir_changes >= THR_MAX_DIRCHG) { st.done = 1; return 1; }
    }
    st.last_dir = dir;
    st.t = dir > 0 ? tt + (st.mx - tt) / 2.0 : tt - (tt - st.mn) / 2.0;
    return 0;
}

// Walks up to TRIAL_DEPTH levels of the tree given the totals of a pass:
// tot[m] regions stay active under node m's threshold and tot[TRIAL_M + m]
// is the error of the regions it finishes (e_abar of Algorithm 3).
__device__ inline void walk_tree(SearchState &st, const double *tot) {
    double thr[TRIAL_M];
    build_tree(st, thr);
    int node = 0;
    for (int level = 0; level < TRIAL_DEPTH; ++level) {
        if (st.trials >= THR_MAX_TRIALS) { st.done = 1; return; }
        const double tt = thr[node];
        const double s_abar = (double)st.n - tot[node];
        const double e_abar = tot[TRIAL_M + node];
        const bool mem_ok = s_abar > 0.5 * (double)st.n;
        const bool acc_ok = e_abar <= st.P_max * st.allowance;
        if (search_step(st, tt, mem_ok, acc_ok)) return;
        node = st.last_dir > 0 ? 2 * node + 1 : 2 * node + 2;
    }
}

// ---------------------------------------------------------------------------
// Error histogram of the regions a threshold search works on (A_rel), so
// that most trials are decided without a pass over the list. A bin is
// 2^-HIST_MBITS of a binade: the key of E is its binary64 pattern shifted
// right by HIST_SHIFT (exponent and HIST_MBITS significand bits), and bin j
// holds key kmax - j, kmax the key of the largest E; everything further
// down falls into the last bin. Counts are exact; a bin's sum is the exact
// integer sum of its values' significands with HIST_DROP low bits dropped
// (one scale per bin), so the sums are deterministic and the bounds drawn
// from them are rigorous.
// ---------------------------------------------------------------------------
constexpr int HIST_MBITS = 5;
constexpr int HIST_SHIFT = 52 - HIST_MBITS;
constexpr int HIST_DROP = 21;                  // 32 of 53 significand bits kept
constexpr int HIST_THREADS = 1024;
constexpr int HIST_UNROLL = 8;        // regions a thread loads at once

__device__ inline uint64_t hist_key(double e) {
    return __builtin_bit_cast(uint64_t, e) >> HIST_SHIFT;
}

// Regions (at most) one histogram block adds up: whole segments, as many
// as the packed LDS word allows, so that a long list needs few blocks and
// few global atomics.
constexpr int64_t HIST_RANGE = 8192;
static_assert(HIST_RANGE % SEG == 0 && HIST_RANGE >= BSEG &&
                  HIST_RANGE <= (1 << 13),
              "histogram block range");

// Adds the A_rel regions of [s0, s1) (at most HIST_RANGE of them) to the
// histogram: in LDS one 64-bit atomic per region, holding the count in bits
// 50 and up and the significand sum below (the sum of at most 2^13 32-bit
// significands stays under 2^45, the count under 2^14), then one pair of
// global atomics per non-empty bin.
__device__ inline void hist_segment(int64_t s0, int64_t s1,
                                    const double *__restrict__ E,
                                    const uint8_t *__restrict__ A_rel,
                                    uint64_t kmax, uint32_t *__restrict__ gcnt,
                                    unsigned long long *__restrict__ gsum) {
    constexpr unsigned long long ONE = 1ull << 50;
    __shared__ unsigned long long lcs[HIST_BINS];
    for (int b = threadIdx.x; b < HIST_BINS; b += blockDim.x) lcs[b] = 0;
    __syncthreads();
    // HIST_UNROLL regions a thread at a time, all their loads (flags and
    // errors alike: the errors' cache lines are fetched anyway) issued
    // before the first atomic; the integer sums do not depend on the order
    const int64_t stride = blockDim.x;
    for (int64_t c0 = s0 + threadIdx.x; c0 < s1; c0 += HIST_UNROLL * stride) {
        uint8_t a[HIST_UNROLL];
        uint64_t bits[HIST_UNROLL];
#pragma unroll
        for (int k = 0; k < HIST_UNROLL; ++k) {
            const int64_t i = c0 + k * stride;
            a[k] = i < s1 ? A_rel[i] : 0;
            bits[k] = i < s1 ? __builtin_bit_cast(uint64_t, E[i]) : 0;
        }
#pragma unroll
        for (int k = 0; k < HIST_UNROLL; ++k) {
            if (!a[k]) continue;
            const uint64_t key = bits[k] >> HIST_SHIFT;
            uint64_t j = key >= kmax ? 0 : kmax - key;
            if (j > HIST_BINS - 1) j = HIST_BINS - 1;
            unsigned long long add = ONE;
            if (j < HIST_BINS - 1) {
                const uint64_t ef = (bits[k] >> 52) & 0x7ff;
                uint64_t m = bits[k] & ((1ull << 52) - 1);
                if (ef) m |= 1ull << 52;
                add += (unsigned long long)(m >> HIST_DROP);
            }
            atomicAdd(&lcs[j], add);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < HIST_BINS; b += blockDim.x) {
        const unsigned long long v = lcs[b];
        if (v) {
            atomicAdd(&gcnt[b], (uint32_t)(v >> 50));
            atomicAdd(&gsum[b], v & (ONE - 1));
        }
    }
}

// Decides trials from a histogram's bound tables while it can (one
// thread): for the bin j holding t, regions in bins above j have E > t and
// those below have E < t, so the count and error sum of the regions kept
// active lie in intervals (plo[j] and phi[j + 1], the sums already widened
// by a relative margin of 1e-12, far wider than the rounding of the exact
// pass's sums); a trial is decided when both requirements come out the same
// at both ends. Stops at the first undecided trial (left to an exact pass)
// or when the search ends. The tables may be in LDS or global memory.
__device__ inline void bounds_walk(SearchState &st,
                                   const double2 *__restrict__ plo,
                                   const double2 *__restrict__ phi) {
    const uint64_t kmax = hist_key(st.mx);
    const double n = (double)st.n;
    while (!st.done) {
        if (st.trials >= THR_MAX_TRIALS) { st.done = 1; break; }
        const double t = st.t;
        const uint64_t kt = hist_key(t);
        double c_lo, c_hi, s_lo, s_hi;
        if (kt > kmax) {                       // above every error
            c_lo = c_hi = 0.0;
            s_lo = s_hi = 0.0;
        } else {
            uint64_t j = kmax - kt;
            if (j > HIST_BINS - 1) j = HIST_BINS - 1;
            const double2 lo2 = plo[j], hi2 = phi[j + 1];
            c_lo = lo2.x;
            c_hi = hi2.x;
            s_lo = lo2.y;
            s_hi = hi2.y;
        }
        bool mem_ok, acc_ok = false;
        if (n - c_hi > 0.5 * n) mem_ok = true;
        else if (!(n - c_lo > 0.5 * n)) mem_ok = false;
        else break;                            // undecided
        if (mem_ok) {
            const double lim = st.P_max * st.allowance;
            const double slack = 1e-12 * (fabs(st.e_it) + fabs(lim));
            if (st.e_it - s_lo <= lim - slack) acc_ok = true;
            else if (st.e_it - s_hi > lim + slack) acc_ok = false;
            else break;                        // undecided
        }
        search_step(st, t, mem_ok, acc_ok);
    }
}

// Builds the bound tables of a histogram (HIST_THREADS threads), decides
// as many trials as they allow (bounds_walk) and leaves the state in *gst.
// The search starts from `init`. The tables are also stored in tlo / thi
// (HIST_TAB entries each), so that the trials following each exact pass
// can be decided from them as well. Clears the histogram for the next
// search.
__device__ inline void hist_walk(const SearchState &init,
                                 SearchState *__restrict__ gst,
                                 uint32_t *__restrict__ gcnt,
                                 unsigned long long *__restrict__ gsum,
                                 double2 *__restrict__ tlo,
                                 double2 *__restrict__ thi) {
    // bin j's bounds for a trial: {count above, lower error sum above} and
    // {count above, upper error sum above}, the sums already widened by the
    // margin, so a trial reads two 16-byte words
    __shared__ double2 plo[HIST_BINS + 1], phi[HIST_BINS + 1];
    __shared__ double csum[HIST_THREADS / 64 + 1][3];
    constexpr int PER = HIST_BINS / HIST_THREADS;
    const uint64_t kmax = hist_key(init.mx);
    double c[PER], l[PER], u[PER];
    const int b0 = threadIdx.x * PER;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = b0 + q;
        const uint32_t cnt = gcnt[j];
        const unsigned long long sm = gsum[j];
        gcnt[j] = 0;
        gsum[j] = 0;
        c[q] = (double)cnt;
        if (j < HIST_BINS - 1) {
            // all values of bin j share the exponent field of key kmax - j
            const int64_t key = (int64_t)kmax - j;
            int64_t ef = key >> HIST_MBITS;
            if (ef < 1) ef = 1;
            const double scale = ldexp(1.0, (int)(ef - 1075 + HIST_DROP));
            l[q] = key < 0 ? 0.0 : (double)sm * scale;
            u[q] = key < 0 ? 0.0 : ((double)sm + (double)cnt) * scale;
        } else {
            // below the lower edge of bin HIST_BINS - 2
            const int64_t key = (int64_t)kmax - (HIST_BINS - 2);
            const double edge = key <= 0 ? 0.0
                : __builtin_bit_cast(double, (uint64_t)key << HIST_SHIFT);
            l[q] = 0.0;
            u[q] = (double)cnt * edge;
        }
    }
    // exclusive prefix sums from the top bin: chunk totals, a shuffle scan
    // within each wave, the wave totals in order (fixed order throughout)
    double tot[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < PER; ++q) { tot[0] += c[q]; tot[1] += l[q]; tot[2] += u[q]; }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double ex[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double x = tot[a];
        for (int o = 1; o < 64; o <<= 1) {
            const double y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        const double before = __shfl_up(x, 1);
        ex[a] = lane ? before : 0.0;
        if (lane == 63) csum[wave][a] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double acc = 0.0;
        for (int w = 0; w < HIST_THREADS / 64; ++w) {
            const double x = csum[w][threadIdx.x];
            csum[w][threadIdx.x] = acc;
            acc += x;
        }
        csum[HIST_THREADS / 64][threadIdx.x] = acc;
    }
    __syncthreads();
    {
        double a = csum[wave][0] + ex[0], b = csum[wave][1] + ex[1],
               d = csum[wave][2] + ex[2];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const double2 lo2 = make_double2(a, b * (1.0 - 1e-12));
            const double2 hi2 = make_double2(a, d * (1.0 + 1e-12));
            plo[b0 + q] = lo2;
            phi[b0 + q] = hi2;
            tlo[b0 + q] = lo2;
            thi[b0 + q] = hi2;
            a += c[q];
            b += l[q];
            d += u[q];
        }
        if (threadIdx.x == HIST_THREADS - 1) {
            const double2 lo2 = make_double2(a, b * (1.0 - 1e-12));
            const double2 hi2 = make_double2(a, d * (1.0 + 1e-12));
            plo[HIST_BINS] = lo2;
            phi[HIST_BINS] = hi2;
            tlo[HIST_BINS] = lo2;
            thi[HIST_BINS] = hi2;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    SearchState st = init;
    st.table = 1;
    bounds_walk(st, plo, phi);
    *gst = st;
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
// FILTER + parent update + SPLIT of one segment [s0, s1) of at most SEGLEN
// regions by one block of NT threads: the flags of all SEGLEN / NT rounds
// are read first (region s0 + r * NT + tid in round r, coalesced), their
// wave ballots give the prefix in (round, wave) order after one barrier,
// and the survivors are then copied and bisected: the survivor at output
// index j = base + prefix goes to j (lower half) and j + na (upper half),
// with Vp[j - vp_shift] = V. With a non-null inst_out, the children are
// tagged with `tag`. DC > 0 fixes the dimension at compile time (d is then
// ignored), so a box takes exactly DC registers per coordinate array.
// ---------------------------------------------------------------------------
template <int SEGLEN, int NT = LIST_THREADS, int DC = 0>
__device__ inline void compact_segment(
    int d, int64_t s0, int64_t s1, int mode, double t,
    const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
    const double *__restrict__ V, const uint8_t *__restrict__ K,
    const double *__restrict__ lo, const double *__restrict__ w,
    int64_t ld_in, int64_t base, int64_t na, double *__restrict__ lo_out,
    double *__restrict__ w_out, int64_t ld_out, double *__restrict__ Vp,
    int64_t vp_shift, uint32_t *__restrict__ inst_out, uint32_t tag) {
    constexpr int CS_ROUNDS = SEGLEN / NT;
    constexpr int DA = DC > 0 ? DC : PG_DIM_MAX;   // coordinate registers
    if constexpr (DC > 0) d = DC;
    static_assert(CS_ROUNDS % 2 == 0, "compaction pairs rounds");
    constexpr int NW = NT / 64;
    __shared__ uint32_t wcnt[CS_ROUNDS * NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t act = 0, pre[CS_ROUNDS];
#pragma unroll
    for (int r = 0; r < CS_ROUNDS; ++r) {
        const int64_t i = s0 + r * NT + threadIdx.x;
        const bool a = i < s1 && mode != 0 && A_rel[i] &&
                       (mode == 1 || E[i] > t);
        const uint64_t mask = __ballot(a);
        pre[r] = __popcll(mask & below);
        act |= (a ? 1u : 0u) << r;
        if (lane == 0) wcnt[r * NW + wave] = __popcll(mask);
    }
    __syncthreads();
    // destinations of the thread's survivors, round by round
    int64_t dst[CS_ROUNDS];
    {
        uint32_t run = 0;                   // survivors before round r
#pragma unroll
        for (int r = 0; r < CS_ROUNDS; ++r) {
            uint32_t rbase = run;
            for (int q = 0; q < NW; ++q) {
                if (q < wave) rbase += wcnt[r * NW + q];
                run += wcnt[r * NW + q];
            }
            dst[r] = base + rbase + pre[r];
        }
    }
    // two rounds at a time: both rounds' boxes are loaded before either is
    // written, so a thread has two rounds of loads in flight
#pragma unroll
    for (int r0 = 0; r0 < CS_ROUNDS; r0 += 2) {
        double l[2][DA], ww[2][DA], v[2];
        int ax[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!((act >> (r0 + h)) & 1u)) continue;
            const int64_t i = s0 + (r0 + h) * NT + threadIdx.x;
            ax[h] = K[i];
            v[h] = V[i];
#pragma unroll
            for (int k = 0; k < DA; ++k) {
                if (k < d) {
                    l[h][k] = lo[k * ld_in + i];
                    ww[h][k] = w[k * ld_in + i];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!((act >> (r0 + h)) & 1u)) continue;
            const int64_t j = dst[r0 + h];
#pragma unroll
            for (int k = 0; k < DA; ++k) {
                if (k < d) {
                    const double half = ww[h][k] * 0.5;
                    const bool sp = k == ax[h];
                    lo_out[k * ld_out + j] = l[h][k];
                    w_out[k * ld_out + j] = sp ? half : ww[h][k];
                    lo_out[k * ld_out + j + na] = sp ? l[h][k] + half : l[h][k];
                    w_out[k * ld_out + j + na] = sp ? half : ww[h][k];
                }
            }
            Vp[j - vp_shift] = v[h];
            if (inst_out) {
                inst_out[j] = tag;
                inst_out[j + na] = tag;
            }
        }
    }
}

}  // namespace pg
