// pg_batch.hip -- gfx950 list kernels for many integrals in one list.
//
// Every integral (slot) of a batched run keeps its regions contiguous, so a
// batched kernel is the single-integral kernel applied to each slot's
// segments with the slot's offsets and parameters; the per-segment
// arithmetic is the same code (pg_device.hpp). One block per segment, one
// block per slot for the reductions and the threshold walks.
#include "pg_device.hpp"

#include <hip/hip_runtime.h>

namespace pg {

// Expands the segment table and the classify items of every live slot: one
// block per slot (slots in list order), its threads striding over the
// slot's segments.
__global__ void __launch_bounds__(256)
k_batch_tables(const int32_t *__restrict__ order,
               const BInst *__restrict__ inst, BSeg *__restrict__ segs,
               BCls *__restrict__ cls) {
    const uint32_t slot = (uint32_t)order[blockIdx.x];
    const BInst I = inst[slot];
    if (!I.paired) {
        for (int64_t j = threadIdx.x; j < I.nseg; j += blockDim.x) {
            const int64_t s0 = I.start + j * BSEG;
            const int64_t s1 = s0 + BSEG < I.start + I.n ? s0 + BSEG : I.start + I.n;
            segs[I.seg0 + j] = BSeg{s0, s1, slot, 0};
            cls[I.cls0 + j] = BCls{s0, s1, I.seg0 + j, -1, slot, 0};
        }
        return;
    }
    const int64_t half = I.n / 2;
    const int64_t nh = (half + BSEG - 1) / BSEG;
    for (int64_t j = threadIdx.x; j < nh; j += blockDim.x) {
        const int64_t q0 = j * BSEG, q1 = q0 + BSEG < half ? q0 + BSEG : half;
        segs[I.seg0 + j] = BSeg{I.start + q0, I.start + q1, slot, 0};
        segs[I.seg0 + nh + j] = BSeg{I.start + half + q0, I.start + half + q1,
                                     slot, 1};
        cls[I.cls0 + j] = BCls{q0, q1, I.seg0 + j, I.seg0 + nh + j, slot, 0};
    }
}

// TWO-LEVEL-ERROR + REL-ERR-CLASSIFY + per-segment sums, one item per block.
__global__ void __launch_bounds__(LIST_THREADS)
k_batch_classify(const BCls *__restrict__ cls, const BInst *__restrict__ inst,
                 const double *__restrict__ V, double *__restrict__ E,
                 const double *__restrict__ Vp, uint8_t *__restrict__ A,
                 SegPartials part) {
    const BCls c = cls[blockIdx.x];
    const BInst &I = inst[c.slot];
    const int64_t half = I.n / 2;
    classify_segment(I.paired, c.q0, c.q1, I.start, I.start + half,
                     I.start / 2, V, E, Vp, I.tau, I.relerr, A, part, c.s_lo,
                     c.s_hi);
}

// Per-slot totals of its segment partials and the exclusive scan of their
// counts (offsets within the slot), one block per slot.
__global__ void __launch_bounds__(REDUCE_THREADS)
k_batch_reduce(const int32_t *__restrict__ order,
               const BInst *__restrict__ inst, SegPartials part,
               uint32_t *__restrict__ offsets, Totals *__restrict__ tot,
               Totals *__restrict__ host_tot) {
    const int slot = order[blockIdx.x];
    const BInst &I = inst[slot];
    const Totals t = reduce_scan_segments(I.seg0, I.nseg, part, offsets, tot + slot);
    // the host's copy (mapped pinned host memory), when given
    if (host_tot && threadIdx.x == 0) host_tot[slot] = t;
}

// Threshold trials of every searching slot: block per segment, the sums of
// the slot's TRIAL_M candidate thresholds over the segment.
__global__ void __launch_bounds__(LIST_THREADS)
k_batch_trials(const BSeg *__restrict__ segs, int64_t nseg,
               const BInst *__restrict__ inst, const double *__restrict__ E,
               const uint8_t *__restrict__ A_rel,
               const SearchState *__restrict__ states,
               double *__restrict__ tpart) {
    constexpr int NW = LIST_THREADS / 64;
    __shared__ double rows[NW][TRIAL_M][65];    // padded: no bank conflicts
    __shared__ double wsum[NW][2 * TRIAL_M];
    const BSeg sg = segs[blockIdx.x];
    if (!inst[sg.slot].searching || states[sg.slot].done) return;
    double thr[TRIAL_M];
    build_tree(states[sg.slot], thr);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t cnt[TRIAL_M];
    double fe[TRIAL_M];
#pragma unroll
    for (int m = 0; m < TRIAL_M; ++m) { cnt[m] = 0; fe[m] = 0.0; }
    for (int64_t i0 = sg.start + wave * 64; i0 < sg.end; i0 += LIST_THREADS) {
        const int64_t i = i0 + lane;
        const bool valid = i < sg.end;
        const double e = valid ? E[i] : 0.0;
        const bool a = valid && A_rel[i] != 0;
#pragma unroll
        for (int m = 0; m < TRIAL_M; ++m) {
            const bool act = a && e > thr[m];
            cnt[m] += (uint32_t)__popcll(__ballot(act));
            // the finished regions' error, summed directly (exactly 0
            // when every region this threshold finishes carries none)
            fe[m] += act ? 0.0 : e;
        }
    }
#pragma unroll
    for (int m = 0; m < TRIAL_M; ++m) rows[wave][m][lane] = fe[m];
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
        tpart[(int64_t)threadIdx.x * nseg + blockIdx.x] = t;
    }
}

// Error histograms of every searching slot (block per segment), then the
// trials they decide (block per slot).
// Segment-table entries one histogram block takes (see k_batch_hist).
constexpr int BHIST_SEGS = HIST_RANGE / BSEG;
static_assert(BHIST_SEGS >= 1, "histogram block range");

__global__ void __launch_bounds__(LIST_THREADS)
k_batch_hist(const BSeg *__restrict__ segs, int64_t nseg,
             const BInst *__restrict__ inst,
             const SearchState *__restrict__ states,
             const double *__restrict__ E, const uint8_t *__restrict__ A_rel,
             uint32_t *__restrict__ cnt, unsigned long long *__restrict__ sum) {
    // BHIST_SEGS consecutive table entries a block; a slot's entries cover
    // consecutive regions (lower halves, then upper halves), so each run of
    // one slot is one range of at most HIST_RANGE regions, and a slot's
    // histogram receives a quarter of the flushes it would with a block
    // per segment
    const int64_t a0 = (int64_t)blockIdx.x * BHIST_SEGS;
    const int64_t a1 = a0 + BHIST_SEGS < nseg ? a0 + BHIST_SEGS : nseg;
    for (int64_t a = a0; a < a1;) {
        const uint32_t slot = segs[a].slot;
        int64_t b = a + 1;
        while (b < a1 && segs[b].slot == slot) ++b;
        if (inst[slot].searching && !states[slot].done)
            hist_segment(segs[a].start, segs[b - 1].end, E, A_rel,
                         hist_key(states[slot].mx),
                         cnt + (size_t)slot * HIST_BINS,
                         sum + (size_t)slot * HIST_BINS);
        a = b;
    }
}

__global__ void __launch_bounds__(HIST_THREADS)
k_batch_hist_walk(const int32_t *__restrict__ order,
                  const BInst *__restrict__ inst,
                  SearchState *__restrict__ states, uint32_t *__restrict__ cnt,
                  unsigned long long *__restrict__ sum,
                  double2 *__restrict__ tlo, double2 *__restrict__ thi) {
    const int slot = order[blockIdx.x];
    if (!inst[slot].searching || states[slot].done) return;
    const SearchState init = states[slot];
    hist_walk(init, states + slot, cnt + (size_t)slot * HIST_BINS,
              sum + (size_t)slot * HIST_BINS, tlo + (size_t)slot * HIST_TAB,
              thi + (size_t)slot * HIST_TAB);
}

// Adds each searching slot's segment sums in a fixed order and walks its
// tree, then the trials after it that the slot's histogram bound tables
// decide; one block per slot.
__global__ void __launch_bounds__(SCAN_THREADS)
k_batch_walk(const int32_t *__restrict__ order, const BInst *__restrict__ inst,
             int64_t nseg, const double *__restrict__ tpart,
             SearchState *__restrict__ states, const double2 *__restrict__ tlo,
             const double2 *__restrict__ thi) {
    __shared__ double tot[2 * TRIAL_M];
    const int slot = order[blockIdx.x];
    const BInst &I = inst[slot];
    if (!I.searching || states[slot].done) return;
    sum_trial_parts(tpart + I.seg0, I.nseg, nseg, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        SearchState st = states[slot];
        walk_tree(st, tot);
        if (st.table)
            bounds_walk(st, tlo + (size_t)slot * HIST_TAB,
                        thi + (size_t)slot * HIST_TAB);
        states[slot] = st;
    }
}

__device__ inline int batch_mode(const BInst &I, const SearchState &S) {
    if (!I.live) return 0;
    return (I.searching && S.ok) ? 2 : 1;
}

// Count and sums of the survivors of every segment (A_rel, or A_rel and
// E > t_acc after a successful search; nothing for slots that end).
__global__ void __launch_bounds__(LIST_THREADS)
k_batch_count(const BSeg *__restrict__ segs, const BInst *__restrict__ inst,
              const SearchState *__restrict__ states,
              const double *__restrict__ V, const double *__restrict__ E,
              const uint8_t *__restrict__ A_rel, SegPartials part) {
    const BSeg sg = segs[blockIdx.x];
    const int mode = batch_mode(inst[sg.slot], states[sg.slot]);
    count_segment(sg.start, sg.end, mode, states[sg.slot].t_acc, V, E, A_rel,
                  part, blockIdx.x);
}

// FILTER + parent update + SPLIT of every segment into its slot's block of
// the next list. A slot whose next block starts at s keeps its parents'
// values at Vp[s / 2 + k] (k-th survivor), which is where the classify pass
// of the next iteration looks for them; blocks of 2 na regions give
// disjoint parent ranges whatever the parity of s.
// Twice the list kernels' threads, so that a BSEG-long segment takes four
// regions a thread (two load-then-store steps, as in the single list's
// compaction), and the dimension a template argument, so that a thread's
// two boxes take 4 D registers (two blocks a CU up to D = 6).
constexpr int BCOMPACT_THREADS = 2 * LIST_THREADS;

template <int D>
__global__ void __launch_bounds__(BCOMPACT_THREADS)
k_batch_compact(const BSeg *__restrict__ segs, const BInst *__restrict__ inst,
                const SearchState *__restrict__ states,
                const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
                const double *__restrict__ V, const uint8_t *__restrict__ K,
                const double *__restrict__ lo, const double *__restrict__ w,
                int64_t ld, const uint32_t *__restrict__ offsets,
                double *__restrict__ lo_out, double *__restrict__ w_out,
                double *__restrict__ Vp, uint32_t *__restrict__ inst_out) {
    const BSeg sg = segs[blockIdx.x];
    const BInst &I = inst[sg.slot];
    const int mode = batch_mode(I, states[sg.slot]);
    if (mode == 0) return;
    compact_segment<BSEG, BCOMPACT_THREADS, D>(
        D, sg.start, sg.end, mode, states[sg.slot].t_acc, A_rel, E, V, K, lo,
        w, ld, I.out_start + offsets[blockIdx.x], I.na, lo_out, w_out, ld, Vp,
        I.out_start - I.out_start / 2, inst_out, sg.slot);
}

struct BatchBox {
    double a[PG_DIM_MAX], width[PG_DIM_MAX];
};

// UNIFORM-SPLIT of new integrals (axis 0 varying fastest, corners a_k plus
// digit * width_k rounded twice as written), block row y = j-th new slot.
__global__ void k_batch_init(int d, int g, int64_t n, const BatchBox B,
                             const int32_t *__restrict__ new_slots,
                             const BInst *__restrict__ inst,
                             double *__restrict__ lo, double *__restrict__ w,
                             int64_t ld, uint32_t *__restrict__ inst_out) {
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t slot = (uint32_t)new_slots[blockIdx.y];
    const int64_t j = inst[slot].out_start + r;
    int64_t q = r;
    for (int k = 0; k < d; ++k) {
        const int64_t digit = q % g;
        q /= g;
        const double off = (double)digit * B.width[k];
        lo[k * ld + j] = B.a[k] + off;
        w[k * ld + j] = B.width[k];
    }
    inst_out[j] = slot;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_batch_tables(hipStream_t st, int nslots, const int32_t *order,
                               const BInst *inst, BSeg *segs, BCls *cls) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_tables, dim3((unsigned)nslots), dim3(256), 0,
                       st, order, inst, segs, cls);
    return hipGetLastError();
}

hipError_t launch_batch_classify(hipStream_t st, int64_t ncls, const BCls *cls,
                                 const BInst *inst, const double *V, double *E,
                                 const double *Vp, uint8_t *A,
                                 SegPartials part) {
    if (ncls <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_classify, dim3((unsigned)ncls), dim3(LIST_THREADS),
                       0, st, cls, inst, V, E, Vp, A, part);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(hipStream_t st, int nslots,
                               const int32_t *order, const BInst *inst,
                               SegPartials part, uint32_t *offsets,
                               Totals *tot, Totals *host_tot) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_reduce, dim3(nslots), dim3(REDUCE_THREADS), 0, st,
                       order, inst, part, offsets, tot, host_tot);
    return hipGetLastError();
}

hipError_t launch_batch_search_pass(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, double *tpart,
                                    const double2 *tlo, const double2 *thi) {
    if (nseg <= 0 || nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_trials, dim3((unsigned)nseg), dim3(LIST_THREADS),
                       0, st, segs, nseg, inst, E, A_rel, states, tpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_walk, dim3(nslots), dim3(SCAN_THREADS), 0, st,
                       order, inst, nseg, tpart, states, tlo, thi);
    return hipGetLastError();
}

hipError_t launch_batch_search_hist(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, uint32_t *cnt,
                                    unsigned long long *sum, double2 *tlo,
                                    double2 *thi) {
    if (nseg <= 0 || nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_hist,
                       dim3((unsigned)((nseg + BHIST_SEGS - 1) / BHIST_SEGS)),
                       dim3(LIST_THREADS), 0, st, segs, nseg, inst, states, E,
                       A_rel, cnt, sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_hist_walk, dim3(nslots), dim3(HIST_THREADS), 0,
                       st, order, inst, states, cnt, sum, tlo, thi);
    return hipGetLastError();
}

hipError_t launch_batch_count(hipStream_t st, int64_t nseg, const BSeg *segs,
                              const BInst *inst, const SearchState *states,
                              const double *V, const double *E,
                              const uint8_t *A_rel, SegPartials part) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_count, dim3((unsigned)nseg), dim3(LIST_THREADS),
                       0, st, segs, inst, states, V, E, A_rel, part);
    return hipGetLastError();
}

hipError_t launch_batch_compact(hipStream_t st, int d, int64_t nseg,
                                const BSeg *segs, const BInst *inst,
                                const SearchState *states,
                                const uint8_t *A_rel, const double *E,
                                const double *V, const uint8_t *K,
                                const double *lo, const double *w, int64_t ld,
                                const uint32_t *offsets, double *lo_out,
                                double *w_out, double *Vp,
                                uint32_t *inst_out) {
    if (nseg <= 0) return hipSuccess;
    static_assert(PG_DIM_MIN == 2 && PG_DIM_MAX == 10, "one kernel per dimension");
    decltype(&k_batch_compact<2>) k = nullptr;
    switch (d) {
    case 2: k = k_batch_compact<2>; break;
    case 3: k = k_batch_compact<3>; break;
    case 4: k = k_batch_compact<4>; break;
    case 5: k = k_batch_compact<5>; break;
    case 6: k = k_batch_compact<6>; break;
    case 7: k = k_batch_compact<7>; break;
    case 8: k = k_batch_compact<8>; break;
    case 9: k = k_batch_compact<9>; break;
    case 10: k = k_batch_compact<10>; break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)nseg), dim3(BCOMPACT_THREADS), 0, st,
                       segs, inst, states, A_rel, E, V, K, lo, w, ld, offsets,
                       lo_out, w_out, Vp, inst_out);
    return hipGetLastError();
}

hipError_t launch_batch_init(hipStream_t st, int d, int g, const double *a,
                             const double *width, int nnew,
                             const int32_t *new_slots, const BInst *inst,
                             double *lo, double *w, int64_t ld,
                             uint32_t *inst_out) {
    if (nnew <= 0) return hipSuccess;
    BatchBox B;
    int64_t n = 1;
    for (int k = 0; k < d; ++k) {
        B.a[k] = a[k];
        B.width[k] = width[k];
        n *= g;
    }
    hipLaunchKernelGGL(k_batch_init, dim3((unsigned)((n + 255) / 256), nnew),
                       dim3(256), 0, st, d, g, n, B, new_slots, inst, lo, w,
                       ld, inst_out);
    return hipGetLastError();
}

}  // namespace pg
