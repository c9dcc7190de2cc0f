// pg_list.hip -- gfx950 list kernels of one PAGANI iteration (Algorithm 2):
// uniform split, two-level error + rel-err classification + sums, the
// threshold search of Algorithm 3, and filter + split. The per-segment
// arithmetic lives in pg_device.hpp, shared with the many-integral kernels.
//
// These kernels are HBM bound; they stream SoA arrays with coalesced
// accesses and reduce in a fixed order (no floating-point atomics), so runs
// are bit-reproducible.
#include "pg_device.hpp"

#include <hip/hip_runtime.h>

namespace pg {

// TWO-LEVEL-ERROR + REL-ERR-CLASSIFY + per-segment sums. Unpaired: block b
// is segment b. Paired: block b takes pairs [b SEG, (b+1) SEG) of the two
// halves and writes segments b (lower half) and nh + b (upper half).
__global__ void __launch_bounds__(LIST_THREADS)
k_classify(int64_t n, int paired, const double *__restrict__ V,
           double *__restrict__ E, const double *__restrict__ Vp, double tau,
           int relerr, uint8_t *__restrict__ A, SegPartials part) {
    const int64_t b = blockIdx.x;
    if (!paired) {
        const int64_t s0 = b * SEG, s1 = s0 + SEG < n ? s0 + SEG : n;
        classify_segment(0, s0, s1, 0, 0, 0, V, E, Vp, tau, relerr, A, part,
                         b, -1);
        return;
    }
    const int64_t half = n / 2;
    const int64_t nh = (half + SEG - 1) / SEG;
    const int64_t q0 = b * SEG, q1 = q0 + SEG < half ? q0 + SEG : half;
    classify_segment(1, q0, q1, 0, half, 0, V, E, Vp, tau, relerr, A, part, b,
                     nh + b);
}

// Per-segment count and sums of A = A_rel AND (E > t); E == nullptr: A_rel.
// With a search state, t is the accepted threshold (or none if it failed).
__global__ void __launch_bounds__(LIST_THREADS)
k_seg_count(int64_t n, int paired, double t, const double *__restrict__ V,
            const double *__restrict__ E, const uint8_t *__restrict__ A_rel,
            const SearchState *__restrict__ S, SegPartials part) {
    int mode = E ? 2 : 1;
    if (S) {
        mode = S->ok ? 2 : 1;
        t = S->t_acc;
    }
    int64_t s0, s1;
    seg_range(blockIdx.x, n, paired, &s0, &s1);
    count_segment(s0, s1, mode, t, V, E, A_rel, part, blockIdx.x);
}

// Single-block totals of the segment partials + exclusive scan of the counts
__global__ void __launch_bounds__(REDUCE_THREADS)
k_reduce_scan(int64_t nseg, SegPartials part, uint32_t *__restrict__ offsets,
              Totals *__restrict__ tot, Totals *__restrict__ host_tot,
              const SearchState *__restrict__ state,
              SearchState *__restrict__ host_state, uint64_t *host_seq,
              uint64_t seq) {
    const Totals t = reduce_scan_segments(0, nseg, part, offsets, tot);
    // the host's copies (pinned host memory mapped into the device's
    // address space), so that no copy has to be queued behind this kernel;
    // the totals straight from registers
    if (threadIdx.x == 0) {
        if (host_tot) *host_tot = t;
        if (host_state) *host_state = *state;
        // then the sequence number the host polls for: once it reads `seq`
        // there, the copies above are visible to it as well
        if (host_seq) {
            __threadfence_system();
            __hip_atomic_store(host_seq, seq, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// The state a search starts from (Algorithm 3): first threshold e_it / n,
// P_max = 0.25, min / max E from the totals of the pass before it.
__device__ inline SearchState search_start(int64_t n, double e_it,
                                           double allowance, int relax,
                                           const Totals &minmax) {
    SearchState s{};
    s.n = n;
    s.e_it = e_it;
    s.allowance = allowance;
    s.relax = relax;
    s.mn = minmax.emin;
    s.mx = minmax.emax;
    s.t = e_it / (double)n;
    s.P_max = 0.25;
    s.t_acc = -__builtin_huge_val();
    return s;
}

__global__ void k_search_init(SearchState *__restrict__ S, int64_t n,
                              double e_it, double allowance, int relax,
                              const Totals *__restrict__ minmax) {
    if (threadIdx.x != 0) return;
    *S = search_start(n, e_it, allowance, relax, *minmax);
}

// Regions per histogram block for a list of more than 256 segments: about
// n / 256, rounded up to whole segments, at most HIST_RANGE.
__host__ __device__ inline int64_t hist_span(int64_t n) {
    const int64_t nseg = (n + SEG - 1) / SEG;
    int64_t per = (nseg + 255) / 256;
    if (per > HIST_RANGE / SEG) per = HIST_RANGE / SEG;
    return per * SEG;
}

// Error histogram of the A_rel regions, one block per segment, then the
// trials it decides (see hist_walk).
__global__ void __launch_bounds__(LIST_THREADS)
k_hist(int64_t n, const double *__restrict__ E,
       const uint8_t *__restrict__ A_rel, const Totals *__restrict__ minmax,
       uint32_t *__restrict__ cnt, unsigned long long *__restrict__ sum) {
    // lists of up to 256 segments: one block each; longer ones: blocks of
    // up to HIST_RANGE regions, about 256 of them
    const int64_t nseg = (n + SEG - 1) / SEG;
    const int64_t span = nseg <= 256 ? SEG : hist_span(n);
    const int64_t s0 = (int64_t)blockIdx.x * span;
    const int64_t s1 = s0 + span < n ? s0 + span : n;
    hist_segment(s0, s1, E, A_rel, hist_key(minmax->emax), cnt, sum);
}

// Starts the search (as k_search_init) and walks the trials the histogram
// decides; its bound tables stay in tlo / thi for the passes after it.
__global__ void __launch_bounds__(HIST_THREADS)
k_hist_walk(SearchState *__restrict__ S, uint32_t *__restrict__ cnt,
            unsigned long long *__restrict__ sum, double2 *__restrict__ tlo,
            double2 *__restrict__ thi, int64_t n, double e_it,
            double allowance, int relax, const Totals *__restrict__ minmax) {
    const SearchState init = search_start(n, e_it, allowance, relax, *minmax);
    hist_walk(init, S, cnt, sum, tlo, thi);
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
    double fe[TRIAL_M];
#pragma unroll
    for (int m = 0; m < TRIAL_M; ++m) { cnt[m] = 0; fe[m] = 0.0; }
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
        blk_part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// Adds the block sums of one pass in a fixed order and walks the tree,
// then decides the trials after it that the histogram's bound tables allow.
__global__ void __launch_bounds__(SCAN_THREADS)
k_trial_walk(int nblk, const double *__restrict__ blk_part,
             SearchState *__restrict__ S, const double2 *__restrict__ tlo,
             const double2 *__restrict__ thi) {
    __shared__ double tot[2 * TRIAL_M];
    if (S->done) return;
    sum_trial_parts(blk_part, nblk, nblk, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        SearchState st = *S;
        walk_tree(st, tot);
        if (st.table) bounds_walk(st, tlo, thi);
        *S = st;
    }
}

// FILTER + parent update + SPLIT: block b compacts segment b; its base is
// the exclusive scan of the segment counts. The dimension is a template
// argument, so a thread's two boxes take 4 D registers.
template <int D>
__global__ void __launch_bounds__(LIST_THREADS)
k_compact_split(int64_t n, int paired, double t,
                const uint8_t *__restrict__ A_rel, const double *__restrict__ E,
                const double *__restrict__ V, const uint8_t *__restrict__ K,
                const double *__restrict__ lo, const double *__restrict__ w,
                int64_t ld_in, const uint32_t *__restrict__ offsets,
                int64_t na, double *__restrict__ lo_out,
                double *__restrict__ w_out, int64_t ld_out,
                double *__restrict__ Vp) {
    int64_t s0, s1;
    seg_range(blockIdx.x, n, paired, &s0, &s1);
    compact_segment<SEG, LIST_THREADS, D>(D, s0, s1, E ? 2 : 1, t, A_rel, E, V,
                                          K, lo, w, ld_in, offsets[blockIdx.x],
                                          na, lo_out, w_out, ld_out, Vp, 0,
                                          nullptr, 0);
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
                              uint32_t *offsets, Totals *tot, Totals *host_tot,
                              const SearchState *state,
                              SearchState *host_state, uint64_t *host_seq,
                              uint64_t seq) {
    hipLaunchKernelGGL(k_reduce_scan, dim3(1), dim3(REDUCE_THREADS), 0, st, nseg,
                       part, offsets, tot, host_tot, state, host_state,
                       host_seq, seq);
    return hipGetLastError();
}

hipError_t launch_search_hist(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              uint32_t *cnt, unsigned long long *sum,
                              double2 *tlo, double2 *thi, double e_it,
                              double allowance, int relax,
                              const Totals *minmax) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_search_init, dim3(1), dim3(64), 0, st, S, n,
                           e_it, allowance, relax, minmax);
        return hipGetLastError();
    }
    const int64_t nseg = seg_count(n, 0);
    const int64_t span = nseg <= 256 ? SEG : hist_span(n);
    hipLaunchKernelGGL(k_hist, dim3((unsigned)((n + span - 1) / span)),
                       dim3(LIST_THREADS), 0, st, n, E, A_rel, minmax, cnt,
                       sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hist_walk, dim3(1), dim3(HIST_THREADS), 0, st, S, cnt,
                       sum, tlo, thi, n, e_it, allowance, relax, minmax);
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
                              double *blk_part, const double2 *tlo,
                              const double2 *thi) {
    const int blocks = trial_blocks(n);
    hipLaunchKernelGGL(k_trials, dim3((unsigned)blocks), dim3(TRIAL_THREADS), 0,
                       st, n, E, A_rel, S, blk_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trial_walk, dim3(1), dim3(SCAN_THREADS), 0, st,
                       blocks, blk_part, S, tlo, thi);
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
    static_assert(PG_DIM_MIN == 2 && PG_DIM_MAX == 10, "one kernel per dimension");
    decltype(&k_compact_split<2>) k = nullptr;
    switch (d) {
    case 2: k = k_compact_split<2>; break;
    case 3: k = k_compact_split<3>; break;
    case 4: k = k_compact_split<4>; break;
    case 5: k = k_compact_split<5>; break;
    case 6: k = k_compact_split<6>; break;
    case 7: k = k_compact_split<7>; break;
    case 8: k = k_compact_split<8>; break;
    case 9: k = k_compact_split<9>; break;
    case 10: k = k_compact_split<10>; break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)seg_count(n, paired)),
                       dim3(LIST_THREADS), 0, st, n, paired, t, A_rel, E, V,
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
