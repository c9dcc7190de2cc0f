// pg_internal.hpp -- types and launchers shared by the kernels and the host
// driver of the PAGANI library (gfx950). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pagani.h"
#include "pg_eval_defs.hpp"

namespace pg {

// Regions handled by one block of the list kernels (classify, threshold
// count, compact + split). A segment is a contiguous run of at most SEG
// regions; segments never straddle the two halves of a paired list.
constexpr int SEG = 1024;
constexpr int LIST_THREADS = 256;
// Segment length of the many-integral list (pg_batch.hip, pg_adjoint.hip):
// the derivative kernel gathers each segment's leaves into one block, which
// wants long segments, while the single list gains from more, shorter
// blocks on its mid-sized lists.
constexpr int BSEG = 2048;
static_assert(SEG <= BSEG && BSEG % SEG == 0, "segment lengths");
// Blocks (at most) and threads per block of a threshold-trial pass.
constexpr int TRIAL_BLOCKS = 256;
constexpr int TRIAL_THREADS = 1024;
// Thresholds tested per trial pass: a complete binary tree of depth 4 of the
// search's possible next steps.
constexpr int TRIAL_DEPTH = 4;
constexpr int TRIAL_M = (1 << TRIAL_DEPTH) - 1;
// Threads of the single-block walk kernels (at least 32 TRIAL_M: the trial
// sums take 16 threads each).
constexpr int SCAN_THREADS = 1024;
// Threads of a block reducing segment partials (single list: one block;
// many integrals: one per slot). A list has at most a few thousand
// segments, and fewer waves shorten the block's barrier and merge.
constexpr int REDUCE_THREADS = 256;


// Segment geometry of a list of n regions (paired: two halves of n/2).
__host__ __device__ inline int64_t seg_count(int64_t n, int paired) {
    if (n <= 0) return 0;
    if (!paired) return (n + SEG - 1) / SEG;
    int64_t half = n / 2;
    return 2 * ((half + SEG - 1) / SEG);
}
__host__ __device__ inline void seg_range(int64_t s, int64_t n, int paired,
                                          int64_t *start, int64_t *end) {
    if (!paired) {
        *start = s * SEG;
        *end = (*start + SEG < n) ? *start + SEG : n;
        return;
    }
    int64_t half = n / 2;
    int64_t nh = (half + SEG - 1) / SEG;
    int64_t base = 0, j = s;
    if (s >= nh) { base = half; j = s - nh; }
    *start = base + j * SEG;
    int64_t e = (j + 1) * SEG;
    *end = base + (e < half ? e : half);
}

// Per-segment partial results written by the list kernels.
struct SegPartials {
    double *v, *e, *av, *ae, *fv, *emin, *emax;
    uint32_t *cnt;
};

// Totals of a list pass, read back by the host.
struct Totals {
    double v, e, av, ae, emin, emax;
    double cnt;      // number of active regions (exact as a double < 2^53)
    double fv;       // sum of V over the regions not active
};

// Limits of the threshold search (the paper bounds it without numbers).
constexpr int THR_MAX_TRIALS = 64;
constexpr int THR_MAX_DIRCHG = 10;

// State of one threshold search (Algorithm 3), kept in device memory.
struct SearchState {
    int64_t n;            // s_it
    double e_it;          // error of the regions being processed
    double allowance;     // e_it - e_b = tau |v_tot| - e_f
    double mn, mx;        // min / max of E over the list
    double t;             // next threshold to try (root of the next pass)
    double P_max;
    double t_acc;         // accepted threshold
    int relax;            // P_max grows at each direction change
    int last_dir, dir_changes, trials;
    int done, ok;
    int table;            // this search's histogram bound tables are stored
};

// Bins of the error histogram a threshold search starts from (per integral).
constexpr int HIST_BINS = 2048;
// Entries of each of the two bound tables a histogram leaves per integral
// (prefix bounds at every bin edge), so that trials are decided from it
// again after each exact pass.
constexpr int HIST_TAB = HIST_BINS + 1;

// ---- many integrals in one list (pg_batch.hip) ---------------------------
// Each live integral of a batched run owns a slot. Its regions are
// contiguous in the list; its survivors' children go to its own block of
// the next list (lower halves, then upper halves), so sibling, parent and
// segment arithmetic is the single-integral arithmetic shifted by `start`.
constexpr int BATCH_MAX_SLOTS = 1024;

struct BInst {
    int64_t start, n;         // its regions in the current list
    int64_t out_start, na;    // survivors; children at out_start + [0, 2 na)
    int64_t seg0, nseg;       // its segments in the segment table
    int64_t cls0, ncls;       // its classify items
    double tau;               // rel_tol
    int32_t relerr, paired;
    int32_t live;             // 0: ends this iteration, nothing survives
    int32_t searching;        // a threshold search runs this iteration
    int64_t fin_base;         // its leaves of this iteration start here
    int32_t owner;            // index of the integral in the caller's batch
    int32_t pad2;
};

// A segment (no segment straddles an integral or the halves of a paired
// integral) and a classify item (a segment, or for paired integrals a range
// of sibling pairs feeding one lower and one upper segment).
struct BSeg {
    int64_t start, end;
    uint32_t slot;
    int32_t pad;
};
struct BCls {
    int64_t q0, q1, s_lo, s_hi;
    uint32_t slot;
    int32_t pad;
};

hipError_t launch_batch_tables(hipStream_t st, int nslots, const int32_t *order,
                               const BInst *inst, BSeg *segs, BCls *cls);
hipError_t launch_batch_classify(hipStream_t st, int64_t ncls, const BCls *cls,
                                 const BInst *inst, const double *V, double *E,
                                 const double *Vp, uint8_t *A,
                                 SegPartials part);
// host_tot (device address of mapped pinned host memory, or NULL): each
// slot's totals are also left there.
hipError_t launch_batch_reduce(hipStream_t st, int nslots,
                               const int32_t *order, const BInst *inst,
                               SegPartials part, uint32_t *offsets,
                               Totals *tot, Totals *host_tot = nullptr);
// One exact pass for every searching slot, then the trials each slot's
// bound tables (tlo / thi: HIST_TAB per slot) decide after it.
hipError_t launch_batch_search_pass(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, double *tpart,
                                    const double2 *tlo, const double2 *thi);
// Histogram of every searching slot's errors and the trials it decides
// (cnt / sum: HIST_BINS per slot, zero on entry and left zero); its bound
// tables go to tlo / thi (HIST_TAB per slot).
hipError_t launch_batch_search_hist(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, uint32_t *cnt,
                                    unsigned long long *sum, double2 *tlo,
                                    double2 *thi);
hipError_t launch_batch_count(hipStream_t st, int64_t nseg, const BSeg *segs,
                              const BInst *inst, const SearchState *states,
                              const double *V, const double *E,
                              const uint8_t *A_rel, SegPartials part);
hipError_t launch_batch_compact(hipStream_t st, int d, int64_t nseg,
                                const BSeg *segs, const BInst *inst,
                                const SearchState *states,
                                const uint8_t *A_rel, const double *E,
                                const double *V, const uint8_t *K,
                                const double *lo, const double *w, int64_t ld,
                                const uint32_t *offsets, double *lo_out,
                                double *w_out, double *Vp,
                                uint32_t *inst_out);
// ---- parameter derivative over the final partition (pg_adjoint.hip) ------
// Largest parameter count of a family (2d at d = PG_DIM_MAX).
constexpr int GRAD_MAX = 2 * PG_DIM_MAX + 2;
// Parameters as the derivative kernels take them: the integrand's (as in
// FParams) and each parameter's constant derivative factor (pg_adjoint.hip).
struct GParams {
    double p[2 * PG_DIM_MAX + 2];
    double gs[GRAD_MAX];
};
// Blocks per segment of the derivative kernel (the leaves are dealt out).
constexpr int ADJ_SPLIT = 4;
// Optional copy of the leaves: SoA [d][ld] corners and widths, the owner
// integral of each; leaf k of an iteration goes to base + k.
struct LeafOut {
    double *lo, *w;
    int32_t *owner;
    int64_t ld, base;
};
int grad_nparams(int family, int d);
bool adjoint_supported(int family, int d);
// gpart holds GRAD_MAX x nseg x ADJ_SPLIT doubles.
hipError_t launch_batch_adjoint(hipStream_t st, int family, int d,
                                int64_t nseg, const BSeg *segs,
                                const BInst *inst, const SearchState *states,
                                const uint8_t *A_rel, const double *E,
                                const double *lo, const double *w, int64_t ld,
                                const GParams *gtab, const Rule &R,
                                double *gpart, const uint32_t *offsets,
                                const LeafOut &out);
// git[slot * GRAD_MAX + q]: this iteration's derivative of each slot.
hipError_t launch_batch_grad_reduce(hipStream_t st, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const GParams *gtab, int np,
                                    const double *gpart, int64_t nseg,
                                    double *git);

// Uniform-Split of `nnew` new integrals: slot new_slots[j] gets g^d boxes
// at inst[slot].out_start of the next list, tagged with its slot.
hipError_t launch_batch_init(hipStream_t st, int d, int g, const double *a,
                             const double *width, int nnew,
                             const int32_t *new_slots, const BInst *inst,
                             double *lo, double *w, int64_t ld,
                             uint32_t *inst_out);

// ---- launchers (pg_evaluate.hip, pg_list.hip); all queue on `st` ---------
hipError_t launch_init(hipStream_t st, int d, int g, const double *a,
                       const double *width, double *lo, double *w,
                       int64_t ld);
// waves: waves per block (1..8), block covers 64 regions. With inst and
// table, region i takes its parameters from table[inst[i]] (P is unused).
hipError_t launch_evaluate(hipStream_t st, int family, int d,
                           const FParams &P, const Rule &R, int64_t n,
                           const double *lo, const double *w, int64_t ld,
                           double *V, double *E, uint8_t *K, int waves,
                           const uint32_t *inst = nullptr,
                           const FParams *table = nullptr);
bool evaluate_supported(int family, int d);
hipError_t launch_fvalues(hipStream_t st, int family, int d, const FParams &P,
                          int64_t n, const double *x, int64_t ld, double *y);
int evaluate_max_waves(int d);
hipError_t launch_classify(hipStream_t st, int64_t n, int paired,
                           const double *V, double *E, const double *Vp,
                           double tau, int relerr, uint8_t *A,
                           SegPartials part);
// S != nullptr: t is the search's accepted threshold (none if it failed).
hipError_t launch_seg_count(hipStream_t st, int64_t n, int paired, double t,
                            const double *V, const double *E,
                            const uint8_t *A_rel, const SearchState *S,
                            SegPartials part);
// host_tot / host_state (device addresses of mapped pinned host memory, or
// NULL): the kernel also leaves there the totals and a copy of *state, and
// then writes `seq` to host_seq (also mapped, or NULL) once both are
// visible to the host.
hipError_t launch_reduce_scan(hipStream_t st, int64_t nseg, SegPartials part,
                              uint32_t *offsets, Totals *tot,
                              Totals *host_tot = nullptr,
                              const SearchState *state = nullptr,
                              SearchState *host_state = nullptr,
                              uint64_t *host_seq = nullptr, uint64_t seq = 0);
// Starts a search in *S (first threshold e_it / n; min / max E from the
// totals `minmax` of the pass before it) and decides the trials its error
// histogram allows (k_hist + k_hist_walk); cnt / sum hold HIST_BINS bins,
// zero on entry and left zero; the histogram's bound tables are left in
// tlo / thi (HIST_TAB entries each).
hipError_t launch_search_hist(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              uint32_t *cnt, unsigned long long *sum,
                              double2 *tlo, double2 *thi, double e_it,
                              double allowance, int relax,
                              const Totals *minmax);
// One pass (TRIAL_DEPTH trials) of the search: k_trials + k_trial_walk,
// which then decides the trials the bound tables tlo / thi allow; a no-op
// once the search has ended. blk_part holds 2 TRIAL_M x TRIAL_BLOCKS
// doubles.
hipError_t launch_search_pass(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              double *blk_part, const double2 *tlo,
                              const double2 *thi);
hipError_t launch_compact_split(hipStream_t st, int d, int64_t n, int paired,
                                double t, const uint8_t *A_rel,
                                const double *E, const double *V,
                                const uint8_t *K, const double *lo,
                                const double *w, int64_t ld_in,
                                const uint32_t *offsets, int64_t n_active,
                                double *lo_out, double *w_out, int64_t ld_out,
                                double *Vp);
hipError_t launch_apply_threshold(hipStream_t st, int64_t n, double t,
                                  const uint8_t *A_rel, const double *E,
                                  uint8_t *A_out);

}  // namespace pg
