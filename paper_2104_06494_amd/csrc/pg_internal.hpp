// pg_internal.hpp -- types and launchers shared by the kernels and the host
// driver of the PAGANI library (gfx950). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pagani.h"

namespace pg {

// Regions handled by one block of the list kernels (classify, threshold
// count, compact + split). A segment is a contiguous run of at most SEG
// regions; segments never straddle the two halves of a paired list.
constexpr int SEG = 2048;
constexpr int LIST_THREADS = 256;
// Blocks (at most) and threads per block of a threshold-trial pass.
constexpr int TRIAL_BLOCKS = 256;
constexpr int TRIAL_THREADS = 1024;
// Thresholds tested per trial pass: a complete binary tree of depth 4 of the
// search's possible next steps.
constexpr int TRIAL_DEPTH = 4;
constexpr int TRIAL_M = (1 << TRIAL_DEPTH) - 1;
// Waves (at most) sharing the 64 regions of an EVALUATE block.
constexpr int EVAL_MAX_WAVES = 8;
// Threads of the single-block reduce/scan kernels.
constexpr int SCAN_THREADS = 1024;

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
// e^x for x <= 0 (the Gaussian's and the C0 integrand's exponent), no
// special cases: Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, with ln 2
// split into two doubles and the reduction done by two FMAs; e^r by the
// degree-11 polynomial interpolating e^r at the 12 Chebyshev points of
// [-ln2/2, ln2/2] (coefficients from 60-digit arithmetic rounded to double;
// the polynomial's relative error is 1.7e-17), Horner's rule; then 2^n by
// ldexp, which underflows gradually and reaches 0 below -745 without a
// test. Largest error 0.91 ulp on 2e5 points of [-745, 0] against a
// 40-digit reference. NaN in, NaN out; x = -inf (an exponent that
// overflowed) gives NaN.
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
    double *v, *e, *av, *ae, *emin, *emax;
    uint32_t *cnt;
};

// Totals of a list pass, read back by the host.
struct Totals {
    double v, e, av, ae, emin, emax;
    double cnt;      // number of active regions (exact as a double < 2^53)
    double pad;
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
    int mem;              // searching under memory pressure
    int last_dir, dir_changes, trials;
    int done, ok;
};

// Bins of the error histogram a threshold search starts from (per integral).
constexpr int HIST_BINS = 2048;

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
hipError_t launch_batch_reduce(hipStream_t st, int nslots,
                               const int32_t *order, const BInst *inst,
                               SegPartials part, uint32_t *offsets,
                               Totals *tot);
hipError_t launch_batch_search_pass(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, double *tpart);
// Histogram of every searching slot's errors and the trials it decides
// (cnt / sum: HIST_BINS per slot, zero on entry and left zero).
hipError_t launch_batch_search_hist(hipStream_t st, int64_t nseg,
                                    const BSeg *segs, int nslots,
                                    const int32_t *order, const BInst *inst,
                                    const double *E, const uint8_t *A_rel,
                                    SearchState *states, uint32_t *cnt,
                                    unsigned long long *sum);
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
// NULL): the kernel also leaves there the totals and a copy of *state.
hipError_t launch_reduce_scan(hipStream_t st, int64_t nseg, SegPartials part,
                              uint32_t *offsets, Totals *tot,
                              Totals *host_tot = nullptr,
                              const SearchState *state = nullptr,
                              SearchState *host_state = nullptr);
hipError_t launch_search_init(hipStream_t st, SearchState *S, int64_t n,
                              double e_it, double allowance, int mem,
                              const Totals *minmax);
// The search's error histogram and the trials it decides (k_hist +
// k_hist_walk); cnt / sum hold HIST_BINS bins, zero on entry and left zero.
hipError_t launch_search_hist(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              uint32_t *cnt, unsigned long long *sum);
// One pass (TRIAL_DEPTH trials) of the search: k_trials + k_trial_walk; a
// no-op once the search has ended. blk_part holds 2 TRIAL_M x TRIAL_BLOCKS
// doubles.
hipError_t launch_search_pass(hipStream_t st, int64_t n, const double *E,
                              const uint8_t *A_rel, SearchState *S,
                              double *blk_part);
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
