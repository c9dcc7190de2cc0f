/*
 * pagani.h -- C interface of the MI355X (gfx950) PAGANI integrator.
 *
 * PAGANI (Sakiotis et al., SC'21) integrates f over a box by refining every
 * live sub-region in lock-step (Section 3.1, Algorithm 2): each iteration
 * evaluates all regions with a degree-7 cubature rule (Section 3.2), refines
 * the error estimates with the two-level scheme, classifies regions as
 * finished or active (Section 3.5.1, and Algorithm 3 for the threshold
 * search of Section 3.5.3), removes the finished ones and bisects the rest.
 *
 * Conventions shared by every entry point
 *  - Return value: a pg_status. Negative values are errors (the message is
 *    in pg_last_error); PG_OK and the positive values are results.
 *  - Host pointers are read (or written) only during the call. Device
 *    pointers must stay valid until the work queued on the context's
 *    stream has finished; the step entry points only queue work.
 *  - Region lists are structure-of-arrays in device memory: lower corners
 *    lo[k * ld + i] and widths w[k * ld + i] for axis k of region i, with
 *    leading dimension ld >= n. Region i is the box [lo_i, lo_i + w_i].
 *  - Integrands are a family id plus a parameter vector (no function
 *    pointers: the integrand is inlined into the evaluation kernel):
 *      PG_PRODUCT_PEAK  prod_k 1 / (a_k^-2 + (x_k - u_k)^2)  params a[d], u[d]
 *                       (a_k != 0)
 *      PG_GAUSSIAN      exp(-sum_k a_k^2 (x_k - u_k)^2)      params a[d], u[d]
 *                       (|a_k| up to about 3e4 on boxes of unit size)
 *      PG_OSCILLATORY   cos(2 pi u_1 + sum_k a_k x_k)        params a[d], u_1
 *      PG_CORNER_PEAK   (1 + sum_k a_k x_k)^-(d+1)          params a[d]
 *                       (1 + sum_k a_k x_k > 0 on the box)
 *      PG_MONOMIAL      prod_k x_k^alpha_k                  params alpha[d]
 *      PG_C0            exp(-sum_k a_k |x_k - u_k|)         params a[d], u[d]
 *      PG_DISCONTINUOUS exp(sum_k a_k x_k) if every x_k < c_k, else 0
 *                                                          params a[d], c[d]
 *      PG_BOX           (sum_k x_k^2)^p                     params p (p >= 0)
 *    (Section 4.1's test functions f1..f8 belong to these families.)
 *  - Dimensions PG_DIM_MIN..PG_DIM_MAX are supported.
 *  - One context serves one caller at a time; calls on one context must not
 *    overlap.
 */
#ifndef PAGANI_H
#define PAGANI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PG_DIM_MIN 2
#define PG_DIM_MAX 10

typedef enum {
    PG_OK = 0,                 /* tolerance met */
    PG_MAX_ITERS = 1,          /* estimate valid, max_iters reached */
    PG_MEMORY_EXHAUSTED = 2,   /* estimate valid, list would exceed the cap
                                  and the threshold search failed (Sec. 3.5.2) */
    PG_NO_ACTIVE = 3,          /* estimate valid, every region finished but
                                  the tolerance is not met (Sec. 3.5.1) */
    PG_EINVAL = -1,            /* invalid argument */
    PG_ENOMEM = -2,            /* workspace too small / allocation failed */
    PG_EHIP = -3,              /* HIP runtime error */
    PG_EUNSUPPORTED = -4       /* family or dimension not built */
} pg_status;

typedef enum {
    PG_PRODUCT_PEAK = 0,
    PG_GAUSSIAN = 1,
    PG_OSCILLATORY = 2,
    PG_CORNER_PEAK = 3,
    PG_MONOMIAL = 4,
    PG_C0 = 5,
    PG_DISCONTINUOUS = 6,
    PG_BOX = 7
} pg_family;

/*
 * Error estimate of a region (the E of EVALUATE, Section 3.2):
 *  PG_ERR_RAW    |R7 - R5|: the degree-7 rule against its embedded
 *                degree-5 rule (the default).
 *  PG_ERR_NULL4  four null rules of the same points (Section 3.2 compares
 *                the basic rule with four further rules, as Cuhre does,
 *                Section 2): N1 of degree 5, N2 and N3 of degree 3, N4 of
 *                degree 1, fully symmetric, mutually orthogonal and of the
 *                degree-7 rule's norm. With e5 = |N1|, e3 = rms(N2, N3),
 *                e1 = |N4| and r = max(e3 / e1, e5 / e3): E = kappa_d r^2
 *                e3 if r <= 1/2 (the values fall like a resolved smooth
 *                integrand's), else max(e5, e3, e1); kappa_d = 2, 2, 3.8,
 *                15, 18, 21, 25, 29, 34 for d = 2..10 (twice the worst
 *                limit ratio of the true error to r^2 e3 over exp(a.x),
 *                and at least 2). No extra integrand evaluations; the
 *                split axis is unchanged.
 */
typedef enum {
    PG_ERR_RAW = 0,
    PG_ERR_NULL4 = 1
} pg_error_rule;

/*
 * How the threshold search (Algorithm 3) relaxes its accuracy requirement.
 * The search starts with P_max = 0.25 of the error the finished regions may
 * still carry and gives up after 10 direction changes or 64 trials.
 *  PG_PMAX_EVERY_CHANGE  P_max grows by 0.10 at every change of search
 *                        direction, up to 0.95, in every search: the rule as
 *                        Section 3.5.3 states it (the default).
 *  PG_PMAX_UNDER_MEMORY  a departure from Section 3.5.3: P_max grows only
 *                        in searches run because the live list would
 *                        overflow its cap (trigger (b) of Section 3.5.2);
 *                        searches run because the estimate's digits have
 *                        settled keep 0.25. It commits less error to
 *                        finished regions, and so ends fewer runs with every
 *                        region finished and the tolerance unmet.
 */
typedef enum {
    PG_PMAX_EVERY_CHANGE = 0,
    PG_PMAX_UNDER_MEMORY = 1
} pg_pmax_relax;

/*
 * The error budget of the threshold search's accuracy requirement
 * (Algorithm 3: finished error <= P_max times the budget). The listing's
 * budget is the error the finished regions may carry, tau |v_tot| - e_f
 * (its e_it - e_b, read so that Section 3.5.3's remark holds: finishing
 * more than it makes convergence impossible).
 *  PG_BUDGET_RESERVE  in a search started because the estimate's digits
 *                     have settled (trigger (a) of Section 3.5.2), the
 *                     finished regions -- those finished earlier and those
 *                     the relative-error test finishes now -- may carry only
 *                     tau times their own estimate, tau |v_f + sum of their
 *                     V| - e_f: by Lemma 1 (Section 3.5.1) the regions left
 *                     active may still end with tau |V| each, and Section
 *                     3.5.2 asks the search not to over-commit finished
 *                     error. A search started because the list would
 *                     overflow (trigger (b)) has the listing's budget:
 *                     there continuing is the only way on (the default).
 *  PG_BUDGET_LISTING  every search has the listing's budget. Under the
 *                     P_max rule of Section 3.5.3 its searches may commit so
 *                     much finished error that every region finishes with
 *                     the tolerance unmet (PG_NO_ACTIVE).
 */
typedef enum {
    PG_BUDGET_RESERVE = 0,
    PG_BUDGET_LISTING = 1
} pg_budget;

typedef struct pg_context pg_context;

typedef struct {
    int family;               /* pg_family */
    int dim;                  /* d */
    const double *params;     /* host array, layout per family (above) */
    int n_params;             /* 2d, 2d, d+1, d, d */
} pg_integrand;

typedef struct {
    double rel_tol;           /* tau_rel (Algorithm 2 input) */
    double abs_tol;           /* tau_abs */
    int init_splits;          /* g: the initial grid has g^d equal boxes */
    int max_iters;            /* it_max */
    int relerr_filter;        /* 1: classify by relative error (default);
                                 0: off, for sign-changing integrands (3.5.1) */
    int threshold_filter;     /* 1: threshold search on (Algorithm 3); 0: off */
    int64_t max_regions;      /* cap on the live list; 0: context capacity */
    int timing;               /* HIP events on the stream: 1 around each
                                 EVALUATE launch (phase_ms[0] only), 2
                                 around every phase; 0: none. Each event
                                 costs the run a few microseconds. */
    const char *trace_path;   /* non-NULL: write the decision trace (below) */
    int error_rule;           /* pg_error_rule */
    int pmax_relax;           /* pg_pmax_relax */
    int budget;               /* pg_budget */
} pg_options;

/* Default options (the inputs of Algorithm 2 and the user flag of Section
   3.5.1): rel_tol 1e-3, abs_tol 1e-20, g = 4, it_max = 100, both filters
   on, cap = capacity, no timing, no trace, error rule PG_ERR_RAW, P_max
   rule PG_PMAX_EVERY_CHANGE, budget PG_BUDGET_RESERVE. A zero-filled
   struct holds the same rules. */
void pg_default_options(pg_options *opt);

typedef struct {
    double estimate;          /* v + v_f */
    double error;             /* e + e_f */
    int status;               /* pg_status (>= 0) */
    int iterations;
    int64_t regions_evaluated;/* sum over iterations of the live count */
    int64_t fevals;           /* regions_evaluated * (2^d + 2d^2 + 2d + 1) */
    int64_t peak_regions;
    int64_t threshold_calls;
    int64_t threshold_trials;
    double phase_ms[4];       /* with timing: evaluate, post-processing
                                 (two-level, classify, sums), threshold
                                 search and the host's decisions, filter +
                                 split (Section 4.3.2); level 1 fills only
                                 the first */
    int64_t eval_launches;    /* number of evaluate kernel launches */
} pg_result;

/*
 * Bytes of device workspace for lists of up to `capacity` regions of up to
 * `dim_max` dimensions (two ping-pong region lists plus V, E, K, A,
 * parents and reduction scratch). Section 4 sets memory up once, outside
 * the timed integration; so does this library: nothing is allocated per
 * iteration. Returns 0 for a dimension outside PG_DIM_MIN..PG_DIM_MAX or a
 * capacity below 2.
 */
size_t pg_workspace_bytes(int dim_max, int64_t capacity);

/*
 * Create a context on HIP device `device`: the once-only set-up that Section
 * 4 keeps out of the timed integration. `workspace` is device memory of
 * at least pg_workspace_bytes(dim_max, capacity) bytes owned by the caller
 * (for example a PyTorch tensor's storage), or NULL to let the context
 * allocate (and later free) it; a caller's workspace must be 256-byte
 * aligned. `stream` is the hipStream_t all work is queued on, owned by the
 * caller; NULL is the device's null stream (PyTorch's default stream).
 * Errors: PG_EINVAL, PG_ENOMEM, PG_EHIP; *out is NULL then.
 */
int pg_context_create(int device, int dim_max, int64_t capacity,
                      void *workspace, size_t ws_bytes, void *stream,
                      pg_context **out);
/* Waits for the context's stream, then frees what the context allocated
   (not a caller's workspace). NULL is ignored. Call it while the HIP
   runtime is still up, not from a process-exit handler. */
void pg_context_destroy(pg_context *ctx);
/* Replace the stream work is queued on (a hipStream_t, NULL = null stream). */
int pg_context_set_stream(pg_context *ctx, void *stream);
/* Waves EVALUATE (Section 3.2) aims to keep in flight on this context's
   runs: blocks x waves per block, the waves of a block splitting the rule's
   points of its 64 regions. 0 restores the default, 2048 (the chip twice
   over); PG_EINVAL outside 256..65536. Meant to change speed only: the
   waves' partial sums are added in another order, so estimates move by
   rounding and a decision on an exact rounding tie could go the other way.
   Set by the autotuner of the many-integral driver. */
int pg_context_set_eval_waves(pg_context *ctx, int target);
/* Message of the last error on this context ("" if none). */
const char *pg_last_error(const pg_context *ctx);

/*
 * Whole run of Algorithm 2 over the box [lo, hi] (host arrays of dim
 * values). Blocks until the result is known. `out` is always written when
 * non-NULL; it holds a valid estimate whenever the return value is >= 0.
 * Errors: PG_EINVAL (lo >= hi on some axis, no positive tolerance, g < 1,
 * g^d above the cap, bad family/params), PG_ENOMEM (cap above capacity),
 * PG_EUNSUPPORTED, PG_EHIP.
 *
 * Decision trace (when opt->trace_path is set), little endian:
 *   header  char magic[8] = "PGTRACE2"; int32 d; int32 family;
 *           int64 pmax_relax, error_rule, budget (the run's rules)
 *   per iteration:
 *     int64 it, n, n_active; int32 thr_invoked, thr_ok, thr_trials,
 *     terminal (-1 = continues, else the pg_status the run ends with);
 *     double t, v, e, v_f, e_f; uint8 K[n]; uint8 A[n] (final flags)
 */
int pg_integrate(pg_context *ctx, const pg_integrand *f, const double *lo,
                 const double *hi, const pg_options *opt, pg_result *out);

/*
 * Many integrals of one family at once (B parameter vectors, row-major
 * params[b * n_params + k], same box [lo, hi] for all), each with its own
 * rel_tol[b] and abs_tol[b] (abs_tol may be NULL: opt->abs_tol for all).
 * Every integral runs exactly the iteration of pg_integrate (Algorithm 2)
 * with the options in opt, opt->max_regions being the cap of each integral;
 * the integrals share one region list and every kernel launch. At most
 * min(B, capacity / cap, 1024) integrals are in flight at a time; the rest
 * start as others finish. out[b] receives integral b's result (phase_ms
 * and the trace are not recorded). Returns PG_OK, or an error as
 * pg_integrate does (no integral has a result then).
 */
int pg_integrate_batch(pg_context *ctx, int family, int dim, int B,
                       const double *params, int n_params, const double *lo,
                       const double *hi, const double *rel_tol,
                       const double *abs_tol, const pg_options *opt,
                       pg_result *out);

/*
 * Optional copy of the partition a run ends on (its leaves: every region
 * finished on the way, by the relative-error test of Section 3.5.1 or a
 * threshold of Algorithm 3, and the live list when the run stops). Device
 * arrays owned by the caller: lo and w are structure-of-arrays [dim][ld]
 * (leaf k, axis j at j * ld + k), owner[ld] the index in the batch of the
 * integral a leaf belongs to (may be NULL). The run writes n leaves, in
 * iteration order; it fails with PG_ENOMEM if more than ld would be needed.
 */
typedef struct {
    double *lo;
    double *w;
    int32_t *owner;
    int64_t ld;
    int64_t n;          /* out */
} pg_leaves;

/*
 * pg_integrate plus the derivative of the estimate with respect to the
 * integrand's parameters (grad[n_params], host), taken over the partition
 * the run ends on: the estimate is the sum of the degree-7 rule values of
 * the leaves (Section 3.1: the finished regions' contributions plus the
 * live list's), and each is a weighted sum of f at points that do not move
 * with the parameters, so the derivative is the same weighted sum of
 * df/dparameter. Families with parameter derivatives: product peak and
 * Gaussian (a then u), oscillatory (a then u_1), corner peak (a);
 * PG_EUNSUPPORTED otherwise. leaves may be NULL. Runs through the batched
 * driver as a batch of one, so it takes the same decisions as
 * pg_integrate_batch on this integral. Returns like pg_integrate.
 */
int pg_integrate_grad(pg_context *ctx, const pg_integrand *f,
                      const double *lo, const double *hi,
                      const pg_options *opt, pg_result *out, double *grad,
                      pg_leaves *leaves);

/*
 * pg_integrate_batch plus each integral's parameter derivative over its
 * own final partition, grad[b * n_params + k] (host). leaves (may be NULL)
 * receives every integral's leaves, tagged by owner. Returns like
 * pg_integrate_batch.
 */
int pg_integrate_batch_grad(pg_context *ctx, int family, int dim, int B,
                            const double *params, int n_params,
                            const double *lo, const double *hi,
                            const double *rel_tol, const double *abs_tol,
                            const pg_options *opt, pg_result *out,
                            double *grad, pg_leaves *leaves);

/*
 * View of the live region list H of Algorithm 2 as the last pg_integrate
 * left it: the n regions of its last iteration with their V, (refined) E,
 * split axis K and rel-err flags A (Section 3.1 names these lists). Device
 * pointers into the context's workspace, valid until the next call that
 * uses the context; ld is the context's capacity. PG_EINVAL for NULL
 * arguments; n is 0 before the first run.
 */
typedef struct {
    int dim;
    int64_t n, ld;
    const double *lo, *w, *V, *E;
    const uint8_t *K, *A;
} pg_regions_view;
int pg_last_regions(const pg_context *ctx, pg_regions_view *out);

/* ---- the steps of one iteration, on caller-supplied device arrays ---- */

/*
 * EVALUATE (Section 3.2): for each of n regions, V = the degree-7
 * Genz-Malik rule, E = |R7 - R5| (its embedded degree-5 rule) and K = the
 * axis of largest fourth divided difference (ties within 1e-10 of the
 * maximum, or within 1e-12 of the size of the values entering the
 * differences, go to the widest axis, then the lowest index). Inputs lo, w
 * (ld >= n); outputs V[n], E[n], K[n]. Queued on the context's stream.
 */
int pg_evaluate(pg_context *ctx, const pg_integrand *f, int64_t n,
                const double *lo, const double *w, int64_t ld, double *V,
                double *E, uint8_t *K);

/*
 * pg_evaluate with the error estimate chosen by error_rule (pg_error_rule;
 * PG_EINVAL for other values). V and K are the same as pg_evaluate's.
 */
int pg_evaluate_rule(pg_context *ctx, const pg_integrand *f, int error_rule,
                     int64_t n, const double *lo, const double *w, int64_t ld,
                     double *V, double *E, uint8_t *K);

/*
 * The integrand alone: y[i] = f(x_i) for n points x_i with coordinates
 * x[k * ld + i] (device arrays). Section 3.2 evaluates f at the rule's
 * points; this is the same inlined code EVALUATE uses, for checking an
 * integrand and for counting its cost (the FLOP per evaluation in the
 * evaluate roofline). Queued on the context's stream. PG_EINVAL for bad
 * n / ld or NULL arrays, PG_EUNSUPPORTED for a family or dimension not
 * built.
 */
int pg_integrand_values(pg_context *ctx, const pg_integrand *f, int64_t n,
                        const double *x, int64_t ld, double *y);

/*
 * TWO-LEVEL-ERROR + REL-ERR-CLASSIFY + the sums of Algorithm 2 on n
 * regions. When `paired` is 1, n is even and regions i and i + n/2 are the
 * halves of the parent whose estimate is Vp[i]; E is then refined in place
 *   delta = |V_i + V_j - Vp| / 4, S = E_i + E_j,
 *   E <- E (1 + 2 delta / S) + delta   (E + delta when S = 0).
 * A[i] = 1 (active) iff E_i > rel_tol |V_i| (always 1 with relerr_filter 0).
 * sums (host, 8 doubles): sum V, sum E, sum A V, sum A E, sum A, min E,
 * max E, sum (1 - A) V. Blocks until the sums are known.
 */
int pg_classify(pg_context *ctx, int64_t n, int paired, const double *V,
                double *E, const double *Vp, double rel_tol,
                int relerr_filter, uint8_t *A, double *sums);

/*
 * THRESHOLD-CLASSIFY (Algorithm 3, Section 3.5.3) on n regions with errors
 * E and rel-err flags A_rel: searches t such that A = A_rel AND (E > t)
 * finishes more than half of the regions while the error of the regions it
 * finishes, summed over them, is <= P_max * allowance. e_it is the list's
 * total error (the first t is e_it / n). pg_integrate passes as allowance
 * the listing's e_it - e_b = tau |v_tot| - e_f, or, under
 * PG_BUDGET_RESERVE for a search the memory trigger did not start,
 * tau |v_f + sum of V over A_rel = 0| - e_f (see pg_budget; pg_classify
 * returns that sum). P_max starts at 0.25; with relax != 0 it grows by
 * 0.10 per direction change (max 0.95), as Section 3.5.3 states; with
 * relax = 0 it stays 0.25 (pg_integrate passes 0 only under
 * PG_PMAX_UNDER_MEMORY for a search the memory trigger did not start). At
 * most 64 trials and 10 direction changes. Returns 1 in *ok with t and
 * A_out (device, n bytes) on success; 0 and A_out = A_rel on failure.
 * PG_EINVAL for an empty list, a NULL argument or a non-finite e_it or
 * allowance. Blocks.
 */
int pg_threshold_search(pg_context *ctx, int64_t n, const double *E,
                        const uint8_t *A_rel, double e_it, double allowance,
                        int relax, uint8_t *A_out, int *ok, double *t,
                        int *trials);

/*
 * FILTER + parent update + SPLIT (the last three steps of Algorithm 2's
 * loop; Section 3.4 bisects every active region): stable compaction of the
 * regions with
 * A[i] = 1; the j-th survivor is bisected along axis K[i] into the lower
 * half at index j and the upper half at index j + n_active of the output
 * list (ld_out >= 2 n_active), and Vp[j] = V[i]. Writes *n_active (host).
 * Blocks until *n_active is known. Device arrays: lo, w (ld_in >= n), K, V,
 * A in; lo_out, w_out, Vp out (must not overlap the inputs). PG_EINVAL for
 * a bad dimension, n / ld or ld_out, or a NULL array.
 */
int pg_filter_split(pg_context *ctx, int dim, int64_t n, const double *lo,
                    const double *w, int64_t ld_in, const uint8_t *K,
                    const double *V, const uint8_t *A, double *lo_out,
                    double *w_out, int64_t ld_out, double *Vp,
                    int64_t *n_active);

/* ---- for callers that cannot allocate ---- */

/* Largest list pg_filter_split_noalloc accepts, and the bytes of device
   memory its scratch holds on every GPU the library runs on (from the first
   call on that GPU until the process ends). */
#define PG_NOALLOC_MAX_REGIONS (1LL << 26)
#define PG_NOALLOC_SCRATCH_BYTES (5u << 20)

/*
 * pg_filter_split for callers that cannot allocate device memory: code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc. It needs no context and calls no allocating routine: the
 * compaction's scratch (per-segment sums and counts, segment offsets,
 * totals) is a static device array of PG_NOALLOC_SCRATCH_BYTES per GPU,
 * whose address is looked up on the first call on each device. The caller
 * still owns every input and output. Arguments, layouts and results are
 * pg_filter_split's; work is queued on `stream` (a hipStream_t on the
 * current device, NULL = its null stream) and the call blocks until
 * *n_active is known and the output list is written. Errors (return
 * value only; there is no context to hold a message): PG_EINVAL for
 * n > PG_NOALLOC_MAX_REGIONS, a bad dimension, n / ld or ld_out, or a NULL
 * array; PG_EHIP for a HIP failure. Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (other streams, other threads)
 * race and must not be made.
 */
int pg_filter_split_noalloc(void *stream, int dim, int64_t n,
                            const double *lo, const double *w, int64_t ld_in,
                            const uint8_t *K, const double *V,
                            const uint8_t *A, double *lo_out, double *w_out,
                            int64_t ld_out, double *Vp, int64_t *n_active);

#ifdef __cplusplus
}
#endif
#endif /* PAGANI_H */
