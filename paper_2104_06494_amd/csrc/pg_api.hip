// pg_api.hip -- host driver and C interface of the PAGANI library.
//
// pg_integrate runs Algorithm 2 of the paper: per iteration one EVALUATE
// launch over the live list, one TWO-LEVEL + CLASSIFY launch with a
// single-block reduce/scan, one 64-byte read-back for the termination test
// and the threshold triggers, the threshold search of Algorithm 3 when it
// is triggered (several candidate thresholds tested per pass over the list,
// see search()), and one FILTER + SPLIT launch that writes the next list
// into the other half of a ping-pong buffer. Nothing is allocated per
// iteration; all buffers live in one workspace sized at context creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pg_internal.hpp"

using namespace pg;

// Waves in flight EVALUATE aims for by default: the chip twice over (256
// CUs x 4 SIMDs x 2).
constexpr int64_t EVAL_WAVE_TARGET = 2048;

struct pg_context {
    int device = 0;
    hipStream_t stream = nullptr;            // nullptr: the null stream
    int64_t wave_target = EVAL_WAVE_TARGET;  // EVALUATE's waves in flight
    int dim_max = 0;
    int64_t cap = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    double *lo[2] = {nullptr, nullptr}, *w[2] = {nullptr, nullptr};
    double *V = nullptr, *E = nullptr, *Vp = nullptr;
    uint8_t *K = nullptr, *A = nullptr, *A2 = nullptr;
    SegPartials part{};
    uint32_t *off = nullptr;
    double *search_part = nullptr;
    Totals *dtot = nullptr, *htot = nullptr;
    SearchState *dstate = nullptr, *hstate = nullptr;
    // device addresses of htot / hstate (pinned host memory mapped into
    // the device's address space): kernels leave the values the host reads
    // there directly, so no copy is queued before a wait
    Totals *htot_dev = nullptr;
    SearchState *hstate_dev = nullptr;
    // sequence word written after them (mapped as well), and the last value
    // the host asked for: the host polls it instead of waiting for the
    // stream, so it sees the values as soon as they land
    uint64_t *hseq = nullptr, *hseq_dev = nullptr;
    uint64_t seq = 0;
    // many-integral runs
    uint32_t *inst[2] = {nullptr, nullptr};
    // the slot header of a many-integral run, one device block (per run:
    // slot table, order, new-slot list, search states, in that order) and
    // its pinned staging copies, so that each upload is one copy
    char *b_hdr = nullptr, *hb_hdr = nullptr;
    BInst *b_inst = nullptr;
    SearchState *b_state = nullptr, *hb_state = nullptr;
    Totals *b_tot = nullptr, *hb_tot = nullptr;
    Totals *hb_tot_dev = nullptr;            // device address of hb_tot
    FParams *b_table = nullptr, *hb_table = nullptr;
    int32_t *b_order = nullptr, *hb_order = nullptr;
    int32_t *b_new = nullptr, *hb_new = nullptr;   // hb_*: host values
    BSeg *b_segs = nullptr;
    BCls *b_cls = nullptr;
    double *b_tpart = nullptr;
    int64_t nseg_max = 0;
    // parameter derivative over the final partition
    GParams *b_gtable = nullptr, *hb_gtable = nullptr;
    double *b_gpart = nullptr;
    double *b_git = nullptr, *hb_git = nullptr;
    // error histograms of threshold searches (one per slot; slot 0 serves
    // single-integral runs), zero between searches
    uint32_t *hcnt = nullptr;
    unsigned long long *hsum = nullptr;
    // the bound tables each search's histogram leaves (one pair per slot)
    double2 *htlo = nullptr, *hthi = nullptr;
    std::vector<hipEvent_t> events;
    std::string err;
    // live list left by the last pg_integrate
    int last_cur = 0, last_dim = 0;
    int64_t last_n = 0;
};

namespace {

constexpr size_t ALIGN = 256;
// Pinned staging copies of the slot header, used in turn (a copy is reused
// only after a stream synchronisation has passed since its last upload).
constexpr int INST_STAGES = 4;

// Offsets in the slot header of a run with K slots: slot table, order,
// new-slot list, search states. An upload copies the prefix up to the end
// of the last part it needs, in one copy.
constexpr size_t hdr_round(size_t x) { return (x + 255) / 256 * 256; }
struct HdrLayout {
    size_t order, nw, state, end_inst, end_order, end_new, end_state;
};
constexpr HdrLayout hdr_layout(size_t K) {
    HdrLayout h{};
    h.end_inst = sizeof(BInst) * K;
    h.order = hdr_round(h.end_inst);
    h.end_order = h.order + sizeof(int32_t) * K;
    h.nw = hdr_round(h.end_order);
    h.end_new = h.nw + sizeof(int32_t) * K;
    h.state = hdr_round(h.end_new);
    h.end_state = h.state + sizeof(SearchState) * K;
    return h;
}
constexpr size_t HDR_MAX = hdr_round(hdr_layout(BATCH_MAX_SLOTS).end_state);

struct Layout {
    size_t lo[2], w[2], V, E, Vp, K, A, A2;
    size_t pv, pe, pav, pae, pfv, pmin, pmax, pcnt, off;
    size_t inst[2], b_hdr, b_tot, b_table, b_segs,
        b_cls, b_tpart, b_gtable, b_gpart, b_git, hcnt, hsum, htlo, hthi;
    size_t search_part, dtot, dstate, total;
    int64_t nseg;
};

size_t bump(size_t &at, size_t bytes) {
    at = (at + ALIGN - 1) / ALIGN * ALIGN;
    const size_t r = at;
    at += bytes;
    return r;
}

Layout layout(int dim_max, int64_t cap) {
    Layout L{};
    size_t at = 0;
    const size_t list = sizeof(double) * (size_t)dim_max * (size_t)cap;
    for (int b = 0; b < 2; ++b) {
        L.lo[b] = bump(at, list);
        L.w[b] = bump(at, list);
    }
    L.V = bump(at, sizeof(double) * cap);
    L.E = bump(at, sizeof(double) * cap);
    L.Vp = bump(at, sizeof(double) * cap);
    L.K = bump(at, cap);
    L.A = bump(at, cap);
    L.A2 = bump(at, cap);
    // segments: single list <= 2 ceil(cap / SEG) + 2 (the many-integral
    // list's BSEG-long segments number fewer); many integrals add at
    // most two partial segments per slot
    L.nseg = 2 * ((cap + SEG - 1) / SEG) + 2 * BATCH_MAX_SLOTS + 2;
    L.pv = bump(at, sizeof(double) * L.nseg);
    L.pe = bump(at, sizeof(double) * L.nseg);
    L.pav = bump(at, sizeof(double) * L.nseg);
    L.pae = bump(at, sizeof(double) * L.nseg);
    L.pfv = bump(at, sizeof(double) * L.nseg);
    L.pmin = bump(at, sizeof(double) * L.nseg);
    L.pmax = bump(at, sizeof(double) * L.nseg);
    L.pcnt = bump(at, sizeof(uint32_t) * L.nseg);
    L.off = bump(at, sizeof(uint32_t) * L.nseg);
    L.search_part = bump(at, sizeof(double) * 2 * TRIAL_M * TRIAL_BLOCKS);
    for (int q = 0; q < 2; ++q) L.inst[q] = bump(at, sizeof(uint32_t) * cap);
    L.b_hdr = bump(at, HDR_MAX);
    L.b_tot = bump(at, sizeof(Totals) * BATCH_MAX_SLOTS);
    L.b_table = bump(at, sizeof(FParams) * BATCH_MAX_SLOTS);
    L.b_segs = bump(at, sizeof(BSeg) * L.nseg);
    L.b_cls = bump(at, sizeof(BCls) * L.nseg);
    L.b_tpart = bump(at, sizeof(double) * 2 * TRIAL_M * L.nseg);
    L.b_gtable = bump(at, sizeof(GParams) * BATCH_MAX_SLOTS);
    L.b_gpart = bump(at, sizeof(double) * GRAD_MAX * ADJ_SPLIT * L.nseg);
    L.b_git = bump(at, sizeof(double) * GRAD_MAX * BATCH_MAX_SLOTS);
    L.hcnt = bump(at, sizeof(uint32_t) * HIST_BINS * BATCH_MAX_SLOTS);
    L.hsum = bump(at, sizeof(unsigned long long) * HIST_BINS * BATCH_MAX_SLOTS);
    L.htlo = bump(at, sizeof(double2) * HIST_TAB * BATCH_MAX_SLOTS);
    L.hthi = bump(at, sizeof(double2) * HIST_TAB * BATCH_MAX_SLOTS);
    L.dtot = bump(at, sizeof(Totals));
    L.dstate = bump(at, sizeof(SearchState));
    L.total = (at + ALIGN - 1) / ALIGN * ALIGN;
    return L;
}

int fail(pg_context *ctx, int code, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));
int fail(pg_context *ctx, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIP_OR_FAIL(ctx, expr)                                                 \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(ctx, PG_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t npoints(int d) { return (int64_t(1) << d) + 2LL * d * d + 2LL * d + 1; }

// Rule constants of the degree-7 rule and its degree-5 embedded rule per
// orbit (weights relative to the box volume).
// The four null rules of the point set (error rule PG_ERR_NULL4). A fully
// symmetric rule u (one weight per orbit, m_o points each) vanishes on
// x^alpha iff <u, g_alpha> = 0, with <u, v> = sum_o m_o u_o v_o and
// g_alpha[o] the mean of x^alpha over orbit o; up to degree 5 only
// alpha = 0, x1^2, x1^4, x1^2 x2^2 matter. Degree 5: the one direction
// orthogonal to all four, which is w7 - w5. Degree 1: within span{g_0,
// g_x2}, orthogonal to g_0. Degree 3 (orthogonal to the degree-5 one):
// span{g_x4, g_x2y2} with span{g_0, g_x2} projected out, orthonormalised.
// Each is scaled to the norm of w7. Worked in long double from the exact
// rational weights and generator squares, then rounded once, so every
// weight is correct to about an ulp (in double, one pass loses up to 1e5
// ulps on the small vertex weights at d = 10).
void make_null_rules(int d, const double w7d[5], double nul[4][5]) {
    using LD = long double;
    const LD m[5] = {1.0L, 2.0L * d, 2.0L * d, 2.0L * d * (d - 1),
                     std::ldexp(1.0L, d)};
    const LD s2[5] = {0.0L, 9.0L / 70.0L, 9.0L / 10.0L, 9.0L / 10.0L,
                      9.0L / 19.0L};
    const LD D9 = 19683.0L;
    const LD w7[5] = {(12824.0L - 9120.0L * d + 400.0L * d * d) / D9,
                      980.0L / 6561.0L, (1820.0L - 400.0L * d) / D9,
                      200.0L / D9, 6859.0L / D9 / std::ldexp(1.0L, d)};
    const LD w5[5] = {(729.0L - 950.0L * d + 50.0L * d * d) / 729.0L,
                      245.0L / 486.0L, (265.0L - 100.0L * d) / 1458.0L,
                      25.0L / 729.0L, 0.0L};
    auto dot = [&](const LD *u, const LD *v) {
        LD s = 0.0L;
        for (int o = 0; o < 5; ++o) s += m[o] * u[o] * v[o];
        return s;
    };
    // subtract from u its component along a (a != 0)
    auto remove = [&](LD *u, const LD *a) {
        const LD c = dot(u, a) / dot(a, a);
        for (int o = 0; o < 5; ++o) u[o] -= c * a[o];
    };
    // the norm of the basic rule as the library evaluates it
    LD n7 = 0.0L;
    for (int o = 0; o < 5; ++o) n7 += m[o] * (LD)w7d[o] * (LD)w7d[o];
    n7 = std::sqrt(n7);
    auto scale_to = [&](LD *u) {
        const LD c = n7 / std::sqrt(dot(u, u));
        for (int o = 0; o < 5; ++o) u[o] *= c;
    };
    LD g0[5], a[5], b[5], c[5], e[5];
    for (int o = 0; o < 5; ++o) {
        // share of the orbit's points with a non-zero x1 (and x2)
        const LD on1 = o == 0 ? 0.0L : (o <= 2 ? 1.0L / d : (o == 3 ? 2.0L / d : 1.0L));
        const LD on12 = o == 3 ? 2.0L / (d * (d - 1.0L)) : (o == 4 ? 1.0L : 0.0L);
        g0[o] = 1.0L;
        a[o] = w7[o] - w5[o];
        e[o] = on1 * s2[o];
        b[o] = on1 * s2[o] * s2[o];
        c[o] = on12 * s2[o] * s2[o];
    }
    // each projection twice (the second pass removes what the first left
    // through rounding)
    for (int pass = 0; pass < 2; ++pass) remove(e, g0);       // degree 1
    for (int pass = 0; pass < 2; ++pass) {
        remove(b, g0);
        remove(b, e);
    }
    for (int pass = 0; pass < 2; ++pass) {                     // degree 3
        remove(c, g0);
        remove(c, e);
        remove(c, b);
    }
    scale_to(a);
    scale_to(b);
    scale_to(c);
    scale_to(e);
    for (int o = 0; o < 5; ++o) {
        nul[0][o] = (double)a[o];
        nul[1][o] = (double)b[o];
        nul[2][o] = (double)c[o];
        nul[3][o] = (double)e[o];
    }
}

Rule make_rule(int d, int err_rule) {
    Rule R{};
    const double D9 = 19683.0;
    R.lam2 = std::sqrt(9.0 / 70.0);
    R.lam3 = std::sqrt(9.0 / 10.0);
    R.lam4 = std::sqrt(9.0 / 10.0);
    R.lam5 = std::sqrt(9.0 / 19.0);
    const double w7[5] = {(12824.0 - 9120.0 * d + 400.0 * d * d) / D9,
                          980.0 / 6561.0, (1820.0 - 400.0 * d) / D9,
                          200.0 / D9, 6859.0 / D9 / std::ldexp(1.0, d)};
    const double w5[5] = {(729.0 - 950.0 * d + 50.0 * d * d) / 729.0,
                          245.0 / 486.0, (265.0 - 100.0 * d) / 1458.0,
                          25.0 / 729.0, 0.0};
    for (int k = 0; k < 5; ++k) {
        R.w7[k] = w7[k];
        R.wn[k] = w7[k] - w5[k];
    }
    R.err_rule = err_rule;
    if (err_rule == PG_ERR_NULL4) {
        // twice max(1, L_d), L_d = sup over directions a of the limit
        // (|a| -> 0) of the degree-7 error over r^2 e3 for exp(a.x):
        // 0.050, 0.354, 1.896, 7.038, 8.724, 10.17, 12.03, 14.28, 16.87
        static const double kappa[PG_DIM_MAX + 1] = {
            0.0, 0.0, 2.0, 2.0, 3.8, 15.0, 18.0, 21.0, 25.0, 29.0, 34.0};
        make_null_rules(d, w7, R.nul);
        R.kappa = kappa[d];
    }
    return R;
}

int make_params(pg_context *ctx, const pg_integrand *f, FParams *P) {
    if (!f || !f->params) return fail(ctx, PG_EINVAL, "integrand is NULL");
    const int d = f->dim;
    if (d < PG_DIM_MIN || d > PG_DIM_MAX)
        return fail(ctx, PG_EUNSUPPORTED, "dimension %d outside [%d, %d]", d,
                    PG_DIM_MIN, PG_DIM_MAX);
    if (d > ctx->dim_max)
        return fail(ctx, PG_EINVAL, "dimension %d above the context's %d", d,
                    ctx->dim_max);
    int need;
    switch (f->family) {
    case PG_PRODUCT_PEAK: case PG_GAUSSIAN: need = 2 * d; break;
    case PG_OSCILLATORY: need = d + 1; break;
    case PG_CORNER_PEAK: case PG_MONOMIAL: need = d; break;
    case PG_C0: case PG_DISCONTINUOUS: need = 2 * d; break;
    case PG_BOX: need = 1; break;
    default: return fail(ctx, PG_EUNSUPPORTED, "unknown family %d", f->family);
    }
    if (f->n_params != need)
        return fail(ctx, PG_EINVAL, "family %d in %d dimensions takes %d "
                    "parameters, got %d", f->family, d, need, f->n_params);
    if (!evaluate_supported(f->family, d))
        return fail(ctx, PG_EUNSUPPORTED, "family %d, d = %d not built",
                    f->family, d);
    std::memset(P, 0, sizeof *P);
    const double *p = f->params;
    for (int k = 0; k < need; ++k)
        if (!std::isfinite(p[k]))
            return fail(ctx, PG_EINVAL, "parameter %d is not finite", k);
    switch (f->family) {
    case PG_PRODUCT_PEAK:
        for (int k = 0; k < d; ++k) {
            if (p[k] == 0.0) return fail(ctx, PG_EINVAL, "a_%d = 0", k);
            P->p[k] = 1.0 / (p[k] * p[k]);
            P->p[d + k] = p[d + k];
        }
        break;
    case PG_GAUSSIAN:
        for (int k = 0; k < d; ++k) {
            P->p[k] = p[k] * p[k];
            P->p[d + k] = p[d + k];
        }
        break;
    case PG_OSCILLATORY:
        for (int k = 0; k < d; ++k) P->p[k] = p[k];
        P->p[d] = 2.0 * M_PI * p[d];
        break;
    case PG_C0: case PG_DISCONTINUOUS:
        for (int k = 0; k < 2 * d; ++k) P->p[k] = p[k];
        break;
    case PG_BOX: {
        const double q = p[0];
        if (q < 0) return fail(ctx, PG_EINVAL, "box power p = %g < 0", q);
        P->p[0] = q;
        if (q <= 64 && q == std::floor(q)) {
            P->p[1] = 0.0;
            P->p[2] = q;
        } else if (q <= 64 && 2 * q == std::floor(2 * q)) {
            P->p[1] = 1.0;
            P->p[2] = std::floor(q);
        } else {
            P->p[1] = 2.0;
        }
        break;
    }
    default:
        for (int k = 0; k < d; ++k) P->p[k] = p[k];
        if (f->family == PG_MONOMIAL)
            for (int k = 0; k < d; ++k)
                if (p[k] < 0 || p[k] != std::floor(p[k]) || p[k] > 64)
                    return fail(ctx, PG_EINVAL, "alpha_%d must be an integer "
                                "in [0, 64]", k);
        break;
    }
    return PG_OK;
}

// Parameters of the derivative kernels (layout: see pg_adjoint.hip). The
// values were validated by make_params.
void make_gparams(int family, int d, const double *p, GParams *G) {
    std::memset(G, 0, sizeof *G);
    switch (family) {
    case PG_PRODUCT_PEAK:
        for (int k = 0; k < d; ++k) {
            G->p[k] = 1.0 / (p[k] * p[k]);
            G->p[d + k] = p[d + k];
            G->gs[k] = 2.0 / (p[k] * p[k] * p[k]);
            G->gs[d + k] = 2.0;
        }
        break;
    case PG_GAUSSIAN:
        for (int k = 0; k < d; ++k) {
            G->p[k] = p[k];
            G->p[d + k] = p[d + k];
            G->gs[k] = -2.0 * p[k];
            G->gs[d + k] = 2.0 * p[k] * p[k];
        }
        break;
    case PG_OSCILLATORY:
        for (int k = 0; k < d; ++k) {
            G->p[k] = p[k];
            G->gs[k] = -1.0;
        }
        G->p[d] = 2.0 * M_PI * p[d];
        G->gs[d] = -2.0 * M_PI;
        break;
    default:
        for (int k = 0; k < d; ++k) {
            G->p[k] = p[k];
            G->gs[k] = -(double)(d + 1);
        }
        break;
    }
}

// Waves per evaluation block: enough blocks x waves to reach `target`
// waves, at most the number of work units allows.
int eval_waves(int d, int64_t n, int64_t target) {
    const int64_t blocks = (n + 63) / 64;
    int w = 1;
    const int wmax = evaluate_max_waves(d);
    while (w < wmax && blocks * w < target) w *= 2;
    return w;
}

int sync_tot(pg_context *ctx, Totals *out) {
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->htot, ctx->dtot, sizeof(Totals),
                                    hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    *out = *ctx->htot;
    return PG_OK;
}

// Sequence number for the next reduce that publishes to the host.
uint64_t next_seq(pg_context *ctx) { return ++ctx->seq; }

// Longest a host wait for one reduce's totals may take. Everything queued
// before that reduce (one iteration's kernels, or a batch of search passes)
// takes milliseconds even on the longest lists, so a wait this long means
// the stream is stuck behind other work or a kernel that does not end.
constexpr double WAIT_LIMIT_S = 300.0;

// Wait until the reduce tagged `seq` has published its values to the mapped
// host copies: spin on the sequence word; every 1024 polls ask the stream
// whether it has stopped (then the word must be there, else the kernel
// failed) or has failed, and give up with PG_EHIP after WAIT_LIMIT_S.
int wait_seq(pg_context *ctx, uint64_t seq) {
    const volatile uint64_t *word = ctx->hseq;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 1;; ++k) {
        if (*word == seq) break;
        if ((k & 1023) == 0) {
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e == hipSuccess) {
                if (*word == seq) break;
                return fail(ctx, PG_EHIP, "stream idle before the totals "
                            "of reduce %llu arrived", (unsigned long long)seq);
            }
            if (e != hipErrorNotReady)
                return fail(ctx, PG_EHIP, "stream failed: %s",
                            hipGetErrorString(e));
            const std::chrono::duration<double> dt =
                std::chrono::steady_clock::now() - t0;
            if (dt.count() > WAIT_LIMIT_S)
                return fail(ctx, PG_EHIP, "no totals of reduce %llu after %.0f s",
                            (unsigned long long)seq, dt.count());
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PG_OK;
}

// The totals of the reduce tagged `seq` (launched with host_tot =
// ctx->htot_dev and host_seq = ctx->hseq_dev).
int wait_tot(pg_context *ctx, uint64_t seq, Totals *out) {
    int rc = wait_seq(ctx, seq);
    if (rc) return rc;
    *out = *ctx->htot;
    return PG_OK;
}

// THRESHOLD-CLASSIFY (Algorithm 3) on the list (E, A_rel) of n regions; its
// state lives on the device (see k_trial_walk). Passes are queued in
// batches of 3, 5 and 8 (most searches end in the first) and the host
// waits once per batch; passes after the search has ended return at once.
// With `count`, the count pass of the accepted threshold (segment counts,
// offsets and sums of the surviving regions, into ctx->dtot) is queued
// behind each batch, so the same wait also delivers the compaction's
// inputs.
constexpr int SEARCH_BATCHES[3] = {3, 5, 8};

struct SearchOut {
    int ok = 0, trials = 0;
    double t = -HUGE_VAL;
};

struct CountReq {
    int paired;
    const double *V;
    Totals *tot;     // host copy of the count totals (when ok)
};

int search(pg_context *ctx, int64_t n, const double *E, const uint8_t *A_rel,
           double e_it, double allowance, int relax, const CountReq *count,
           SearchOut *out) {
    const int max_passes = (THR_MAX_TRIALS + TRIAL_DEPTH - 1) / TRIAL_DEPTH;
    hipStream_t st = ctx->stream;
    *out = SearchOut{};
    // min / max E were left in ctx->dtot by the pass that preceded the call;
    // most trials are decided from the error histogram, exact passes take
    // over from the first one it leaves open
    HIP_OR_FAIL(ctx, launch_search_hist(st, n, E, A_rel, ctx->dstate,
                                        ctx->hcnt, ctx->hsum, ctx->htlo,
                                        ctx->hthi, e_it, allowance, relax,
                                        ctx->dtot));
    int passes = 0;
    for (int bi = -1; bi < 3 && passes < max_passes; ++bi) {
        const int batch =
            bi < 0 ? 0 : std::min(SEARCH_BATCHES[bi], max_passes - passes);
        for (int k = 0; k < batch; ++k)
            HIP_OR_FAIL(ctx, launch_search_pass(st, n, E, A_rel, ctx->dstate,
                                                ctx->search_part, ctx->htlo,
                                                ctx->hthi));
        passes += batch;
        if (count) {
            HIP_OR_FAIL(ctx, launch_seg_count(st, n, count->paired, 0.0,
                                              count->V, E, A_rel, ctx->dstate,
                                              ctx->part));
            // the totals and the search state go straight to the host
            const uint64_t sq = next_seq(ctx);
            HIP_OR_FAIL(ctx, launch_reduce_scan(st, seg_count(n, count->paired),
                                                ctx->part, ctx->off,
                                                ctx->dtot, ctx->htot_dev,
                                                ctx->dstate, ctx->hstate_dev,
                                                ctx->hseq_dev, sq));
            const int rc = wait_seq(ctx, sq);
            if (rc) return rc;
        } else {
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->hstate, ctx->dstate,
                                            sizeof(SearchState),
                                            hipMemcpyDeviceToHost, st));
            HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        }
        if (ctx->hstate->done) break;
    }
    const SearchState &S = *ctx->hstate;
    out->ok = S.done && S.ok;
    out->t = out->ok ? S.t_acc : -HUGE_VAL;
    out->trials = S.trials;
    if (count && out->ok) *count->tot = *ctx->htot;
    return PG_OK;
}

int validate_list(pg_context *ctx, int64_t n, int64_t ld) {
    if (n < 0) return fail(ctx, PG_EINVAL, "n = %lld < 0", (long long)n);
    if (ld < n) return fail(ctx, PG_EINVAL, "ld %lld < n %lld", (long long)ld,
                            (long long)n);
    if (n > ctx->cap)
        return fail(ctx, PG_ENOMEM, "n = %lld above the context capacity %lld",
                    (long long)n, (long long)ctx->cap);
    return PG_OK;
}

// Whether a threshold search relaxes P_max at its direction changes
// (Section 3.5.3 relaxes it in every search; the memory-only option only in
// searches triggered because the list would overflow its cap).
int relax_pmax(const pg_options &o, bool memory_trigger) {
    return o.pmax_relax == PG_PMAX_EVERY_CHANGE || memory_trigger ? 1 : 0;
}

// The error the regions a threshold search finishes may carry (the
// allowance of its accuracy requirement; v_f, e_f: the estimate and error
// of the regions finished in earlier iterations; fv: the summed V of the
// regions the relative-error test finishes in this one). The listing's
// e_it - e_b = tau |v_tot| - e_f; under PG_BUDGET_RESERVE, a search started
// because the estimate's digits have settled lets the finished regions
// carry only tau times their own estimate, tau |v_f + fv| - e_f: by Lemma 1
// the regions left active may still end with tau |V| each, and Section
// 3.5.2 asks such a search not to over-commit finished error. A search run
// because the list would overflow has the listing's allowance (continuing
// is then the only way on).
double search_allowance(const pg_options &o, bool memory_trigger, double tau,
                        double v_tot, double v_f, double e_f, double fv) {
    if (o.budget == PG_BUDGET_RESERVE && !memory_trigger)
        return tau * std::fabs(v_f + fv) - e_f;
    return tau * std::fabs(v_tot) - e_f;
}

// Option checks shared by the single and the batched drivers.
int check_rules(pg_context *ctx, const pg_options &o) {
    if (o.error_rule != PG_ERR_RAW && o.error_rule != PG_ERR_NULL4)
        return fail(ctx, PG_EINVAL, "unknown error rule %d", o.error_rule);
    if (o.pmax_relax != PG_PMAX_EVERY_CHANGE &&
        o.pmax_relax != PG_PMAX_UNDER_MEMORY)
        return fail(ctx, PG_EINVAL, "unknown P_max rule %d", o.pmax_relax);
    if (o.budget != PG_BUDGET_RESERVE && o.budget != PG_BUDGET_LISTING)
        return fail(ctx, PG_EINVAL, "unknown search budget %d", o.budget);
    return PG_OK;
}

struct TraceRec {
    int64_t it, n, n_active;
    int32_t thr_invoked, thr_ok, thr_trials, terminal;
    double t, v, e, v_f, e_f;
};

}  // namespace

extern "C" {

void pg_default_options(pg_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->rel_tol = 1e-3;
    opt->abs_tol = 1e-20;
    opt->init_splits = 4;
    opt->max_iters = 100;
    opt->relerr_filter = 1;
    opt->threshold_filter = 1;
}

size_t pg_workspace_bytes(int dim_max, int64_t capacity) {
    if (dim_max < PG_DIM_MIN || dim_max > PG_DIM_MAX || capacity < 2) return 0;
    return layout(dim_max, capacity).total;
}

int pg_context_create(int device, int dim_max, int64_t capacity,
                      void *workspace, size_t ws_bytes, void *stream,
                      pg_context **out) {
    if (!out) return PG_EINVAL;
    *out = nullptr;
    if (dim_max < PG_DIM_MIN || dim_max > PG_DIM_MAX) return PG_EINVAL;
    if (capacity < 2 || capacity > (int64_t(1) << 31)) return PG_EINVAL;
    const Layout L = layout(dim_max, capacity);
    if (workspace && ws_bytes < L.total) return PG_ENOMEM;
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % ALIGN))
        return PG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PG_EHIP;
    pg_context *ctx = new pg_context();
    ctx->device = device;
    ctx->dim_max = dim_max;
    ctx->cap = capacity;
    if (workspace) {
        ctx->ws = workspace;
        ctx->ws_bytes = ws_bytes;
    } else {
        if (hipMalloc(&ctx->ws, L.total) != hipSuccess) {
            delete ctx;
            return PG_ENOMEM;
        }
        ctx->ws_bytes = L.total;
        ctx->own_ws = true;
    }
    ctx->stream = (hipStream_t)stream;      // NULL: the null stream
    if (hipHostMalloc((void **)&ctx->htot, sizeof(Totals),
                      hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hstate, sizeof(SearchState),
                      hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->htot_dev, ctx->htot, 0) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->hstate_dev, ctx->hstate, 0) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hseq, 64,
                      hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->hseq_dev, ctx->hseq, 0) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_hdr, HDR_MAX * INST_STAGES, 0) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_gtable,
                      sizeof(GParams) * BATCH_MAX_SLOTS, 0) != hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_git,
                      sizeof(double) * GRAD_MAX * BATCH_MAX_SLOTS, 0) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_state,
                      sizeof(SearchState) * BATCH_MAX_SLOTS, 0) != hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_tot, sizeof(Totals) * BATCH_MAX_SLOTS,
                      hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->hb_tot_dev, ctx->hb_tot, 0) !=
            hipSuccess ||
        hipHostMalloc((void **)&ctx->hb_table,
                      sizeof(FParams) * BATCH_MAX_SLOTS, 0) != hipSuccess ||
        !(ctx->hb_order = new (std::nothrow) int32_t[BATCH_MAX_SLOTS]) ||
        !(ctx->hb_new = new (std::nothrow) int32_t[BATCH_MAX_SLOTS])) {
        pg_context_destroy(ctx);
        return PG_ENOMEM;
    }
    *ctx->hseq = 0;
    char *b = (char *)ctx->ws;
    for (int q = 0; q < 2; ++q) {
        ctx->lo[q] = (double *)(b + L.lo[q]);
        ctx->w[q] = (double *)(b + L.w[q]);
    }
    ctx->V = (double *)(b + L.V);
    ctx->E = (double *)(b + L.E);
    ctx->Vp = (double *)(b + L.Vp);
    ctx->K = (uint8_t *)(b + L.K);
    ctx->A = (uint8_t *)(b + L.A);
    ctx->A2 = (uint8_t *)(b + L.A2);
    ctx->part.v = (double *)(b + L.pv);
    ctx->part.e = (double *)(b + L.pe);
    ctx->part.av = (double *)(b + L.pav);
    ctx->part.ae = (double *)(b + L.pae);
    ctx->part.fv = (double *)(b + L.pfv);
    ctx->part.emin = (double *)(b + L.pmin);
    ctx->part.emax = (double *)(b + L.pmax);
    ctx->part.cnt = (uint32_t *)(b + L.pcnt);
    ctx->off = (uint32_t *)(b + L.off);
    ctx->search_part = (double *)(b + L.search_part);
    for (int q = 0; q < 2; ++q) ctx->inst[q] = (uint32_t *)(b + L.inst[q]);
    ctx->b_hdr = b + L.b_hdr;
    ctx->b_tot = (Totals *)(b + L.b_tot);
    ctx->b_table = (FParams *)(b + L.b_table);
    ctx->b_segs = (BSeg *)(b + L.b_segs);
    ctx->b_cls = (BCls *)(b + L.b_cls);
    ctx->b_tpart = (double *)(b + L.b_tpart);
    ctx->b_gtable = (GParams *)(b + L.b_gtable);
    ctx->b_gpart = (double *)(b + L.b_gpart);
    ctx->b_git = (double *)(b + L.b_git);
    ctx->hcnt = (uint32_t *)(b + L.hcnt);
    ctx->hsum = (unsigned long long *)(b + L.hsum);
    ctx->htlo = (double2 *)(b + L.htlo);
    ctx->hthi = (double2 *)(b + L.hthi);
    if (hipMemset(ctx->hcnt, 0, L.hsum + sizeof(unsigned long long) * HIST_BINS *
                                         BATCH_MAX_SLOTS - L.hcnt) != hipSuccess) {
        pg_context_destroy(ctx);
        return PG_EHIP;
    }
    ctx->nseg_max = L.nseg;
    ctx->dtot = (Totals *)(b + L.dtot);
    ctx->dstate = (SearchState *)(b + L.dstate);
    *out = ctx;
    return PG_OK;
}

void pg_context_destroy(pg_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->htot) (void)hipHostFree(ctx->htot);
    if (ctx->hstate) (void)hipHostFree(ctx->hstate);
    if (ctx->hseq) (void)hipHostFree(ctx->hseq);
    void *pinned[] = {ctx->hb_hdr, ctx->hb_state, ctx->hb_tot, ctx->hb_table,
                      ctx->hb_gtable, ctx->hb_git};
    for (void *q : pinned)
        if (q) (void)hipHostFree(q);
    delete[] ctx->hb_order;
    delete[] ctx->hb_new;
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    delete ctx;
}

int pg_context_set_stream(pg_context *ctx, void *stream) {
    if (!ctx) return PG_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return PG_OK;
}

int pg_context_set_eval_waves(pg_context *ctx, int target) {
    if (!ctx) return PG_EINVAL;
    if (target == 0) target = (int)EVAL_WAVE_TARGET;
    if (target < 256 || target > 65536)
        return fail(ctx, PG_EINVAL, "wave target %d outside 256..65536", target);
    ctx->wave_target = target;
    return PG_OK;
}

const char *pg_last_error(const pg_context *ctx) {
    return ctx ? ctx->err.c_str() : "no context";
}

int pg_evaluate(pg_context *ctx, const pg_integrand *f, int64_t n,
                const double *lo, const double *w, int64_t ld, double *V,
                double *E, uint8_t *K) {
    return pg_evaluate_rule(ctx, f, PG_ERR_RAW, n, lo, w, ld, V, E, K);
}

int pg_evaluate_rule(pg_context *ctx, const pg_integrand *f, int error_rule,
                     int64_t n, const double *lo, const double *w, int64_t ld,
                     double *V, double *E, uint8_t *K) {
    if (!ctx) return PG_EINVAL;
    if (error_rule != PG_ERR_RAW && error_rule != PG_ERR_NULL4)
        return fail(ctx, PG_EINVAL, "unknown error rule %d", error_rule);
    FParams P;
    int rc = make_params(ctx, f, &P);
    if (rc) return rc;
    if (ld < n || n < 0) return fail(ctx, PG_EINVAL, "bad n / ld");
    if (n == 0) return PG_OK;
    if (!lo || !w || !V || !E || !K)
        return fail(ctx, PG_EINVAL, "NULL array");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    const Rule R = make_rule(f->dim, error_rule);
    HIP_OR_FAIL(ctx, launch_evaluate(ctx->stream, f->family, f->dim, P, R, n,
                                     lo, w, ld, V, E, K,
                                     eval_waves(f->dim, n, ctx->wave_target)));
    return PG_OK;
}

int pg_integrand_values(pg_context *ctx, const pg_integrand *f, int64_t n,
                        const double *x, int64_t ld, double *y) {
    if (!ctx) return PG_EINVAL;
    FParams P;
    int rc = make_params(ctx, f, &P);
    if (rc) return rc;
    if (ld < n || n < 0) return fail(ctx, PG_EINVAL, "bad n / ld");
    if (n == 0) return PG_OK;
    if (!x || !y) return fail(ctx, PG_EINVAL, "NULL array");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, launch_fvalues(ctx->stream, f->family, f->dim, P, n, x,
                                    ld, y));
    return PG_OK;
}

int pg_classify(pg_context *ctx, int64_t n, int paired, const double *V,
                double *E, const double *Vp, double rel_tol,
                int relerr_filter, uint8_t *A, double *sums) {
    if (!ctx) return PG_EINVAL;
    int rc = validate_list(ctx, n, n);
    if (rc) return rc;
    if (paired && (n % 2)) return fail(ctx, PG_EINVAL, "paired list of odd n");
    if (!V || !E || !A || !sums || (paired && !Vp))
        return fail(ctx, PG_EINVAL, "NULL array");
    if (n == 0) {
        for (int k = 0; k < 8; ++k) sums[k] = 0.0;
        sums[5] = HUGE_VAL;
        sums[6] = -HUGE_VAL;
        return PG_OK;
    }
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, launch_classify(ctx->stream, n, paired ? 1 : 0, V, E, Vp,
                                     rel_tol, relerr_filter, A, ctx->part));
    HIP_OR_FAIL(ctx, launch_reduce_scan(ctx->stream, seg_count(n, paired),
                                        ctx->part, ctx->off, ctx->dtot));
    Totals T;
    rc = sync_tot(ctx, &T);
    if (rc) return rc;
    sums[0] = T.v; sums[1] = T.e; sums[2] = T.av; sums[3] = T.ae;
    sums[4] = T.cnt; sums[5] = T.emin; sums[6] = T.emax; sums[7] = T.fv;
    return PG_OK;
}

int pg_threshold_search(pg_context *ctx, int64_t n, const double *E,
                        const uint8_t *A_rel, double e_it, double allowance,
                        int relax, uint8_t *A_out, int *ok, double *t,
                        int *trials) {
    if (!ctx) return PG_EINVAL;
    if (!std::isfinite(allowance) || !std::isfinite(e_it))
        return fail(ctx, PG_EINVAL, "e_it %g or allowance %g not finite", e_it,
                    allowance);
    int rc = validate_list(ctx, n, n);
    if (rc) return rc;
    if (n == 0 || !E || !A_rel || !A_out || !ok || !t || !trials)
        return fail(ctx, PG_EINVAL, "empty list or NULL argument");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    // min / max of E over the whole list (the count pass over E records them)
    HIP_OR_FAIL(ctx, launch_seg_count(ctx->stream, n, 0, -HUGE_VAL, E, E,
                                      A_rel, nullptr, ctx->part));
    HIP_OR_FAIL(ctx, launch_reduce_scan(ctx->stream, seg_count(n, 0),
                                        ctx->part, ctx->off, ctx->dtot));
    SearchOut so;
    rc = search(ctx, n, E, A_rel, e_it, allowance, relax ? 1 : 0, nullptr, &so);
    if (rc) return rc;
    *ok = so.ok;
    *t = so.ok ? so.t : NAN;
    *trials = so.trials;
    HIP_OR_FAIL(ctx, launch_apply_threshold(ctx->stream, n,
                                            so.ok ? so.t : -HUGE_VAL, A_rel,
                                            E, A_out));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return PG_OK;
}

int pg_filter_split(pg_context *ctx, int dim, int64_t n, const double *lo,
                    const double *w, int64_t ld_in, const uint8_t *K,
                    const double *V, const uint8_t *A, double *lo_out,
                    double *w_out, int64_t ld_out, double *Vp,
                    int64_t *n_active) {
    if (!ctx) return PG_EINVAL;
    if (dim < PG_DIM_MIN || dim > PG_DIM_MAX)
        return fail(ctx, PG_EINVAL, "dimension %d", dim);
    int rc = validate_list(ctx, n, ld_in);
    if (rc) return rc;
    if (!n_active) return fail(ctx, PG_EINVAL, "n_active is NULL");
    *n_active = 0;
    if (n == 0) return PG_OK;
    if (!lo || !w || !K || !V || !A || !lo_out || !w_out || !Vp)
        return fail(ctx, PG_EINVAL, "NULL array");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, launch_seg_count(ctx->stream, n, 0, 0.0, V, nullptr, A,
                                      nullptr, ctx->part));
    HIP_OR_FAIL(ctx, launch_reduce_scan(ctx->stream, seg_count(n, 0),
                                        ctx->part, ctx->off, ctx->dtot));
    Totals T;
    rc = sync_tot(ctx, &T);
    if (rc) return rc;
    const int64_t na = (int64_t)T.cnt;
    if (ld_out < 2 * na)
        return fail(ctx, PG_EINVAL, "ld_out %lld < 2 n_active %lld",
                    (long long)ld_out, (long long)(2 * na));
    HIP_OR_FAIL(ctx, launch_compact_split(ctx->stream, dim, n, 0, 0.0, A,
                                          nullptr, V, K, lo, w, ld_in,
                                          ctx->off, na, lo_out, w_out, ld_out,
                                          Vp));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    *n_active = na;
    return PG_OK;
}

int pg_last_regions(const pg_context *ctx, pg_regions_view *out) {
    if (!ctx || !out) return PG_EINVAL;
    out->dim = ctx->last_dim;
    out->n = ctx->last_n;
    out->ld = ctx->cap;
    out->lo = ctx->lo[ctx->last_cur];
    out->w = ctx->w[ctx->last_cur];
    out->V = ctx->V;
    out->E = ctx->E;
    out->K = ctx->K;
    out->A = ctx->A;
    return PG_OK;
}

int pg_integrate(pg_context *ctx, const pg_integrand *f, const double *lo,
                 const double *hi, const pg_options *opt, pg_result *out) {
    if (!ctx) return PG_EINVAL;
    pg_result res;
    std::memset(&res, 0, sizeof res);
    res.estimate = NAN;
    res.error = NAN;
    if (out) *out = res;
    ctx->err.clear();
    pg_options o;
    if (opt) o = *opt;
    else pg_default_options(&o);
    FParams P;
    int rc = make_params(ctx, f, &P);
    if (rc) return rc;
    const int d = f->dim;
    if (!lo || !hi) return fail(ctx, PG_EINVAL, "bounds are NULL");
    for (int k = 0; k < d; ++k)
        if (!(lo[k] < hi[k]) || !std::isfinite(lo[k]) || !std::isfinite(hi[k]))
            return fail(ctx, PG_EINVAL, "empty or infinite range on axis %d", k);
    if (!(o.rel_tol > 0.0) && !(o.abs_tol > 0.0))
        return fail(ctx, PG_EINVAL, "no positive tolerance");
    if (o.init_splits < 1) return fail(ctx, PG_EINVAL, "init_splits < 1");
    if (o.max_iters < 1) return fail(ctx, PG_EINVAL, "max_iters < 1");
    if (int rc_rules = check_rules(ctx, o)) return rc_rules;
    const int64_t cap = o.max_regions > 0 ? o.max_regions : ctx->cap;
    if (cap > ctx->cap)
        return fail(ctx, PG_ENOMEM, "max_regions %lld above the capacity %lld",
                    (long long)cap, (long long)ctx->cap);
    int64_t n = 1;
    for (int k = 0; k < d; ++k) {
        n *= o.init_splits;
        if (n > cap)
            return fail(ctx, PG_EINVAL, "initial grid %d^%d above the cap %lld",
                        o.init_splits, d, (long long)cap);
    }
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    const Rule R = make_rule(d, o.error_rule);
    const double tau = o.rel_tol;
    const int64_t ld = ctx->cap;
    hipStream_t st = ctx->stream;

    FILE *tr = nullptr;
    std::vector<uint8_t> hK, hA;
    std::vector<double> hE;
    if (o.trace_path) {
        tr = std::fopen(o.trace_path, "wb");
        if (!tr) return fail(ctx, PG_EINVAL, "cannot open %s", o.trace_path);
        const char magic[8] = {'P', 'G', 'T', 'R', 'A', 'C', 'E', '2'};
        const int32_t hd[2] = {d, f->family};
        // the run's rules, which a replay must share
        const int64_t rules[3] = {o.pmax_relax, o.error_rule, o.budget};
        std::fwrite(magic, 1, 8, tr);
        std::fwrite(hd, 4, 2, tr);
        std::fwrite(rules, 8, 3, tr);
    }
    // timing events: 5 per iteration (level 1 records only the two around
    // EVALUATE, level 2 all five)
    const int timing = o.timing < 0 ? 0 : o.timing;
    if (timing) {
        const size_t need = 5 * (size_t)o.max_iters;
        while (ctx->events.size() < need) {
            hipEvent_t e;
            // timing only: no system-scope fence (and so no cache write-back)
            // when an event is recorded; the times are read after the
            // run's final stream synchronisation
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) !=
                hipSuccess) {
                if (tr) std::fclose(tr);
                return fail(ctx, PG_EHIP, "hipEventCreate failed");
            }
            ctx->events.push_back(e);
        }
    }
#define RUN_FAIL(expr)                                                         \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            if (tr) std::fclose(tr);                                           \
            return fail(ctx, PG_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
        }                                                                      \
    } while (0)
#define RUN_RC(expr)                                                           \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_) {                                                             \
            if (tr) std::fclose(tr);                                           \
            return rc_;                                                        \
        }                                                                      \
    } while (0)

    {
        double a[PG_DIM_MAX], width[PG_DIM_MAX];
        for (int k = 0; k < d; ++k) {
            a[k] = lo[k];
            width[k] = (hi[k] - lo[k]) / (double)o.init_splits;
        }
        RUN_FAIL(launch_init(st, d, o.init_splits, a, width, ctx->lo[0],
                             ctx->w[0], ld));
    }
    int cur = 0;
    double v_f = 0.0, e_f = 0.0, v_tot = 0.0, e_tot = 0.0, prev_vtot = NAN;
    int status = PG_MAX_ITERS;
    int it;
    res.peak_regions = n;
    int nev = 0;
    for (it = 1; it <= o.max_iters; ++it) {
        const int paired = it > 1;
        hipEvent_t *ev = timing ? &ctx->events[5 * (it - 1)] : nullptr;
        if (timing) RUN_FAIL(hipEventRecord(ev[0], st));
        RUN_FAIL(launch_evaluate(st, f->family, d, P, R, n, ctx->lo[cur],
                                 ctx->w[cur], ld, ctx->V, ctx->E, ctx->K,
                                 eval_waves(d, n, ctx->wave_target)));
        ++nev;
        if (timing) RUN_FAIL(hipEventRecord(ev[1], st));
        res.regions_evaluated += n;
        RUN_FAIL(launch_classify(st, n, paired, ctx->V, ctx->E, ctx->Vp, tau,
                                 o.relerr_filter, ctx->A, ctx->part));
        const int64_t nseg = seg_count(n, paired);
        const uint64_t sq = next_seq(ctx);
        RUN_FAIL(launch_reduce_scan(st, nseg, ctx->part, ctx->off, ctx->dtot,
                                    ctx->htot_dev, nullptr, nullptr,
                                    ctx->hseq_dev, sq));
        if (timing > 1) RUN_FAIL(hipEventRecord(ev[2], st));
        Totals T;
        RUN_RC(wait_tot(ctx, sq, &T));
        const double v = T.v, e = T.e;
        v_tot = v + v_f;
        e_tot = e + e_f;
        TraceRec rec{};
        rec.it = it;
        rec.n = n;
        rec.terminal = -1;
        rec.t = NAN;
        rec.v = v;
        rec.e = e;
        rec.v_f = v_f;
        rec.e_f = e_f;
        const bool terminated =
            (e_tot <= tau * std::fabs(v_tot)) || (e_tot <= o.abs_tol);
        double av = T.av, ae = T.ae;
        int64_t n_act = (int64_t)T.cnt;
        const int64_t n_rel = n_act;
        SearchOut so;
        if (terminated) {
            status = PG_OK;
            rec.terminal = PG_OK;
        } else {
            const bool trig_a = o.threshold_filter && it >= 2 &&
                                std::fabs(v_tot - prev_vtot) <=
                                    tau * std::fabs(v_tot);
            const bool trig_b = o.threshold_filter && 2 * n_rel > cap;
            if (trig_a || trig_b) {
                ++res.threshold_calls;
                rec.thr_invoked = 1;
                Totals T2;
                const CountReq cr{paired, ctx->V, &T2};
                RUN_RC(search(ctx, n, ctx->E, ctx->A, e,
                              search_allowance(o, trig_b, tau, v_tot, v_f, e_f,
                                               T.fv),
                              relax_pmax(o, trig_b), &cr, &so));
                res.threshold_trials += so.trials;
                rec.thr_ok = so.ok;
                rec.thr_trials = so.trials;
                if (so.ok) {
                    rec.t = so.t;
                    av = T2.av;
                    ae = T2.ae;
                    n_act = (int64_t)T2.cnt;
                }
                // after a failed search the queued count pass recounted
                // A_rel, so the segment offsets equal the classify pass's
            }
            if (!so.ok && 2 * n_rel > cap) {
                status = PG_MEMORY_EXHAUSTED;
                rec.terminal = status;
            }
        }
        if (timing > 1) RUN_FAIL(hipEventRecord(ev[3], st));
        if (rec.terminal < 0) {
            prev_vtot = v_tot;
            if (n_act == 0) {
                status = PG_NO_ACTIVE;
                rec.terminal = status;
            } else if (it == o.max_iters) {
                status = PG_MAX_ITERS;
                rec.terminal = status;
            }
        }
        rec.n_active = rec.terminal == PG_OK ? n_rel : n_act;
        if (tr) {
            hK.resize(n);
            hA.resize(n);
            RUN_FAIL(hipMemcpyAsync(hK.data(), ctx->K, n, hipMemcpyDeviceToHost, st));
            RUN_FAIL(hipMemcpyAsync(hA.data(), ctx->A, n, hipMemcpyDeviceToHost, st));
            if (so.ok) {
                hE.resize(n);
                RUN_FAIL(hipMemcpyAsync(hE.data(), ctx->E, n * sizeof(double),
                                        hipMemcpyDeviceToHost, st));
            }
            RUN_FAIL(hipStreamSynchronize(st));
            if (so.ok)
                for (int64_t i = 0; i < n; ++i)
                    hA[i] = (uint8_t)(hA[i] && hE[i] > so.t);
            std::fwrite(&rec, sizeof rec, 1, tr);
            std::fwrite(hK.data(), 1, n, tr);
            std::fwrite(hA.data(), 1, n, tr);
        }
        if (rec.terminal >= 0) {
            if (timing > 1) RUN_FAIL(hipEventRecord(ev[4], st));
            break;
        }
        v_f = v - av + v_f;
        e_f = e - ae + e_f;
        RUN_FAIL(launch_compact_split(st, d, n, paired, so.ok ? so.t : 0.0,
                                      ctx->A, so.ok ? ctx->E : nullptr, ctx->V,
                                      ctx->K, ctx->lo[cur], ctx->w[cur], ld,
                                      ctx->off, n_act, ctx->lo[1 - cur],
                                      ctx->w[1 - cur], ld, ctx->Vp));
        if (timing > 1) RUN_FAIL(hipEventRecord(ev[4], st));
        cur = 1 - cur;
        n = 2 * n_act;
        res.peak_regions = std::max<int64_t>(res.peak_regions, n);
    }
    if (it > o.max_iters) it = o.max_iters;
    RUN_FAIL(hipStreamSynchronize(st));
    if (tr) std::fclose(tr);
    tr = nullptr;
    if (timing) {
        // the stream has drained, but a trailing marker can still be
        // reported as pending for a moment: wait for the last event itself
        (void)hipEventSynchronize(
            ctx->events[5 * (it - 1) + (timing > 1 ? 4 : 1)]);
        for (int q = 0; q < it; ++q) {
            hipEvent_t *ev = &ctx->events[5 * q];
            float ms;
            for (int ph = 0; ph < (timing > 1 ? 4 : 1); ++ph) {
                if (hipEventElapsedTime(&ms, ev[ph], ev[ph + 1]) == hipSuccess)
                    res.phase_ms[ph] += ms;
            }
        }
    }
    ctx->last_cur = cur;
    ctx->last_n = n;
    ctx->last_dim = d;
    res.estimate = v_tot;
    res.error = e_tot;
    res.status = status;
    res.iterations = it;
    res.fevals = res.regions_evaluated * npoints(d);
    res.eval_launches = nev;
    if (out) *out = res;
    return status;
#undef RUN_FAIL
#undef RUN_RC
}


// Many integrals of one family in one region list (see pg_batch.hip): each
// live integral runs exactly the iteration of pg_integrate, with its own
// tolerance, cap and state; they share every kernel launch. At most
// min(B, capacity / cap, BATCH_MAX_SLOTS) integrals are live at once (each
// may grow to `cap` regions); the others start as slots free up.
// With grad, each iteration also adds the parameter derivative of the rule
// values of the regions that leave the list for good (the leaves of the
// final partition, see pg_adjoint.hip); with leaves, those are copied out.
static int run_batch(pg_context *ctx, int family, int dim, int B,
                     const double *params, int n_params, const double *lo,
                     const double *hi, const double *rel_tol,
                     const double *abs_tol, const pg_options *opt,
                     pg_result *out, double *grad, pg_leaves *leaves) {
    if (!ctx) return PG_EINVAL;
    ctx->err.clear();
    if (B < 1 || !params || !rel_tol || !out || !lo || !hi)
        return fail(ctx, PG_EINVAL, "bad batch arguments");
    pg_options o;
    if (opt) o = *opt;
    else pg_default_options(&o);
    const int d = dim;
    std::vector<FParams> fp(B);
    for (int b = 0; b < B; ++b) {
        pg_integrand f{family, dim, params + (size_t)b * n_params, n_params};
        int rc = make_params(ctx, &f, &fp[b]);
        if (rc) return rc;
        if (!(rel_tol[b] > 0.0) && !((abs_tol ? abs_tol[b] : o.abs_tol) > 0.0))
            return fail(ctx, PG_EINVAL, "integral %d has no positive tolerance", b);
    }
    const bool want_grad = grad != nullptr || leaves != nullptr;
    std::vector<GParams> gp;
    if (want_grad) {
        if (!adjoint_supported(family, d) || grad_nparams(family, d) != n_params)
            return fail(ctx, PG_EUNSUPPORTED,
                        "no parameter derivative for family %d", family);
        if (leaves && (!leaves->lo || !leaves->w || leaves->ld < 0))
            return fail(ctx, PG_EINVAL, "leaves: NULL array or ld < 0");
        gp.resize(B);
        for (int b = 0; b < B; ++b)
            make_gparams(family, d, params + (size_t)b * n_params, &gp[b]);
        if (grad)
            for (size_t q = 0; q < (size_t)B * n_params; ++q) grad[q] = 0.0;
        if (leaves) leaves->n = 0;
    }
    for (int k = 0; k < d; ++k)
        if (!(lo[k] < hi[k]) || !std::isfinite(lo[k]) || !std::isfinite(hi[k]))
            return fail(ctx, PG_EINVAL, "empty or infinite range on axis %d", k);
    if (o.init_splits < 1 || o.max_iters < 1)
        return fail(ctx, PG_EINVAL, "init_splits / max_iters < 1");
    if (int rc_rules = check_rules(ctx, o)) return rc_rules;
    const int64_t cap = o.max_regions > 0 ? o.max_regions : ctx->cap;
    if (cap > ctx->cap)
        return fail(ctx, PG_ENOMEM, "max_regions %lld above the capacity %lld",
                    (long long)cap, (long long)ctx->cap);
    int64_t g_d = 1;
    for (int k = 0; k < d; ++k) {
        g_d *= o.init_splits;
        if (g_d > cap)
            return fail(ctx, PG_EINVAL, "initial grid above the cap");
    }
    const int K = (int)std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)B, ctx->cap / cap,
                              (int64_t)BATCH_MAX_SLOTS}));
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const Rule R = make_rule(d, o.error_rule);
    const int64_t ld = ctx->cap;
    double a[PG_DIM_MAX], width[PG_DIM_MAX];
    for (int k = 0; k < d; ++k) {
        a[k] = lo[k];
        width[k] = (hi[k] - lo[k]) / (double)o.init_splits;
    }

    struct Slot {
        int b = -1, it = 0;
        double v_f = 0, e_f = 0, prev = NAN, v_tot = 0, e_tot = 0;
        int64_t start = 0, n = 0, n_rel = 0;
        int paired = 0;
    };
    std::vector<Slot> slots(K);
    std::vector<int> order, free_slots;
    for (int k = K - 1; k >= 0; --k) free_slots.push_back(k);
    for (int b = 0; b < B; ++b) {
        std::memset(&out[b], 0, sizeof(pg_result));
        out[b].estimate = NAN;
        out[b].error = NAN;
    }
    int next_b = 0;
    int cur = 0;
    // host copy of the slot table; every upload goes through the pinned
    // staging copies in turn (at most two uploads in a row are not separated
    // by a stream synchronisation, so a copy is never rewritten while its
    // last upload may still be pending)
    std::vector<BInst> HIv(K);
    BInst *HI = HIv.data();
    int stage = 0;
    std::vector<Totals> Tc(K);                  // classify totals per slot
    // derivative sums of the last adjoint launch, read after the next
    // synchronisation: (slot, integral) pairs they belong to
    std::vector<std::pair<int, int>> git_owner;
    int64_t n_leaves = 0;
    auto take_git = [&]() {
        if (grad)
            for (auto &sb : git_owner)
                for (int q = 0; q < n_params; ++q)
                    grad[(size_t)sb.second * n_params + q] +=
                        ctx->hb_git[(size_t)sb.first * GRAD_MAX + q];
        git_owner.clear();
    };
    auto finish = [&](int k, int status) {
        Slot &S = slots[k];
        pg_result &r = out[S.b];
        r.estimate = S.v_tot;
        r.error = S.e_tot;
        r.status = status;
        r.iterations = S.it;
        r.fevals = r.regions_evaluated * npoints(d);
        r.eval_launches = S.it;
        HI[k].live = 0;
    };
    // admit integrals into free slots; their boxes go to [running, ...) of
    // the list being built
    int64_t running = 0;
    int nnew = 0;
    auto admit = [&]() {
        nnew = 0;
        while (next_b < B && !free_slots.empty()) {
            const int k = free_slots.back();
            free_slots.pop_back();
            Slot &S = slots[k];
            S = Slot{};
            S.b = next_b++;
            S.start = running;
            S.n = g_d;
            ctx->hb_table[k] = fp[S.b];
            if (want_grad) ctx->hb_gtable[k] = gp[S.b];
            std::memset(&HI[k], 0, sizeof(BInst));
            HI[k].out_start = running;
            ctx->hb_new[nnew++] = k;
            order.push_back(k);
            running += g_d;
        }
    };
    // the slot header: one upload of the prefix a phase needs
    const HdrLayout hl = hdr_layout((size_t)K);
    ctx->b_inst = (BInst *)ctx->b_hdr;
    ctx->b_order = (int32_t *)(ctx->b_hdr + hl.order);
    ctx->b_new = (int32_t *)(ctx->b_hdr + hl.nw);
    ctx->b_state = (SearchState *)(ctx->b_hdr + hl.state);
    enum { UP_INST, UP_ORDER, UP_NEW, UP_STATE };
    auto upload = [&](int upto) -> int {
        char *h = ctx->hb_hdr + (size_t)stage * HDR_MAX;
        stage = (stage + 1) % INST_STAGES;
        std::memcpy(h, HI, sizeof(BInst) * K);
        size_t bytes = hl.end_inst;
        if (upto >= UP_ORDER) {
            std::memcpy(h + hl.order, ctx->hb_order, sizeof(int32_t) * K);
            bytes = hl.end_order;
        }
        if (upto >= UP_NEW) {
            std::memcpy(h + hl.nw, ctx->hb_new, sizeof(int32_t) * K);
            bytes = hl.end_new;
        }
        if (upto >= UP_STATE) {
            std::memcpy(h + hl.state, ctx->hb_state, sizeof(SearchState) * K);
            bytes = hl.end_state;
        }
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->b_hdr, h, bytes,
                                        hipMemcpyHostToDevice, st));
        return PG_OK;
    };
#define BRUN(expr)                                                             \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_) return rc_;                                                   \
    } while (0)

    admit();
    if (nnew) {
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->b_table, ctx->hb_table,
                                        sizeof(FParams) * K,
                                        hipMemcpyHostToDevice, st));
        if (want_grad)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->b_gtable, ctx->hb_gtable,
                                            sizeof(GParams) * K,
                                            hipMemcpyHostToDevice, st));
        BRUN(upload(UP_NEW));
        HIP_OR_FAIL(ctx, launch_batch_init(st, d, o.init_splits, a, width, nnew,
                                           ctx->b_new, ctx->b_inst,
                                           ctx->lo[cur], ctx->w[cur], ld,
                                           ctx->inst[cur]));
    }
    int64_t n_total = running;
    const FParams dummy{};
    while (!order.empty()) {
        // ---- per-slot layout of the current list
        int64_t seg0 = 0, cls0 = 0;
        for (size_t q = 0; q < order.size(); ++q) {
            const int k = order[q];
            Slot &S = slots[k];
            ++S.it;
            out[S.b].regions_evaluated += S.n;
            out[S.b].peak_regions = std::max<int64_t>(out[S.b].peak_regions, S.n);
            BInst &I = HI[k];
            I.start = S.start;
            I.n = S.n;
            I.paired = S.paired;
            I.tau = rel_tol[S.b];
            I.relerr = o.relerr_filter;
            I.live = 1;
            I.searching = 0;
            I.seg0 = seg0;
            I.cls0 = cls0;
            if (S.paired) {
                const int64_t nh = (S.n / 2 + BSEG - 1) / BSEG;
                I.nseg = 2 * nh;
                I.ncls = nh;
            } else {
                I.nseg = (S.n + BSEG - 1) / BSEG;
                I.ncls = I.nseg;
            }
            seg0 += I.nseg;
            cls0 += I.ncls;
            ctx->hb_order[q] = k;
        }
        const int nslots = (int)order.size();
        const int64_t nseg = seg0, ncls = cls0;
        if (nseg > ctx->nseg_max)
            return fail(ctx, PG_ENOMEM, "segment table overflow");
        BRUN(upload(UP_ORDER));
        // ---- EVALUATE, TWO-LEVEL + CLASSIFY, per-slot sums
        HIP_OR_FAIL(ctx, launch_evaluate(st, family, d, dummy, R, n_total,
                                         ctx->lo[cur], ctx->w[cur], ld, ctx->V,
                                         ctx->E, ctx->K,
                                         eval_waves(d, n_total, ctx->wave_target),
                                         ctx->inst[cur], ctx->b_table));
        HIP_OR_FAIL(ctx, launch_batch_tables(st, nslots, ctx->b_order,
                                             ctx->b_inst, ctx->b_segs,
                                             ctx->b_cls));
        HIP_OR_FAIL(ctx, launch_batch_classify(st, ncls, ctx->b_cls,
                                               ctx->b_inst, ctx->V, ctx->E,
                                               ctx->Vp, ctx->A, ctx->part));
        // the slots' totals go straight to the mapped host copy
        HIP_OR_FAIL(ctx, launch_batch_reduce(st, nslots, ctx->b_order,
                                             ctx->b_inst, ctx->part, ctx->off,
                                             ctx->b_tot, ctx->hb_tot_dev));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        take_git();
        // ---- termination test and threshold triggers, per slot
        int searching = 0;
        for (int k : order) {
            Slot &S = slots[k];
            const Totals &T = ctx->hb_tot[k];
            Tc[k] = T;
            const double tau = rel_tol[S.b];
            const double atol = abs_tol ? abs_tol[S.b] : o.abs_tol;
            S.v_tot = T.v + S.v_f;
            S.e_tot = T.e + S.e_f;
            S.n_rel = (int64_t)T.cnt;
            if (S.e_tot <= tau * std::fabs(S.v_tot) || S.e_tot <= atol) {
                finish(k, PG_OK);
                continue;
            }
            const bool trig_a = o.threshold_filter && S.it >= 2 &&
                                std::fabs(S.v_tot - S.prev) <= tau * std::fabs(S.v_tot);
            const bool trig_b = o.threshold_filter && 2 * S.n_rel > cap;
            if (trig_a || trig_b) {
                SearchState z{};
                z.n = S.n;
                z.e_it = T.e;
                z.allowance = search_allowance(o, trig_b, tau, S.v_tot, S.v_f,
                                               S.e_f, T.fv);
                z.relax = relax_pmax(o, trig_b);
                z.mn = T.emin;
                z.mx = T.emax;
                z.t = T.e / (double)S.n;
                z.P_max = 0.25;
                z.t_acc = -HUGE_VAL;
                ctx->hb_state[k] = z;
                HI[k].searching = 1;
                ++out[S.b].threshold_calls;
                ++searching;
            }
        }
        BRUN(upload(searching ? UP_STATE : UP_INST));
        // ---- THRESHOLD-CLASSIFY for every slot that needs it
        if (searching) {
            const int max_passes =
                (THR_MAX_TRIALS + TRIAL_DEPTH - 1) / TRIAL_DEPTH;
            HIP_OR_FAIL(ctx, launch_batch_search_hist(
                                 st, nseg, ctx->b_segs, nslots, ctx->b_order,
                                 ctx->b_inst, ctx->E, ctx->A, ctx->b_state,
                                 ctx->hcnt, ctx->hsum, ctx->htlo, ctx->hthi));
            int passes = 0;
            for (int bi = -1; bi < 3 && passes < max_passes; ++bi) {
                const int batch = bi < 0 ? 0
                    : std::min(SEARCH_BATCHES[bi], max_passes - passes);
                for (int q = 0; q < batch; ++q)
                    HIP_OR_FAIL(ctx, launch_batch_search_pass(
                                         st, nseg, ctx->b_segs, nslots,
                                         ctx->b_order, ctx->b_inst, ctx->E,
                                         ctx->A, ctx->b_state, ctx->b_tpart,
                                         ctx->htlo, ctx->hthi));
                passes += batch;
                HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->hb_state, ctx->b_state,
                                                sizeof(SearchState) * K,
                                                hipMemcpyDeviceToHost, st));
                HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
                bool all = true;
                for (int k : order)
                    if (HI[k].searching && !ctx->hb_state[k].done) all = false;
                if (all) break;
            }
            // a search that has not ended has not accepted (ok is set only
            // with done), so the device's states need no correction
            for (int k : order)
                if (HI[k].searching)
                    out[slots[k].b].threshold_trials += ctx->hb_state[k].trials;
        }
        // ---- survivors per slot
        HIP_OR_FAIL(ctx, launch_batch_count(st, nseg, ctx->b_segs, ctx->b_inst,
                                            ctx->b_state, ctx->V, ctx->E,
                                            ctx->A, ctx->part));
        // the slots' totals go straight to the mapped host copy
        HIP_OR_FAIL(ctx, launch_batch_reduce(st, nslots, ctx->b_order,
                                             ctx->b_inst, ctx->part, ctx->off,
                                             ctx->b_tot, ctx->hb_tot_dev));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
        running = 0;
        std::vector<int> next_order;
        for (int k : order) {
            Slot &S = slots[k];
            BInst &I = HI[k];
            if (!I.live) {                             // converged above
                free_slots.push_back(k);
                continue;
            }
            const bool ok = I.searching && ctx->hb_state[k].ok;
            int status = -1;
            if (!ok && 2 * S.n_rel > cap) status = PG_MEMORY_EXHAUSTED;
            const int64_t n_act = (int64_t)ctx->hb_tot[k].cnt;
            if (status < 0 && n_act == 0) status = PG_NO_ACTIVE;
            if (status < 0 && S.it == o.max_iters) status = PG_MAX_ITERS;
            if (status >= 0) {
                finish(k, status);
                free_slots.push_back(k);
                continue;
            }
            // finished contributions: this iteration's sums (v, e) less the
            // survivors' (from the classify pass unless a threshold was
            // accepted, as in pg_integrate)
            const Totals &T = Tc[k];
            const Totals &Ts = ok ? ctx->hb_tot[k] : T;
            S.prev = S.v_tot;
            S.v_f = T.v - Ts.av + S.v_f;
            S.e_f = T.e - Ts.ae + S.e_f;
            I.out_start = running;
            I.na = n_act;
            running += 2 * n_act;
            S.start = I.out_start;
            S.n = 2 * n_act;
            S.paired = 1;
            next_order.push_back(k);
        }
        // ---- derivative over this iteration's leaves: all regions of an
        // integral that ends, the non-survivors of the others
        if (want_grad) {
            int64_t fin = 0;
            for (int k : order) {
                BInst &I = HI[k];
                I.fin_base = fin;
                I.owner = slots[k].b;
                fin += I.live ? I.n - I.na : I.n;
                git_owner.emplace_back(k, slots[k].b);
            }
            if (leaves && n_leaves + fin > leaves->ld)
                return fail(ctx, PG_ENOMEM, "more than %lld leaves",
                            (long long)leaves->ld);
            BRUN(upload(UP_INST));
            LeafOut lout{};
            if (leaves) {
                lout.lo = leaves->lo;
                lout.w = leaves->w;
                lout.owner = leaves->owner;
                lout.ld = leaves->ld;
                lout.base = n_leaves;
            }
            HIP_OR_FAIL(ctx, launch_batch_adjoint(
                                 st, family, d, nseg, ctx->b_segs, ctx->b_inst,
                                 ctx->b_state, ctx->A, ctx->E, ctx->lo[cur],
                                 ctx->w[cur], ld, ctx->b_gtable, R,
                                 ctx->b_gpart, ctx->off, lout));
            HIP_OR_FAIL(ctx, launch_batch_grad_reduce(
                                 st, nslots, ctx->b_order, ctx->b_inst,
                                 ctx->b_gtable, n_params, ctx->b_gpart, nseg,
                                 ctx->b_git));
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->hb_git, ctx->b_git,
                                            sizeof(double) * GRAD_MAX * K,
                                            hipMemcpyDeviceToHost, st));
            n_leaves += fin;
        }
        order.swap(next_order);
        admit();
        BRUN(upload(nnew ? UP_NEW : UP_INST));
        HIP_OR_FAIL(ctx, launch_batch_compact(
                             st, d, nseg, ctx->b_segs, ctx->b_inst,
                             ctx->b_state, ctx->A, ctx->E, ctx->V, ctx->K,
                             ctx->lo[cur], ctx->w[cur], ld, ctx->off,
                             ctx->lo[1 - cur], ctx->w[1 - cur], ctx->Vp,
                             ctx->inst[1 - cur]));
        if (nnew) {
            HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->b_table, ctx->hb_table,
                                            sizeof(FParams) * K,
                                            hipMemcpyHostToDevice, st));
            if (want_grad)
                HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->b_gtable, ctx->hb_gtable,
                                                sizeof(GParams) * K,
                                                hipMemcpyHostToDevice, st));
            HIP_OR_FAIL(ctx, launch_batch_init(st, d, o.init_splits, a, width,
                                               nnew, ctx->b_new, ctx->b_inst,
                                               ctx->lo[1 - cur], ctx->w[1 - cur],
                                               ld, ctx->inst[1 - cur]));
        }
        cur = 1 - cur;
        n_total = running;
    }
    HIP_OR_FAIL(ctx, hipStreamSynchronize(st));
    take_git();
    if (leaves) leaves->n = n_leaves;
#undef BRUN
    return PG_OK;
}

int pg_integrate_batch(pg_context *ctx, int family, int dim, int B,
                       const double *params, int n_params, const double *lo,
                       const double *hi, const double *rel_tol,
                       const double *abs_tol, const pg_options *opt,
                       pg_result *out) {
    return run_batch(ctx, family, dim, B, params, n_params, lo, hi, rel_tol,
                     abs_tol, opt, out, nullptr, nullptr);
}

int pg_integrate_batch_grad(pg_context *ctx, int family, int dim, int B,
                            const double *params, int n_params,
                            const double *lo, const double *hi,
                            const double *rel_tol, const double *abs_tol,
                            const pg_options *opt, pg_result *out,
                            double *grad, pg_leaves *leaves) {
    if (!grad) {
        if (ctx) ctx->err = "grad is NULL";
        return PG_EINVAL;
    }
    return run_batch(ctx, family, dim, B, params, n_params, lo, hi, rel_tol,
                     abs_tol, opt, out, grad, leaves);
}

int pg_integrate_grad(pg_context *ctx, const pg_integrand *f,
                      const double *lo, const double *hi,
                      const pg_options *opt, pg_result *out, double *grad,
                      pg_leaves *leaves) {
    if (!ctx) return PG_EINVAL;
    if (!f || !grad || !out) {
        ctx->err = "integrand, grad or out is NULL";
        return PG_EINVAL;
    }
    pg_options o;
    if (opt) o = *opt;
    else pg_default_options(&o);
    const double rt = o.rel_tol, at = o.abs_tol;
    const int rc = run_batch(ctx, f->family, f->dim, 1, f->params, f->n_params,
                             lo, hi, &rt, &at, &o, out, grad, leaves);
    return rc < 0 ? rc : out->status;
}

}  // extern "C"
