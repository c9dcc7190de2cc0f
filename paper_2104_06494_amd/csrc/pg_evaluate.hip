// pg_evaluate.hip -- launchers of the EVALUATE kernels (pg_eval_kernels.hpp,
// instantiated per family in pg_eval_family.hip).
#include "pg_internal.hpp"

#include <hip/hip_runtime.h>

namespace pg {

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
typedef void (*EvalKernel)(const FParams, const Rule, int64_t, const double *,
                           const double *, int64_t, double *, double *,
                           uint8_t *, const uint32_t *, const FParams *);
typedef void (*FvalKernel)(const FParams, int64_t, const double *, int64_t,
                           double *);
// defined per family in pg_eval_family.hip
template <int FAM> EvalKernel eval_family(int d, bool batch);
template <int FAM> FvalKernel fval_family(int d);

static EvalKernel eval_kernel(int family, int d, bool batch) {
    switch (family) {
    case PG_PRODUCT_PEAK: return eval_family<PG_PRODUCT_PEAK>(d, batch);
    case PG_GAUSSIAN: return eval_family<PG_GAUSSIAN>(d, batch);
    case PG_OSCILLATORY: return eval_family<PG_OSCILLATORY>(d, batch);
    case PG_CORNER_PEAK: return eval_family<PG_CORNER_PEAK>(d, batch);
    case PG_MONOMIAL: return eval_family<PG_MONOMIAL>(d, batch);
    case PG_C0: return eval_family<PG_C0>(d, batch);
    case PG_DISCONTINUOUS: return eval_family<PG_DISCONTINUOUS>(d, batch);
    case PG_BOX: return eval_family<PG_BOX>(d, batch);
    default: return nullptr;
    }
}

static FvalKernel fval_kernel(int family, int d) {
    switch (family) {
    case PG_PRODUCT_PEAK: return fval_family<PG_PRODUCT_PEAK>(d);
    case PG_GAUSSIAN: return fval_family<PG_GAUSSIAN>(d);
    case PG_OSCILLATORY: return fval_family<PG_OSCILLATORY>(d);
    case PG_CORNER_PEAK: return fval_family<PG_CORNER_PEAK>(d);
    case PG_MONOMIAL: return fval_family<PG_MONOMIAL>(d);
    case PG_C0: return fval_family<PG_C0>(d);
    case PG_DISCONTINUOUS: return fval_family<PG_DISCONTINUOUS>(d);
    case PG_BOX: return fval_family<PG_BOX>(d);
    default: return nullptr;
    }
}

hipError_t launch_fvalues(hipStream_t st, int family, int d, const FParams &P,
                          int64_t n, const double *x, int64_t ld, double *y) {
    FvalKernel k = fval_kernel(family, d);
    if (!k) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       P, n, x, ld, y);
    return hipGetLastError();
}

bool evaluate_supported(int family, int d) {
    return eval_kernel(family, d, false) != nullptr;
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
                           double *V, double *E, uint8_t *K, int waves,
                           const uint32_t *inst, const FParams *table) {
    EvalKernel k = eval_kernel(family, d, inst != nullptr);
    if (!k) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    // the kernel assigns work units to waves by u mod W with a bit mask
    if (waves < 1 || waves > EVAL_MAX_WAVES || (waves & (waves - 1)))
        return hipErrorInvalidValue;
    const int64_t blocks = (n + 63) / 64;
    const size_t lds = sizeof(double) * 64 * (size_t)(d + (waves > 1 ? 5 * waves : 0));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * waves), lds, st, P,
                       R, n, lo, w, ld, V, E, K, inst, table);
    return hipGetLastError();
}


}  // namespace pg
