// pg_noalloc.hip -- FILTER + parent update + SPLIT for callers that cannot
// allocate device memory (code under stream capture, serving loops and
// harnesses that forbid hipMalloc).
//
// pg_filter_split keeps the compaction's scratch (per-segment partial sums
// and counts, the scanned segment offsets and the totals) in a context's
// workspace. This variant keeps them in one file-scope device array per GPU,
// sized for lists of up to PG_NOALLOC_MAX_REGIONS regions, and otherwise
// runs the same kernels. The array's device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels: in host code the array's name is a host
// stand-in, not a device pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pg_internal.hpp"

using namespace pg;

namespace {

constexpr int64_t NA_MAX_SEGS = PG_NOALLOC_MAX_REGIONS / SEG;
static_assert(PG_NOALLOC_MAX_REGIONS % SEG == 0, "whole segments");

// Layout of the scratch: seven double partials and the count per segment,
// the segment offsets, the totals.
constexpr size_t NA_ALIGN = 256;
constexpr size_t na_round(size_t x) { return (x + NA_ALIGN - 1) / NA_ALIGN * NA_ALIGN; }
constexpr size_t NA_PART_D = na_round(sizeof(double) * NA_MAX_SEGS);
constexpr size_t NA_PART_U = na_round(sizeof(uint32_t) * NA_MAX_SEGS);
constexpr size_t NA_BYTES = 7 * NA_PART_D + 2 * NA_PART_U + na_round(sizeof(Totals));
static_assert(NA_BYTES <= PG_NOALLOC_SCRATCH_BYTES, "scratch layout");

__device__ __align__(256) unsigned char scratch[PG_NOALLOC_SCRATCH_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
unsigned char *na_ptr[NA_MAX_DEVICES] = {};

// Device address of this device's scratch (the current device), looked up
// on the first call on that device.
int scratch_for_current_device(unsigned char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PG_EHIP;
    if (dev < 0 || dev >= NA_MAX_DEVICES) return PG_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return PG_EHIP;
        na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = na_ptr[dev];
    return PG_OK;
}

}  // namespace

extern "C" int pg_filter_split_noalloc(void *stream, int dim, int64_t n,
                                       const double *lo, const double *w,
                                       int64_t ld_in, const uint8_t *K,
                                       const double *V, const uint8_t *A,
                                       double *lo_out, double *w_out,
                                       int64_t ld_out, double *Vp,
                                       int64_t *n_active) {
    if (!n_active) return PG_EINVAL;
    *n_active = 0;
    if (dim < PG_DIM_MIN || dim > PG_DIM_MAX) return PG_EINVAL;
    if (n < 0 || ld_in < n) return PG_EINVAL;
    if (n > PG_NOALLOC_MAX_REGIONS) return PG_EINVAL;
    if (n == 0) return PG_OK;
    if (!lo || !w || !K || !V || !A || !lo_out || !w_out || !Vp) return PG_EINVAL;
    unsigned char *base = nullptr;
    int rc = scratch_for_current_device(&base);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);

    SegPartials part;
    size_t at = 0;
    double **dp[7] = {&part.v, &part.e, &part.av, &part.ae, &part.fv, &part.emin,
                      &part.emax};
    for (double **p : dp) {
        *p = reinterpret_cast<double *>(base + at);
        at += NA_PART_D;
    }
    part.cnt = reinterpret_cast<uint32_t *>(base + at);
    at += NA_PART_U;
    uint32_t *off = reinterpret_cast<uint32_t *>(base + at);
    at += NA_PART_U;
    Totals *tot = reinterpret_cast<Totals *>(base + at);

    // every scratch word the kernels read is written by them first (each
    // segment's partials by its block, the offsets and totals by the scan),
    // so nothing is cleared between calls
    if (launch_seg_count(st, n, 0, 0.0, V, nullptr, A, nullptr, part) != hipSuccess)
        return PG_EHIP;
    if (launch_reduce_scan(st, seg_count(n, 0), part, off, tot) != hipSuccess)
        return PG_EHIP;
    Totals T;
    if (hipMemcpyAsync(&T, tot, sizeof(Totals), hipMemcpyDeviceToHost, st) != hipSuccess)
        return PG_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PG_EHIP;
    const int64_t na = (int64_t)T.cnt;
    if (ld_out < 2 * na) return PG_EINVAL;
    if (launch_compact_split(st, dim, n, 0, 0.0, A, nullptr, V, K, lo, w, ld_in,
                             off, na, lo_out, w_out, ld_out, Vp) != hipSuccess)
        return PG_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PG_EHIP;
    *n_active = na;
    return PG_OK;
}
