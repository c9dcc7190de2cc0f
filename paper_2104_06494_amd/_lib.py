"""ctypes binding of libpagani.so (the HIP library built from csrc/).

Argument marshalling only: every step of the method runs in the library's
kernels. PyTorch provides the device memory (workspace and arrays) and the
stream work is queued on. Importing this module on a machine without the
built library raises immediately; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpagani.so")

PG_DIM_MIN, PG_DIM_MAX = 2, 10
FAMILY_ID = {"product_peak": 0, "gaussian": 1, "oscillatory": 2,
             "corner_peak": 3, "monomial": 4, "c0": 5, "discontinuous": 6,
             "box": 7}
ERROR_RULE = {"raw": 0, "null4": 1}
# P_max relaxation of the threshold search: at every direction change
# (Section 3.5.3, the default) or only in searches under memory pressure
PMAX_RELAX = {"paper": 0, "memory": 1}
# Error budget of a threshold search started because the estimate's digits
# have settled: keep back what the active regions may still end with
# (Lemma 1, the default) or nothing
BUDGET = {"reserve": 0, "listing": 1}
STATUS = {0: "OK", 1: "MAX_ITERS", 2: "MEMORY_EXHAUSTED", 3: "NO_ACTIVE",
          -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSUPPORTED"}

EXPORTS = ["pg_default_options", "pg_workspace_bytes", "pg_context_create",
           "pg_context_destroy", "pg_context_set_stream", "pg_last_error",
           "pg_integrate", "pg_last_regions", "pg_evaluate", "pg_classify",
           "pg_threshold_search", "pg_filter_split", "pg_integrand_values",
           "pg_integrate_batch", "pg_integrate_grad", "pg_integrate_batch_grad",
           "pg_evaluate_rule", "pg_filter_split_noalloc", "pg_context_set_eval_waves"]


class Integrand(C.Structure):
    _fields_ = [("family", C.c_int), ("dim", C.c_int),
                ("params", C.POINTER(C.c_double)), ("n_params", C.c_int)]


class Options(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double),
                ("init_splits", C.c_int), ("max_iters", C.c_int),
                ("relerr_filter", C.c_int), ("threshold_filter", C.c_int),
                ("max_regions", C.c_int64), ("timing", C.c_int),
                ("trace_path", C.c_char_p), ("error_rule", C.c_int),
                ("pmax_relax", C.c_int), ("budget", C.c_int)]


class Result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("error", C.c_double),
                ("status", C.c_int), ("iterations", C.c_int),
                ("regions_evaluated", C.c_int64), ("fevals", C.c_int64),
                ("peak_regions", C.c_int64), ("threshold_calls", C.c_int64),
                ("threshold_trials", C.c_int64),
                ("phase_ms", C.c_double * 4), ("eval_launches", C.c_int64)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class RegionsView(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64), ("ld", C.c_int64),
                ("lo", C.c_void_p), ("w", C.c_void_p), ("V", C.c_void_p),
                ("E", C.c_void_p), ("K", C.c_void_p), ("A", C.c_void_p)]


class Leaves(C.Structure):
    _fields_ = [("lo", C.c_void_p), ("w", C.c_void_p), ("owner", C.c_void_p),
                ("ld", C.c_int64), ("n", C.c_int64)]


_lib = None


def load():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2104_06494_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i64 = C.c_void_p, C.c_int64
    L.pg_default_options.argtypes = [C.POINTER(Options)]
    L.pg_default_options.restype = None
    L.pg_workspace_bytes.argtypes = [C.c_int, i64]
    L.pg_workspace_bytes.restype = C.c_size_t
    L.pg_context_create.argtypes = [C.c_int, C.c_int, i64, vp, C.c_size_t, vp,
                                    C.POINTER(vp)]
    L.pg_context_create.restype = C.c_int
    L.pg_context_destroy.argtypes = [vp]
    L.pg_context_destroy.restype = None
    L.pg_context_set_stream.argtypes = [vp, vp]
    L.pg_context_set_stream.restype = C.c_int
    L.pg_last_error.argtypes = [vp]
    L.pg_last_error.restype = C.c_char_p
    L.pg_integrate.argtypes = [vp, C.POINTER(Integrand), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(Options),
                               C.POINTER(Result)]
    L.pg_integrate.restype = C.c_int
    dp = C.POINTER(C.c_double)
    L.pg_integrate_batch.argtypes = [vp, C.c_int, C.c_int, C.c_int, dp, C.c_int,
                                     dp, dp, dp, dp, C.POINTER(Options),
                                     C.POINTER(Result)]
    L.pg_integrate_batch.restype = C.c_int
    L.pg_integrate_grad.argtypes = [vp, C.POINTER(Integrand), dp, dp,
                                    C.POINTER(Options), C.POINTER(Result), dp,
                                    C.POINTER(Leaves)]
    L.pg_integrate_grad.restype = C.c_int
    L.pg_integrate_batch_grad.argtypes = [vp, C.c_int, C.c_int, C.c_int, dp, C.c_int,
                                          dp, dp, dp, dp, C.POINTER(Options),
                                          C.POINTER(Result), dp, C.POINTER(Leaves)]
    L.pg_integrate_batch_grad.restype = C.c_int
    L.pg_last_regions.argtypes = [vp, C.POINTER(RegionsView)]
    L.pg_last_regions.restype = C.c_int
    L.pg_evaluate.argtypes = [vp, C.POINTER(Integrand), i64, vp, vp, i64, vp,
                              vp, vp]
    L.pg_evaluate.restype = C.c_int
    L.pg_evaluate_rule.argtypes = [vp, C.POINTER(Integrand), C.c_int, i64, vp, vp,
                                   i64, vp, vp, vp]
    L.pg_evaluate_rule.restype = C.c_int
    L.pg_integrand_values.argtypes = [vp, C.POINTER(Integrand), i64, vp, i64, vp]
    L.pg_integrand_values.restype = C.c_int
    L.pg_classify.argtypes = [vp, i64, C.c_int, vp, vp, vp, C.c_double, C.c_int,
                              vp, C.POINTER(C.c_double)]
    L.pg_classify.restype = C.c_int
    L.pg_threshold_search.argtypes = [vp, i64, vp, vp, C.c_double, C.c_double,
                                      C.c_int, vp,
                                      C.POINTER(C.c_int), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int)]
    L.pg_threshold_search.restype = C.c_int
    L.pg_filter_split.argtypes = [vp, C.c_int, i64, vp, vp, i64, vp, vp, vp, vp,
                                  vp, i64, vp, C.POINTER(i64)]
    L.pg_filter_split.restype = C.c_int
    L.pg_filter_split_noalloc.argtypes = [vp, C.c_int, i64, vp, vp, i64, vp, vp, vp,
                                          vp, vp, i64, vp, C.POINTER(i64)]
    L.pg_filter_split_noalloc.restype = C.c_int
    L.pg_context_set_eval_waves.argtypes = [vp, C.c_int]
    L.pg_context_set_eval_waves.restype = C.c_int
    _lib = L
    return L
