"""ctypes wrapper of the C oracle -- TEST INFRASTRUCTURE ONLY.

Each function names the part of the paper it follows; the C source carries
the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAGANI_ORACLE_LIB lets the mutation tests load a deliberately broken copy
_LIB_PATH = os.environ.get("PAGANI_ORACLE_LIB",
                           os.path.join(_HERE, "liboracle.so"))
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

FAMILY_ID = {"product_peak": 0, "gaussian": 1, "oscillatory": 2,
             "corner_peak": 3, "monomial": 4, "c0": 5, "discontinuous": 6,
             "box": 7}

STATUS = {0: "OK", 1: "MAX_ITERS", 2: "MEMORY_EXHAUSTED", 3: "NO_ACTIVE"}

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class ReplayStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "axis_override", "axis_hard", "class_override", "class_hard",
        "term_override", "term_hard", "trig_override", "trig_hard",
        "search_hard", "thr_override", "thr_hard", "records")] + [
        ("max_t_rel", C.c_double), ("max_v_rel", C.c_double),
        ("max_e_rel", C.c_double)] + [
        (n, C.c_int64) for n in ("search_hard_it", "gpu_ok", "gpu_trials",
                                 "cpu_ok", "cpu_trials")] + [
        ("gpu_t", C.c_double), ("cpu_t", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def lib(parallel: bool = False):
    """Load liboracle.so (parallel: its OpenMP timing build), building it
    first if it is missing."""
    global _lib, _lib_omp
    if (_lib_omp if parallel else _lib) is not None:
        return _lib_omp if parallel else _lib
    path = _LIB_OMP_PATH if parallel else _LIB_PATH
    if not os.path.exists(path):
        from .build import build
        build()
    L = C.CDLL(path)
    L.oracle_threads.restype = C.c_int
    L.oracle_threads.argtypes = []
    L.oracle_f.restype = C.c_double
    L.oracle_f.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.oracle_npoints.restype = C.c_long
    L.oracle_npoints.argtypes = [C.c_int]
    L.oracle_rule.restype = None
    L.oracle_rule.argtypes = [C.c_int, _dp, _dp, _dp]
    L.oracle_eval_regions.restype = C.c_int
    L.oracle_eval_regions.argtypes = [C.c_int, C.c_int, _dp, C.c_long, _dp, _dp,
                                      C.c_long, C.c_int, _dp, _dp, _u8,
                                      C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
    L.oracle_null_rules.restype = None
    L.oracle_null_rules.argtypes = [C.c_int, _dp]
    L.oracle_two_level.restype = None
    L.oracle_two_level.argtypes = [C.c_long, _dp, _dp, _dp]
    L.oracle_classify.restype = None
    L.oracle_classify.argtypes = [C.c_long, _dp, _dp, C.c_double, C.c_int, _u8]
    L.oracle_sum.restype = C.c_double
    L.oracle_sum.argtypes = [C.c_long, _dp, C.c_void_p]
    L.oracle_threshold_search.restype = C.c_int
    L.oracle_threshold_search.argtypes = [C.c_long, _dp, _u8, C.c_double,
                                          C.c_double, C.c_int, _u8,
                                          C.POINTER(C.c_double),
                                          C.POINTER(C.c_int), C.c_void_p]
    L.oracle_filter_split.restype = C.c_long
    L.oracle_filter_split.argtypes = [C.c_int, C.c_long, _dp, _dp, C.c_long,
                                      _u8, _dp, _u8, _dp, _dp, C.c_long, _dp]
    L.oracle_uniform_split.restype = C.c_long
    L.oracle_uniform_split.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, _dp,
                                       C.c_long]
    L.oracle_integrate.restype = C.c_int
    L.oracle_integrate.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, C.c_double,
                                   C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                   C.c_char_p, _dp,
                                   np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"),
                                   C.POINTER(ReplayStats), C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.oracle_grad_f.restype = C.c_int
    L.oracle_grad_f.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
    L.oracle_grad_regions.restype = C.c_int
    L.oracle_grad_regions.argtypes = [C.c_int, C.c_int, _dp, C.c_long, _dp, _dp,
                                      C.c_long, _dp, _dp]
    if parallel:
        _lib_omp = L
    else:
        _lib = L
    return L


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def npoints(d: int) -> int:
    """Points of the degree-7 rule, 2^d + 2d^2 + 2d + 1 (Section 2.1)."""
    return int(lib().oracle_npoints(d))


def rule(d: int):
    """(w7[5], w5[5], lambda[5]) per-orbit weights relative to the volume."""
    w7, w5, lam = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().oracle_rule(d, w7, w5, lam)
    return w7, w5, lam


ERROR_RULE = {"raw": 0, "null4": 1}

# P_max relaxation of the threshold search: at every direction change of
# every search (Section 3.5.3) or only in searches under memory pressure
PMAX_RELAX = {"paper": 0, "memory": 1}

# Accuracy budget of a threshold search started because the estimate's
# digits have settled: "reserve" keeps back the error the rel-err-active
# regions may still end with (Lemma 1); "listing" keeps nothing back.
BUDGET = {"reserve": 0, "listing": 1}


def null_rules(d: int) -> np.ndarray:
    """[4, 5] per-orbit weights of the four null rules of reading R9
    (degrees 5, 3, 3, 1), each with the degree-7 rule's norm."""
    out = np.zeros(20)
    lib().oracle_null_rules(d, out)
    return out.reshape(4, 5)


def f(family: str, params, x) -> float:
    """One integrand value."""
    x = _f64(x)
    return lib().oracle_f(FAMILY_ID[family], len(x), _f64(params), x)


@dataclass
class RegionEval:
    V: np.ndarray
    E: np.ndarray
    K: np.ndarray
    D: np.ndarray           # [n, d] fourth differences
    floorV: np.ndarray
    floorE: np.ndarray
    floorD: np.ndarray


def eval_regions(family: str, d: int, params, lo, w, error_rule="raw") -> RegionEval:
    """Evaluate step (Section 3.2): V, E (|R7 - R5|, or the four-null-rule
    estimate of reading R9 with error_rule="null4"), split axis K for each
    box. ``lo`` and ``w`` are [d, n] (structure of arrays)."""
    lo, w = _f64(lo), _f64(w)
    n = lo.shape[1]
    V, E = np.zeros(n), np.zeros(n)
    K = np.zeros(n, np.uint8)
    D = np.zeros((n, d))
    fv, fe, fd = np.zeros(n), np.zeros(n), np.zeros(n)
    rc = lib().oracle_eval_regions(FAMILY_ID[family], d, _f64(params), n, lo, w,
                                   n, ERROR_RULE[error_rule], V, E, K, _ptr(D),
                                   _ptr(fv), _ptr(fe), _ptr(fd))
    if rc:
        raise ValueError(f"oracle_eval_regions: {rc}")
    return RegionEval(V, E, K, D, fv, fe, fd)


def two_level(V, E, Vp) -> np.ndarray:
    """Two-Level-Error on a list of 2m regions with parents Vp[m]; returns new E."""
    V, E2, Vp = _f64(V), _f64(E).copy(), _f64(Vp)
    lib().oracle_two_level(len(Vp), V, E2, Vp)
    return E2


def classify(V, E, tau_rel: float, relerr_filter: int = 1) -> np.ndarray:
    """Rel-Err-Classify (Section 3.5.1): 1 = active."""
    V, E = _f64(V), _f64(E)
    A = np.zeros(len(V), np.uint8)
    lib().oracle_classify(len(V), V, E, tau_rel, relerr_filter, A)
    return A


def csum(x, mask=None) -> float:
    x = _f64(x)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    return lib().oracle_sum(len(x), x, _ptr(m))


def threshold_search(E, A_rel, e_it, allow, relax=True):
    """Threshold-Classify (Algorithm 3); with relax, P_max grows by 0.10 at
    each change of direction up to 0.95 (Section 3.5.3), else it stays at
    0.25. The accuracy requirement allows the finished regions an error of
    P_max * allow (the listing's e_it - e_b = tau |v_tot| - e_f, or the
    finished regions' own share under the reserve reading). Returns (ok, A,
    t, trials, tried_ts)."""
    E = _f64(E)
    A_rel = np.ascontiguousarray(A_rel, dtype=np.uint8)
    A = np.zeros(len(E), np.uint8)
    t = C.c_double()
    tr = C.c_int()
    tried = np.zeros(64)
    ok = lib().oracle_threshold_search(len(E), E, A_rel, float(e_it), float(allow),
                                       int(bool(relax)), A,
                                       C.byref(t), C.byref(tr),
                                       _ptr(tried))
    return bool(ok), A, t.value, tr.value, tried[:tr.value].copy()


def filter_split(d, lo, w, K, V, A):
    """Filter + parent update + Split. Returns (lo2[d,2na], w2[d,2na], Vp[na])."""
    lo, w, V = _f64(lo), _f64(w), _f64(V)
    K = np.ascontiguousarray(K, dtype=np.uint8)
    A = np.ascontiguousarray(A, dtype=np.uint8)
    n = lo.shape[1]
    na = int(A.astype(bool).sum())
    lo2, w2 = np.zeros((d, 2 * na)), np.zeros((d, 2 * na))
    Vp = np.zeros(max(na, 1))
    got = lib().oracle_filter_split(d, n, lo, w, n, K, V, A, lo2, w2,
                                    max(2 * na, 1), Vp)
    assert got == na
    return lo2, w2, Vp[:na]


def uniform_split(d, a, b, g):
    """Uniform-Split (Section 3.1): g^d boxes, axis 0 varying fastest."""
    n = g ** d
    lo, w = np.zeros((d, n)), np.zeros((d, n))
    lib().oracle_uniform_split(d, _f64(a), _f64(b), g, lo, w, n)
    return lo, w


@dataclass
class OracleResult:
    estimate: float
    error: float
    status: int
    iterations: int
    regions_evaluated: int
    fevals: int
    peak_regions: int
    threshold_calls: int
    threshold_trials: int
    eval_seconds: float
    seconds: float
    replay: dict | None = None
    grad: np.ndarray | None = None       # d estimate / d params over the leaves
    grad_abs: np.ndarray | None = None   # sum of the absolute terms of grad
    leaf_v: float | None = None          # sum of the leaves' estimates

    @property
    def status_name(self):
        return STATUS.get(self.status, str(self.status))


def integrate(family: str, d: int, params, lo=None, hi=None, rel_tol=1e-3,
              abs_tol=1e-20, init_splits=4, max_iters=100, relerr_filter=1,
              threshold_filter=1, max_regions=1 << 22,
              replay_path: str | None = None, grad: bool = False,
              error_rule: str = "raw", pmax_relax: str = "paper",
              budget: str = "reserve", parallel: bool = False) -> OracleResult:
    """PAGANI main loop (Algorithm 2), free mode or replaying a GPU trace.
    With grad=True also the derivative of the estimate with respect to the
    parameters over the partition the run ends on (its leaves: every region
    finished on the way and the live list at the end). parallel=True runs
    the OpenMP timing build (same results; see threads())."""
    lo = np.zeros(d) if lo is None else _f64(lo)
    hi = np.ones(d) if hi is None else _f64(hi)
    out_d = np.zeros(4)
    out_i = np.zeros(7, np.int64)
    rs = ReplayStats()
    npar = len(np.atleast_1d(params))
    g = np.zeros(npar) if grad else None
    ga = np.zeros(npar) if grad else None
    lv = np.zeros(1)
    rc = lib(parallel).oracle_integrate(FAMILY_ID[family], d, _f64(params), lo, hi,
                                rel_tol, abs_tol, init_splits, max_iters,
                                relerr_filter, threshold_filter,
                                ERROR_RULE[error_rule], PMAX_RELAX[pmax_relax],
                                BUDGET[budget],
                                max_regions,
                                replay_path.encode() if replay_path else None,
                                out_d, out_i, C.byref(rs), _ptr(g), _ptr(ga), _ptr(lv))
    if rc:
        raise RuntimeError(f"oracle_integrate failed with code {rc}")
    return OracleResult(out_d[0], out_d[1], int(out_i[0]), int(out_i[1]),
                        int(out_i[2]), int(out_i[3]), int(out_i[4]),
                        int(out_i[5]), int(out_i[6]), out_d[2], out_d[3],
                        rs.as_dict() if replay_path else None, g, ga, float(lv[0]))


def threads(parallel: bool = True) -> int:
    """Threads the (parallel) build evaluates regions on."""
    return int(lib(parallel).oracle_threads())


def grad_f(family: str, params, x) -> np.ndarray:
    """Partial derivatives of one integrand value with respect to its
    parameters (same layout as params)."""
    x = _f64(x)
    p = _f64(params)
    df = np.zeros(2 * len(x) + 2)
    n = lib().oracle_grad_f(FAMILY_ID[family], len(x), p, x, df)
    if n < 0:
        raise ValueError(f"no parameter gradient for {family}")
    return df[:n]


def grad_regions(family: str, d: int, params, lo, w):
    """Derivative of the summed degree-7 estimates of the regions (SoA
    [d, n] corners and widths) with respect to the parameters, and the sum
    of the absolute terms (the adjoint over a fixed partition)."""
    lo, w = _f64(lo), _f64(w)
    n = lo.shape[1]
    G = np.zeros(2 * d + 2)
    Ga = np.zeros(2 * d + 2)
    k = lib().oracle_grad_regions(FAMILY_ID[family], d, _f64(params), n, lo, w, n, G, Ga)
    if k < 0:
        raise ValueError(f"no parameter gradient for {family}")
    return G[:k], Ga[:k]


def integrate_workload(wl, **kw) -> OracleResult:
    """Convenience: run a ``workloads.Workload``."""
    args = dict(rel_tol=wl.rel_tol, abs_tol=wl.abs_tol,
                init_splits=wl.init_splits, max_iters=wl.max_iters,
                relerr_filter=wl.relerr_filter,
                threshold_filter=wl.threshold_filter,
                max_regions=wl.max_regions)
    args.update(kw)
    return integrate(wl.family, wl.d, wl.params, wl.lo, wl.hi, **args)


__all__ = ["lib", "npoints", "rule", "f", "eval_regions", "two_level",
           "classify", "csum", "threshold_search", "filter_split",
           "uniform_split", "integrate", "integrate_workload", "OracleResult",
           "grad_f", "grad_regions", "null_rules", "ERROR_RULE",
           "RegionEval", "FAMILY_ID", "STATUS", "PMAX_RELAX", "BUDGET", "threads"]
