"""Python front end of the PAGANI library: same operations as include/pagani.h.

All arrays are PyTorch CUDA (HIP) tensors; work is queued on the current
torch stream. Integrands are a family name plus a parameter vector (see
include/pagani.h for the layouts).
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


class PaganiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{L.STATUS.get(code, code)}: {msg}")
        self.code = code


def _stream_handle(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _error_rule(rule):
    if isinstance(rule, str):
        if rule not in L.ERROR_RULE:
            raise ValueError(f"error_rule must be one of {sorted(L.ERROR_RULE)}")
        return L.ERROR_RULE[rule]
    return int(rule)


def _pmax_relax(mode):
    if isinstance(mode, str):
        if mode not in L.PMAX_RELAX:
            raise ValueError(f"pmax_relax must be one of {sorted(L.PMAX_RELAX)}")
        return L.PMAX_RELAX[mode]
    return int(mode)


def _budget(mode):
    if isinstance(mode, str):
        if mode not in L.BUDGET:
            raise ValueError(f"budget must be one of {sorted(L.BUDGET)}")
        return L.BUDGET[mode]
    return int(mode)


def _integrand(family, d, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    arr = (C.c_double * len(p))(*p.tolist())
    f = L.Integrand(L.FAMILY_ID[family] if isinstance(family, str) else int(family),
                    int(d), C.cast(arr, C.POINTER(C.c_double)), len(p))
    return f, arr          # keep arr alive with f


def _check_f64(t, name, device):
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64
            and t.device == device and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on {device}")


def _check_u8(t, name, device):
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.uint8
            and t.device == device and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous uint8 tensor on {device}")


@dataclass
class IntegrateResult:
    estimate: float
    error: float
    status: int
    status_name: str
    iterations: int
    regions_evaluated: int
    fevals: int
    peak_regions: int
    threshold_calls: int
    threshold_trials: int
    phase_ms: list
    eval_launches: int


class Context:
    """A device workspace for region lists of up to `capacity` regions of up
    to `dim_max` dimensions. The workspace is a torch uint8 tensor."""

    def __init__(self, capacity: int = 1 << 22, dim_max: int = L.PG_DIM_MAX,
                 device=None):
        self.lib = L.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) \
            if device is None else torch.device(device)
        nbytes = self.lib.pg_workspace_bytes(dim_max, capacity)
        if nbytes == 0:
            raise ValueError("bad dim_max / capacity")
        # 256-byte aligned view into a slightly larger tensor
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self.ws = self._ws[off:off + nbytes]
        self.capacity, self.dim_max = capacity, dim_max
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.pg_context_create(self.device.index, dim_max, capacity,
                                            _ptr(self.ws), nbytes,
                                            _stream_handle(self.device), C.byref(h))
        if rc != 0:
            raise PaganiError(rc, "pg_context_create failed")
        self.h = h
        _live.add(self)

    def close(self):
        """Destroys the C context (waits for its stream, frees its pinned
        host memory). Idempotent; contexts still open when the interpreter
        exits are closed by an exit handler while HIP is still up."""
        if getattr(self, "h", None):
            with torch.cuda.device(self.device):
                self.lib.pg_context_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # nothing to do once closed; during interpreter shutdown (when even
        # module globals may be gone, hence the bound default) the HIP
        # runtime may already be going away: leave the context to the
        # process exit instead of calling into HIP from a finaliser
        if not getattr(self, "h", None) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_eval_waves(self, target: int = 0):
        """Waves EVALUATE aims to keep in flight (0: the default, 2048);
        changes the order of the waves' partial sums, not the rule."""
        rc = self.lib.pg_context_set_eval_waves(self.h, int(target))
        if rc:
            raise self._err(rc)

    # -- helpers ----------------------------------------------------------
    def _bind_stream(self):
        self.lib.pg_context_set_stream(self.h, _stream_handle(self.device))

    def _soa_ld(self, lo, w):
        """Leading dimension of a [d, n] structure-of-arrays pair."""
        for t, nm in ((lo, "lo"), (w, "w")):
            if not (t.dtype == torch.float64 and t.device == self.device
                    and t.dim() == 2 and t.stride(1) == 1):
                raise TypeError(f"{nm} must be a [d, n] float64 tensor on "
                                f"{self.device} with unit column stride")
        if lo.shape != w.shape:
            raise TypeError("lo and w differ in shape")
        d, n = lo.shape
        ld = lo.stride(0) if d > 1 else n
        if d > 1 and w.stride(0) != ld:
            raise TypeError("lo and w must share their row stride")
        return ld

    def _err(self, rc):
        return PaganiError(rc, self.lib.pg_last_error(self.h).decode())

    # -- whole run -------------------------------------------------------
    def integrate(self, family, d, params, lo=None, hi=None, rel_tol=1e-3,
                  abs_tol=1e-20, init_splits=4, max_iters=100, relerr_filter=1,
                  threshold_filter=1, max_regions=0, timing=False,
                  trace_path=None, error_rule="raw",
                  pmax_relax="paper", budget="reserve") -> IntegrateResult:
        """Algorithm 2 over the box [lo, hi] (default unit cube). error_rule
        "raw" (|R7 - R5|) or "null4" (the four-null-rule estimate);
        pmax_relax "paper" (P_max grows at every direction change of a
        threshold search, Section 3.5.3) or "memory" (only in searches under
        memory pressure); budget "reserve" (a search started because the
        estimate's digits have settled keeps back the error the active
        regions may still end with, Lemma 1) or "listing" (nothing kept
        back)."""
        self._bind_stream()
        f, keep = _integrand(family, d, params)
        lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
        hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
        clo = (C.c_double * d)(*lo.tolist())
        chi = (C.c_double * d)(*hi.tolist())
        o = L.Options()
        self.lib.pg_default_options(C.byref(o))
        o.rel_tol, o.abs_tol = float(rel_tol), float(abs_tol)
        o.init_splits, o.max_iters = int(init_splits), int(max_iters)
        o.relerr_filter, o.threshold_filter = int(relerr_filter), int(threshold_filter)
        # timing: False / 0 none, 1 the EVALUATE launches, True / 2 every phase
        o.max_regions = int(max_regions)
        o.timing = 2 if timing is True else int(timing)
        o.trace_path = trace_path.encode() if trace_path else None
        o.error_rule = _error_rule(error_rule)
        o.pmax_relax = _pmax_relax(pmax_relax)
        o.budget = _budget(budget)
        r = L.Result()
        with torch.cuda.device(self.device):
            rc = self.lib.pg_integrate(self.h, C.byref(f), clo, chi, C.byref(o),
                                       C.byref(r))
        if rc < 0:
            raise self._err(rc)
        return IntegrateResult(**r.as_dict())

    def integrate_batch(self, family, d, params, rel_tol, abs_tol=None,
                        lo=None, hi=None, init_splits=4, max_iters=100,
                        relerr_filter=1, threshold_filter=1, max_regions=0,
                        error_rule="raw", pmax_relax="paper", budget="reserve"):
        """Algorithm 2 for B integrals of one family at once: params is
        [B, n_params], rel_tol a scalar or [B], abs_tol None (1e-20), a
        scalar or [B]; all share the box [lo, hi] and the options, and
        max_regions is the cap of each. Returns a list of B results."""
        return self._batch(family, d, params, rel_tol, abs_tol, lo, hi, init_splits,
                           max_iters, relerr_filter, threshold_filter, max_regions,
                           error_rule=error_rule, pmax_relax=pmax_relax,
                           budget=budget)[0]

    def integrate_batch_grad(self, family, d, params, rel_tol, abs_tol=None,
                             lo=None, hi=None, init_splits=4, max_iters=100,
                             relerr_filter=1, threshold_filter=1, max_regions=0,
                             leaves_capacity=0, error_rule="raw",
                             pmax_relax="paper", budget="reserve"):
        """integrate_batch plus dI/dparams of every integral over its final
        partition: returns (results, grad [B, n_params] numpy, leaves). With
        leaves_capacity > 0, leaves is a dict of device tensors lo, w [d, n]
        and owner [n] (the partition's regions); otherwise None."""
        return self._batch(family, d, params, rel_tol, abs_tol, lo, hi, init_splits,
                           max_iters, relerr_filter, threshold_filter, max_regions,
                           grad=True, leaves_capacity=leaves_capacity,
                           error_rule=error_rule, pmax_relax=pmax_relax,
                           budget=budget)

    def integrate_grad(self, family, d, params, lo=None, hi=None, rel_tol=1e-3,
                       abs_tol=1e-20, init_splits=4, max_iters=100, relerr_filter=1,
                       threshold_filter=1, max_regions=0, leaves_capacity=0,
                       error_rule="raw", pmax_relax="paper", budget="reserve"):
        """One integral and its parameter derivative through the C entry
        point pg_integrate_grad: returns (result, grad [n_params], leaves)."""
        self._bind_stream()
        f, keep = _integrand(family, d, params)
        lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
        hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
        clo = (C.c_double * d)(*lo.tolist())
        chi = (C.c_double * d)(*hi.tolist())
        o = L.Options()
        self.lib.pg_default_options(C.byref(o))
        o.rel_tol, o.abs_tol = float(rel_tol), float(abs_tol)
        o.init_splits, o.max_iters = int(init_splits), int(max_iters)
        o.relerr_filter, o.threshold_filter = int(relerr_filter), int(threshold_filter)
        o.max_regions = int(max_regions)
        o.error_rule = _error_rule(error_rule)
        o.pmax_relax = _pmax_relax(pmax_relax)
        o.budget = _budget(budget)
        g = np.zeros(f.n_params)
        lv, lt = self._leaves(d, leaves_capacity)
        r = L.Result()
        with torch.cuda.device(self.device):
            rc = self.lib.pg_integrate_grad(self.h, C.byref(f), clo, chi, C.byref(o),
                                            C.byref(r), g.ctypes.data_as(C.POINTER(C.c_double)),
                                            C.byref(lv) if lv is not None else None)
        if rc < 0:
            raise self._err(rc)
        return IntegrateResult(**r.as_dict()), g, self._leaves_view(lv, lt)

    def _leaves(self, d, cap):
        if not cap:
            return None, None
        cap = int(cap)
        lo = torch.empty((d, cap), dtype=torch.float64, device=self.device)
        w = torch.empty((d, cap), dtype=torch.float64, device=self.device)
        owner = torch.empty(cap, dtype=torch.int32, device=self.device)
        lv = L.Leaves(lo.data_ptr(), w.data_ptr(), owner.data_ptr(), cap, 0)
        return lv, (lo, w, owner)

    @staticmethod
    def _leaves_view(lv, lt):
        if lv is None:
            return None
        lo, w, owner = lt
        n = lv.n
        return {"n": n, "lo": lo[:, :n], "w": w[:, :n], "owner": owner[:n]}

    def _batch(self, family, d, params, rel_tol, abs_tol, lo, hi, init_splits,
               max_iters, relerr_filter, threshold_filter, max_regions, grad=False,
               leaves_capacity=0, error_rule="raw", pmax_relax="paper",
               budget="reserve"):
        self._bind_stream()
        P = np.ascontiguousarray(np.atleast_2d(np.asarray(params, dtype=np.float64)))
        B, npar = P.shape
        rt = np.ascontiguousarray(np.broadcast_to(np.asarray(rel_tol, np.float64), (B,)))
        lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
        hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
        cp = P.ravel().ctypes.data_as(C.POINTER(C.c_double))
        crt = rt.ctypes.data_as(C.POINTER(C.c_double))
        clo = (C.c_double * d)(*lo.tolist())
        chi = (C.c_double * d)(*hi.tolist())
        at = None
        cat = None
        if abs_tol is not None:
            at = np.ascontiguousarray(np.broadcast_to(np.asarray(abs_tol, np.float64), (B,)))
            cat = at.ctypes.data_as(C.POINTER(C.c_double))
        o = L.Options()
        self.lib.pg_default_options(C.byref(o))
        o.init_splits, o.max_iters = int(init_splits), int(max_iters)
        o.relerr_filter, o.threshold_filter = int(relerr_filter), int(threshold_filter)
        o.max_regions = int(max_regions)
        o.error_rule = _error_rule(error_rule)
        o.pmax_relax = _pmax_relax(pmax_relax)
        o.budget = _budget(budget)
        res = (L.Result * B)()
        fam = L.FAMILY_ID[family] if isinstance(family, str) else int(family)
        g = np.zeros((B, npar)) if grad else None
        lv, lt = self._leaves(d, leaves_capacity) if grad else (None, None)
        with torch.cuda.device(self.device):
            if grad:
                rc = self.lib.pg_integrate_batch_grad(
                    self.h, fam, int(d), int(B), cp, int(npar), clo, chi, crt, cat,
                    C.byref(o), res, g.ctypes.data_as(C.POINTER(C.c_double)),
                    C.byref(lv) if lv is not None else None)
            else:
                rc = self.lib.pg_integrate_batch(self.h, fam, int(d), int(B), cp,
                                                 int(npar), clo, chi, crt, cat,
                                                 C.byref(o), res)
        if rc < 0:
            raise self._err(rc)
        results = [IntegrateResult(**res[b].as_dict()) for b in range(B)]
        return results, g, self._leaves_view(lv, lt)

    def integrate_batch_workload(self, wl, count=None, grad=False, leaves_capacity=0,
                                 **kw):
        """integrate_batch (or integrate_batch_grad with grad=True) over a
        batched workload (its first `count` integrals if given); keyword
        arguments (error_rule, pmax_relax, budget) go to the integrator."""
        B = wl.B if count is None else int(count)
        fn = self.integrate_batch
        kw = dict(kw)
        if grad:
            fn = self.integrate_batch_grad
            kw["leaves_capacity"] = leaves_capacity
        return fn(wl.family, wl.d, wl.params[:B], wl.rel_tol[:B], wl.abs_tol[:B],
                  wl.lo, wl.hi, init_splits=wl.init_splits, max_iters=wl.max_iters,
                  relerr_filter=wl.relerr_filter, threshold_filter=wl.threshold_filter,
                  max_regions=wl.max_regions, **kw)

    def integrate_workload(self, wl, **kw) -> IntegrateResult:
        args = dict(rel_tol=wl.rel_tol, abs_tol=wl.abs_tol,
                    init_splits=wl.init_splits, max_iters=wl.max_iters,
                    relerr_filter=wl.relerr_filter,
                    threshold_filter=wl.threshold_filter,
                    max_regions=wl.max_regions)
        args.update(kw)
        return self.integrate(wl.family, wl.d, wl.params, wl.lo, wl.hi, **args)

    def last_regions(self):
        """The live list left by the last integrate(): dict of tensors viewing
        the workspace (lo, w as [d, n]; V, E; K, A)."""
        v = L.RegionsView()
        rc = self.lib.pg_last_regions(self.h, C.byref(v))
        if rc:
            raise self._err(rc)
        base = self.ws.data_ptr()

        def view(ptr, nbytes, dtype):
            off = ptr - base
            return self.ws[off:off + nbytes].view(dtype)

        d, n, ld = v.dim, v.n, v.ld
        lo = view(v.lo, 8 * ld * d, torch.float64).view(d, ld)[:, :n]
        w = view(v.w, 8 * ld * d, torch.float64).view(d, ld)[:, :n]
        return dict(dim=d, n=n, lo=lo, w=w,
                    V=view(v.V, 8 * n, torch.float64),
                    E=view(v.E, 8 * n, torch.float64),
                    K=view(v.K, n, torch.uint8), A=view(v.A, n, torch.uint8))

    # -- the steps of one iteration ---------------------------------------
    def evaluate(self, family, params, lo, w, error_rule="raw"):
        """EVALUATE on the boxes [lo, lo + w] (lo, w: [d, n] float64 tensors,
        rows may be a strided view with unit element stride and a common row
        stride). Returns (V, E, K); E by error_rule ("raw" or "null4")."""
        self._bind_stream()
        d, n = lo.shape
        ld = self._soa_ld(lo, w)
        V = torch.empty(n, dtype=torch.float64, device=self.device)
        E = torch.empty_like(V)
        K = torch.empty(n, dtype=torch.uint8, device=self.device)
        f, keep = _integrand(family, d, params)
        rc = self.lib.pg_evaluate_rule(self.h, C.byref(f), _error_rule(error_rule), n,
                                       _ptr(lo), _ptr(w), ld, _ptr(V), _ptr(E), _ptr(K))
        if rc:
            raise self._err(rc)
        return V, E, K

    def integrand_values(self, family, params, x):
        """f at the points x ([d, n] float64 tensor, unit column stride)."""
        self._bind_stream()
        ld = self._soa_ld(x, x)
        d, n = x.shape
        y = torch.empty(n, dtype=torch.float64, device=self.device)
        f, keep = _integrand(family, d, params)
        rc = self.lib.pg_integrand_values(self.h, C.byref(f), n, _ptr(x), ld, _ptr(y))
        if rc:
            raise self._err(rc)
        return y

    def classify(self, V, E, Vp=None, paired=False, rel_tol=1e-3, relerr_filter=1):
        """TWO-LEVEL-ERROR (paired lists, in place on E) + REL-ERR-CLASSIFY.
        Returns (A, sums) with sums = [sum V, sum E, sum AV, sum AE, sum A,
        min E, max E, sum (1 - A) V]."""
        self._bind_stream()
        n = V.numel()
        for t, nm in ((V, "V"), (E, "E")):
            _check_f64(t, nm, self.device)
        if paired:
            _check_f64(Vp, "Vp", self.device)
        A = torch.empty(n, dtype=torch.uint8, device=self.device)
        sums = (C.c_double * 8)()
        rc = self.lib.pg_classify(self.h, n, int(paired), _ptr(V), _ptr(E),
                                  _ptr(Vp) if paired else None, float(rel_tol),
                                  int(relerr_filter), _ptr(A), sums)
        if rc:
            raise self._err(rc)
        return A, list(sums)

    def threshold_search(self, E, A_rel, e_it, allowance, relax=True):
        """THRESHOLD-CLASSIFY (Algorithm 3): the finished regions' error may
        reach P_max * allowance; relax: P_max grows at each direction change
        (Section 3.5.3). Returns (ok, A, t, trials)."""
        self._bind_stream()
        _check_f64(E, "E", self.device)
        _check_u8(A_rel, "A_rel", self.device)
        A = torch.empty_like(A_rel)
        ok, t, tr = C.c_int(), C.c_double(), C.c_int()
        rc = self.lib.pg_threshold_search(self.h, E.numel(), _ptr(E), _ptr(A_rel),
                                          float(e_it), float(allowance),
                                          int(bool(relax)), _ptr(A), C.byref(ok),
                                          C.byref(t), C.byref(tr))
        if rc:
            raise self._err(rc)
        return bool(ok.value), A, t.value, tr.value

    def filter_split(self, lo, w, K, V, A):
        """FILTER + parent update + SPLIT. Returns (lo2 [d, 2na], w2, Vp[na])."""
        self._bind_stream()
        d, n = lo.shape
        ld = self._soa_ld(lo, w)
        _check_u8(K, "K", self.device)
        _check_u8(A, "A", self.device)
        _check_f64(V, "V", self.device)
        cap = max(2 * n, 2)
        lo2 = torch.empty(d, cap, dtype=torch.float64, device=self.device)
        w2 = torch.empty_like(lo2)
        Vp = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        na = C.c_int64()
        rc = self.lib.pg_filter_split(self.h, d, n, _ptr(lo), _ptr(w), ld, _ptr(K),
                                      _ptr(V), _ptr(A), _ptr(lo2), _ptr(w2), cap,
                                      _ptr(Vp), C.byref(na))
        if rc:
            raise self._err(rc)
        m = na.value
        return lo2[:, :2 * m].contiguous(), w2[:, :2 * m].contiguous(), Vp[:m].clone()


def filter_split_noalloc(lo, w, K, V, A, lo_out, w_out, Vp):
    """FILTER + parent update + SPLIT into caller-allocated outputs, without a
    context and without allocating (pg_filter_split_noalloc): lo, w are
    [d, n] and lo_out, w_out [d, ld_out] contiguous float64 with
    ld_out >= 2 n_active; Vp holds at least min(n, ld_out // 2) values.
    Queued on torch's current stream. Returns n_active."""
    lib = L.load()
    d, n = lo.shape
    dev = lo.device
    for t, name in ((lo, "lo"), (w, "w"), (V, "V"), (lo_out, "lo_out"),
                    (w_out, "w_out"), (Vp, "Vp")):
        _check_f64(t, name, dev)
    _check_u8(K, "K", dev)
    _check_u8(A, "A", dev)
    ld_out = lo_out.shape[1] if lo_out.dim() == 2 else -1
    if w.shape != lo.shape or w_out.shape != lo_out.shape or lo_out.shape[0] != d:
        raise ValueError("lo, w must be [d, n] and lo_out, w_out [d, ld_out]")
    if min(V.numel(), K.numel(), A.numel()) < n or Vp.numel() < min(n, ld_out // 2):
        raise ValueError("V, K, A need n entries and Vp min(n, ld_out // 2)")
    na = C.c_int64()
    with torch.cuda.device(dev):
        rc = lib.pg_filter_split_noalloc(_stream_handle(dev), d, n, _ptr(lo), _ptr(w),
                                         n, _ptr(K), _ptr(V), _ptr(A), _ptr(lo_out),
                                         _ptr(w_out), ld_out, _ptr(Vp), C.byref(na))
    if rc:
        raise PaganiError(rc, "pg_filter_split_noalloc failed")
    return na.value


_default_ctx = {}
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    """Closes every context still open (the cached ones included) when the
    interpreter exits: Python runs this before it tears its modules down and
    before the C runtime's exit handlers (HIP's, a profiler's) run."""
    _default_ctx.clear()
    for ctx in list(_live):
        try:
            ctx.close()
        except Exception:
            pass


def context(capacity=1 << 22, dim_max=L.PG_DIM_MAX) -> Context:
    """A cached context per (device, capacity, dim_max)."""
    key = (torch.cuda.current_device(), capacity, dim_max)
    if key not in _default_ctx:
        _default_ctx[key] = Context(capacity, dim_max)
    return _default_ctx[key]


def integrate(family, d, params, lo=None, hi=None, capacity=1 << 22, **kw):
    """One-call integration on the current device (see Context.integrate)."""
    return context(capacity).integrate(family, d, params, lo, hi, **kw)
