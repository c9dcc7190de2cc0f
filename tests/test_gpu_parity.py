"""GPU parity: the HIP library (through the C-ABI) against the CPU oracle.

Each test prints the case it runs before touching the GPU.
"""
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import closed_forms as cf

from parity import assert_region_parity, check_free_run, rel_close, search_diff

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_06494_amd as pg
    torch.cuda.set_device(0)
    c = pg.Context(capacity=1 << 21, dim_max=10)
    yield c
    c.close()


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _params(family, d, seed):
    if family == "product_peak":
        return W.product_peak_params(d, seed)
    if family == "gaussian":
        return W.gaussian_params(d, seed)
    if family == "oscillatory":
        return W.oscillatory_params(d, seed)
    return W.corner_peak_params(d, seed)


# ---------------------------------------------------------------------------
# The integrands alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("family,d", [("product_peak", 3), ("gaussian", 5),
                                      ("oscillatory", 8), ("corner_peak", 6)])
def test_integrand_values(ctx, family, d):
    _say("integrand", family, d)
    p = _params(family, d, seed=21)
    x = np.random.default_rng(d).uniform(0, 1, size=(d, 3000))
    y = ctx.integrand_values(family, p, _dev(x)).cpu().numpy()
    ref = np.array([oracle.f(family, p, x[:, i]) for i in range(x.shape[1])])
    # a few ulps of each function, amplified by its argument's rounding
    np.testing.assert_allclose(y, ref, rtol=2e-13, atol=0)


def test_gaussian_exponential_to_two_ulps(ctx):
    """The Gaussian's e^-s over the whole range s in [0, 745] (and beyond,
    where it is 0), against the oracle (glibc): within 2 ulps plus the
    rounding of s itself (|s| ulps of e^-s), denormals by their spacing."""
    _say("integrand exp range")
    d = 2
    p = np.array([1.0, 1.0, 0.0, 0.0])                 # f = exp(-(x1^2 + x2^2))
    rng = np.random.default_rng(17)
    r = np.concatenate([rng.uniform(0, 2, 4000), rng.uniform(0, 27.4, 4000),
                        [0.0, 27.3, 27.5, 30.0]])
    ang = rng.uniform(0, np.pi / 2, r.size)
    x = np.stack([r * np.cos(ang), r * np.sin(ang)])
    y = ctx.integrand_values("gaussian", p, _dev(x)).cpu().numpy()
    ref = np.array([oracle.f("gaussian", p, x[:, i]) for i in range(x.shape[1])])
    s = (x ** 2).sum(axis=0)
    ulp = np.spacing(np.maximum(np.abs(ref), np.finfo(float).tiny))
    tol = (2.0 + 2.0 * s) * ulp + 2 * np.spacing(0.0)
    assert np.all(np.abs(y - ref) <= tol), np.max(np.abs(y - ref) / ulp)
    assert y[-1] == 0.0 and ref[-1] == 0.0


@pytest.mark.parametrize("family,d", [("product_peak", 3), ("product_peak", 8),
                                      ("corner_peak", 2), ("corner_peak", 6),
                                      ("corner_peak", 10)])
def test_peak_reciprocal_to_a_few_ulps(ctx, family, d):
    """The peaks' 1/denominator (refined hardware reciprocal) against the
    oracle's divisions and pow: within the rounding the two sides' different
    operation orders allow (a few ulps per factor of the product peak, the
    (d+1)-fold power of the sum's rounding for the corner peak)."""
    _say("integrand reciprocal", family, d)
    p = _params(family, d, seed=23)
    x = np.random.default_rng(40 + d).uniform(0, 1, size=(d, 4000))
    y = ctx.integrand_values(family, p, _dev(x)).cpu().numpy()
    ref = np.array([oracle.f(family, p, x[:, i]) for i in range(x.shape[1])])
    ulps = np.abs(y - ref) / np.spacing(np.abs(ref))
    bound = 4 * d + 4 if family == "product_peak" else (d + 1) ** 2 + 4
    assert ulps.max() <= bound, (ulps.max(), bound)


# ---------------------------------------------------------------------------
# EVALUATE
# ---------------------------------------------------------------------------

# every dimension the kernels are instantiated for (2..10), ragged tails
CASES = [(fam, d, n) for fam in ("product_peak", "gaussian", "oscillatory", "corner_peak")
         for d, n in ((2, 1), (3, 65), (4, 130), (5, 1000), (6, 3001), (7, 257),
                      (8, 777), (9, 65), (10, 129))]


@pytest.mark.parametrize("family,d,n", CASES)
def test_evaluate_parity(ctx, family, d, n):
    _say("evaluate", family, d, n)
    p = _params(family, d, seed=10 + d)
    lo, w = W.random_boxes(d, n, seed=100 + d + n)
    V, E, K = ctx.evaluate(family, p, _dev(lo), _dev(w))
    torch.cuda.synchronize()
    ref = oracle.eval_regions(family, d, p, lo, w)
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


@pytest.mark.parametrize("family,d,n", [("gaussian", 5, 200_000), ("oscillatory", 8, 140_000),
                                        ("product_peak", 3, 200_000),
                                        ("corner_peak", 6, 140_000)])
def test_evaluate_parity_one_wave_per_block(ctx, family, d, n):
    """Lists long enough that each block runs a single wave."""
    _say("evaluate-large", family, d, n)
    p = _params(family, d, seed=3)
    lo, w = W.random_boxes(d, n, seed=7, dyadic_bits=12)
    V, E, K = ctx.evaluate(family, p, _dev(lo), _dev(w))
    torch.cuda.synchronize()
    ref = oracle.eval_regions(family, d, p, lo, w)
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


VERTEX_CASES = [(d, a, g) for d in (5, 8) for a in (10.0, 1e3, 3e4)
                for g in (0.5, 3.0, 10.0, 30.0)]


@pytest.mark.parametrize("d,a_scale,g", VERTEX_CASES)
def test_gaussian_vertex_points_at_extremes(ctx, d, a_scale, g):
    """The Gaussian at its sharpest (a up to 3e4, the documented limit) on
    boxes whose vertex points lie g Gaussian widths from the centre along
    every axis (lambda5 a h = g), half of them with a vertex exactly on the
    peak u. Exponents reach hundreds, so f = e^-s magnifies any difference
    in how a point's coordinates round: an ulp in x_k moves s by
    2 a^2 t_k ulp(x_k), about 1e-12 of f here (the size of the difference a
    fused c + lambda h, one rounding instead of two, made). Per-region
    parity with the oracle's point-by-point values to the usual bound
    (1e-12 relative plus the oracle's rounding floor)."""
    _say("vertex-extremes", d, a_scale, g)
    rng = np.random.default_rng(int(d * 1000 + g))
    n = 512
    a = a_scale * rng.uniform(0.5, 1.5, size=d)
    u = rng.uniform(0.3, 0.7, size=d)
    lam5 = np.sqrt(9.0 / 19.0)
    h = g / (lam5 * a[:, None]) * rng.uniform(0.8, 1.25, size=(d, n))
    c = u[:, None] + h * lam5 * rng.choice([-1.0, 1.0], size=(d, n))
    c[:, n // 2:] += h[:, n // 2:] * rng.uniform(-0.5, 0.5, size=(d, n - n // 2))
    lo, w = c - h, 2.0 * h
    p = np.concatenate([a, u])
    V, E, K = ctx.evaluate("gaussian", p, _dev(lo), _dev(w))
    torch.cuda.synchronize()
    ref = oracle.eval_regions("gaussian", d, p, lo, w)
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


def test_evaluate_strided_rows(ctx):
    """Rows of lo/w taken from a wider buffer (leading dimension > n)."""
    d, n, ld = 4, 300, 512
    _say("evaluate-strided", d, n, ld)
    p = _params("gaussian", d, seed=1)
    lo, w = W.random_boxes(d, n, seed=2)
    blo = torch.zeros(d, ld, dtype=torch.float64, device="cuda")
    bw = torch.zeros_like(blo)
    blo[:, :n] = _dev(lo)
    bw[:, :n] = _dev(w)
    V, E, K = ctx.evaluate("gaussian", p, blo[:, :n], bw[:, :n])
    ref = oracle.eval_regions("gaussian", d, p, lo, w)
    assert_region_parity(ref, lo, w, V.cpu().numpy(), E.cpu().numpy(), K.cpu().numpy())


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_evaluate_exact_on_monomials(ctx, d):
    """Independent of the oracle: the degree-7 rule is exact on monomials of
    degree <= 7 and its null rule vanishes up to degree 5 (exact rationals)."""
    _say("monomial-exactness", d)
    from itertools import combinations_with_replacement
    lo = np.array([[-0.5], [0.25], [0.0], [-1.0], [0.5], [0.125], [-0.25], [0.0]])[:d]
    w = np.array([[1.0], [0.5], [0.25], [2.0], [0.5], [1.0], [0.75], [0.5]])[:d]
    for deg in (0, 1, 3, 5, 6, 7):
        for combo in combinations_with_replacement(range(d), deg):
            alpha = [0] * d
            for i in combo:
                alpha[i] += 1
            V, E, K = ctx.evaluate("monomial", np.array(alpha, float), _dev(lo), _dev(w))
            v, e = float(V[0]), float(E[0])
            exact = cf.monomial(alpha, lo[:, 0], lo[:, 0] + w[:, 0])
            scale = float(cf.monomial([2 * a for a in alpha], lo[:, 0] - 1e-300,
                                      lo[:, 0] + w[:, 0])) ** 0.5 + 1e-30
            assert abs(Fraction(v) - exact) <= Fraction(1e-13) * Fraction(scale) * 50, (alpha, v, float(exact))
            if deg <= 5:
                assert e <= 1e-13 * scale * 50, (alpha, e)


def test_evaluate_empty_and_invalid(ctx):
    _say("evaluate-edge")
    import paper_2104_06494_amd as pg
    z = torch.zeros(3, 0, dtype=torch.float64, device="cuda")
    V, E, K = ctx.evaluate("gaussian", _params("gaussian", 3, 1), z, z)
    assert V.numel() == 0
    with pytest.raises(pg.PaganiError):
        ctx.evaluate("gaussian", np.ones(5), _dev(np.zeros((3, 4))), _dev(np.ones((3, 4))))
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 11, np.ones(22))


# ---------------------------------------------------------------------------
# TWO-LEVEL + CLASSIFY, THRESHOLD, FILTER + SPLIT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,paired", [(1, 0), (4097, 0), (2, 1), (2 * 5003, 1),
                                      (2 * 70000, 1)])
def test_classify_parity(ctx, n, paired):
    _say("classify", n, paired)
    rng = np.random.default_rng(n)
    V = rng.lognormal(size=n) * 1e-5
    E = V * 10.0 ** rng.uniform(-9, -3, size=n)
    E[::17] = 0.0
    tau = 1e-6
    Vp = None
    if paired:
        m = n // 2
        Vp = V[:m] + V[m:] + rng.normal(scale=1e-9, size=m)
    Vd, Ed = _dev(V), _dev(E)
    A, sums = ctx.classify(Vd, Ed, _dev(Vp) if paired else None, paired=bool(paired),
                           rel_tol=tau)
    E_ref = oracle.two_level(V, E, Vp) if paired else E
    A_ref = oracle.classify(V, E_ref, tau)
    np.testing.assert_allclose(Ed.cpu().numpy(), E_ref, rtol=4e-16, atol=0)
    np.testing.assert_array_equal(A.cpu().numpy(), A_ref)
    ref = [oracle.csum(V), oracle.csum(E_ref), oracle.csum(V, A_ref),
           oracle.csum(E_ref, A_ref), float(A_ref.sum()), E_ref.min(), E_ref.max(),
           oracle.csum(V, 1 - A_ref)]
    for k in (0, 1, 2, 3, 7):
        assert rel_close(sums[k], ref[k], 1e-13), (k, sums[k], ref[k])
    assert sums[4:7] == ref[4:7]


@pytest.mark.parametrize("seed,relax", [(0, 0), (1, 1), (2, 0), (3, 1), (4, 0),
                                        (5, 1), (6, 1)])
def test_threshold_search_parity(ctx, seed, relax):
    """Seeds 5 and 6 keep part of the allowance back for the active regions
    (the reserve of a search started by the settled-digits trigger)."""
    _say("threshold", seed, relax)
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1000, 60000))
    E = rng.lognormal(sigma=2.5, size=n) * 1e-9
    A_rel = (rng.uniform(size=n) < 0.9).astype(np.uint8)
    v = 1.8e-5
    tau = float(10.0 ** rng.uniform(-7, -4))
    e_it = oracle.csum(E)
    e_f = float(rng.uniform(0, 0.3)) * tau * v
    reserve = float(rng.uniform(0, 0.4)) * tau * v if seed >= 5 else 0.0
    allow = tau * v - reserve - e_f
    ok, A, t, trials = ctx.threshold_search(_dev(E), _dev(A_rel, torch.uint8), e_it,
                                            allow, relax)
    rok, rA, rt, rtrials, _ = oracle.threshold_search(E, A_rel, e_it, allow, relax)
    assert (ok, trials) == (rok, rtrials)
    if ok:
        assert rel_close(t, rt, 1e-12)
        diff = np.flatnonzero(A.cpu().numpy() != rA)
        assert all(abs(E[i] - rt) <= 1e-12 * rt for i in diff)
    else:
        np.testing.assert_array_equal(A.cpu().numpy(), A_rel)


THRESH_SPREAD = [(seed, relax, sigma) for seed in (11, 12, 13) for relax in (0, 1)
                 for sigma in (0.2, 1.0, 5.0)]


@pytest.mark.parametrize("seed,relax,sigma", THRESH_SPREAD)
def test_threshold_search_spread(ctx, seed, relax, sigma):
    """Narrow and wide error spreads: many regions share a histogram bin
    (undecided trials, exact passes) or the search runs long (direction
    changes, P_max growth, its limits)."""
    _say("threshold-spread", seed, relax, sigma)
    rng = np.random.default_rng(seed * 7 + relax)
    n = int(rng.integers(3000, 200000))
    v = 1.8e-5
    tau = float(10.0 ** rng.uniform(-8, -3))
    # errors summing to 1.2 to 4 times the tolerance: searches that succeed
    # after 1 or about 30 trials and ones that end at the direction-change
    # or trial limits
    E = rng.lognormal(sigma=sigma, size=n)
    E *= float(rng.uniform(1.2, 4.0)) * tau * v / E.sum()
    A_rel = (rng.uniform(size=n) < 0.8).astype(np.uint8)
    e_it = oracle.csum(E)
    e_f = float(rng.uniform(0, 0.5)) * tau * v
    reserve = float(rng.uniform(0, 0.3)) * tau * v if seed == 13 else 0.0
    allow = tau * v - reserve - e_f
    ok, A, t, trials = ctx.threshold_search(_dev(E), _dev(A_rel, torch.uint8), e_it,
                                            allow, relax)
    rok, rA, rt, rtrials, _ = oracle.threshold_search(E, A_rel, e_it, allow, relax)
    assert (ok, trials) == (rok, rtrials)
    if ok:
        assert rel_close(t, rt, 1e-12)
        diff = np.flatnonzero(A.cpu().numpy() != rA)
        assert all(abs(E[i] - rt) <= 1e-12 * rt for i in diff)
    else:
        np.testing.assert_array_equal(A.cpu().numpy(), A_rel)


@pytest.mark.parametrize("d,n", [(2, 1), (3, 2049), (4, 700), (5, 4096), (6, 3001),
                                 (7, 1025), (8, 10001), (9, 129), (10, 5000)])
def test_filter_split_bit_exact(ctx, d, n):
    _say("filter-split", d, n)
    rng = np.random.default_rng(d * n)
    lo, w = W.random_boxes(d, n, seed=n, dyadic_bits=20)
    K = rng.integers(0, d, size=n).astype(np.uint8)
    V = rng.normal(size=n)
    A = (rng.uniform(size=n) < 0.55).astype(np.uint8)
    lo2, w2, Vp = ctx.filter_split(_dev(lo), _dev(w), _dev(K, torch.uint8), _dev(V),
                                   _dev(A, torch.uint8))
    rlo, rw, rVp = oracle.filter_split(d, lo, w, K, V, A)
    np.testing.assert_array_equal(lo2.cpu().numpy(), rlo)
    np.testing.assert_array_equal(w2.cpu().numpy(), rw)
    np.testing.assert_array_equal(Vp.cpu().numpy(), rVp)


def test_filter_split_none_active(ctx):
    _say("filter-split-empty")
    d, n = 3, 100
    lo, w = W.random_boxes(d, n, seed=1)
    z = torch.zeros(n, dtype=torch.uint8, device="cuda")
    lo2, w2, Vp = ctx.filter_split(_dev(lo), _dev(w), z, _dev(np.ones(n)), z)
    assert lo2.shape == (d, 0) and Vp.numel() == 0


# ---------------------------------------------------------------------------
# Whole runs: oracle replays the GPU's decision trace
# ---------------------------------------------------------------------------

def _replay(ctx, wl, tmp_path, **kw):
    trace = str(tmp_path / "trace.bin")
    r = ctx.integrate_workload(wl, trace_path=trace, **kw)
    o = oracle.integrate_workload(wl, replay_path=trace, **kw)
    return r, o


def _assert_replay(r, o, rel=1e-10):
    rep = o.replay
    hard = {k: v for k, v in rep.items() if k.endswith("_hard") and v}
    assert not hard, (hard, search_diff(rep))
    assert r.status == o.status and r.iterations == o.iterations
    assert r.regions_evaluated == o.regions_evaluated
    assert rel_close(r.estimate, o.estimate, rel), (r.estimate, o.estimate)
    assert rel_close(r.error, o.error, rel), (r.error, o.error)


REPLAY = [
    ("product_peak_d3", lambda: W.product_peak_d3(), {}),
    ("product_peak_d3_1e-6", lambda: W.product_peak_d3(), dict(rel_tol=1e-6)),
    ("gaussian_d5_1e-4", lambda: W.gaussian_d5(), dict(rel_tol=1e-4)),
    ("oscillatory_d8_relerr_off", lambda: W.oscillatory_d8(0), {}),
    ("oscillatory_d8_relerr_on", lambda: W.oscillatory_d8(1), {}),
    ("gaussian_d5_max_iters", lambda: W.gaussian_d5(), dict(max_iters=3)),
    ("gaussian_d5_memory", lambda: W.gaussian_d5(), dict(max_regions=3000,
                                                         threshold_filter=0)),
]


# (P_max rule, search budget): the defaults, the listing's budget without a
# reserve, and the memory-only P_max rule
RULES = [("paper", "reserve"), ("paper", "listing"), ("memory", "reserve")]


@pytest.mark.parametrize("pmax,budget", RULES)
@pytest.mark.parametrize("name,mk,kw", REPLAY, ids=[c[0] for c in REPLAY])
def test_integrate_replay(ctx, tmp_path, name, mk, kw, pmax, budget):
    _say("replay", name, pmax, budget)
    wl = mk()
    r, o = _replay(ctx, wl, tmp_path, pmax_relax=pmax, budget=budget, **kw)
    _assert_replay(r, o)
    sign_changing = wl.family == "oscillatory" and wl.relerr_filter
    if r.status_name in ("OK", "NO_ACTIVE") and not sign_changing:
        exact = cf.exact(wl.family, wl.params, wl.d)
        tau = kw.get("rel_tol", wl.rel_tol)
        check_free_run(r, exact, tau,
                       allow_no_active=(pmax, budget) == ("paper", "listing"))


@pytest.mark.parametrize("pmax,budget", RULES)
def test_headline_workload_replay(ctx, tmp_path, pmax, budget):
    """d=5 Gaussian to 1e-6 with the 2^21-region cap: replay parity, the
    closed form met, the memory trigger fired (the list reached the cap).
    With the P_max rule of Section 3.5.3 and no reserve for the active
    regions the run ends with every region finished and the summed error
    just above the tolerance (NO_ACTIVE); with the reserve (the default),
    or under the memory-only P_max rule, it converges."""
    _say("replay-headline", pmax, budget)
    wl = W.gaussian_d5()
    r, o = _replay(ctx, wl, tmp_path, pmax_relax=pmax, budget=budget)
    _assert_replay(r, o)
    exact = cf.exact(wl.family, wl.params, wl.d)
    listing = (pmax, budget) == ("paper", "listing")
    check_free_run(r, exact, wl.rel_tol, allow_no_active=listing)
    assert r.status_name == ("NO_ACTIVE" if listing else "OK")
    assert r.peak_regions == wl.max_regions


def test_headline_sampled_regions(ctx):
    """Full-size run as the benchmark times it; then the live list of its last
    iteration is sampled and every sampled region is evaluated by the oracle
    (V and K come from the run itself; E is re-evaluated raw on the whole
    list, which is as long as the run's largest launches)."""
    _say("headline-sampled")
    wl = W.gaussian_d5()
    r = ctx.integrate_workload(wl)
    L = ctx.last_regions()
    n = L["n"]
    assert n > 100_000
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(n, size=3000, replace=False))
    lo = L["lo"].cpu().numpy()
    w = L["w"].cpu().numpy()
    V = L["V"].cpu().numpy()
    K = L["K"].cpu().numpy()
    lo_full, w_full = L["lo"].contiguous(), L["w"].contiguous()
    V2, E2, K2 = ctx.evaluate(wl.family, wl.params, lo_full, w_full)
    ref = oracle.eval_regions(wl.family, wl.d, wl.params, lo[:, idx], w[:, idx])
    assert_region_parity(ref, lo[:, idx], w[:, idx], V[idx], E2.cpu().numpy()[idx],
                         K[idx])
    np.testing.assert_array_equal(V2.cpu().numpy(), V)       # same kernel, same bits
    # boxes lie inside the unit cube and their volume does not exceed it
    assert (lo >= 0).all() and (lo + w <= 1).all()
    assert np.prod(w, axis=0).sum() <= 1.0


def test_runs_are_bitwise_reproducible(ctx):
    _say("determinism")
    wl = W.gaussian_d5()
    r1 = ctx.integrate_workload(wl, rel_tol=1e-5)
    r2 = ctx.integrate_workload(wl, rel_tol=1e-5)
    assert (r1.estimate, r1.error, r1.regions_evaluated) == \
        (r2.estimate, r2.error, r2.regions_evaluated)


def test_integrate_on_a_side_stream(ctx):
    """A run queued on another torch stream (the context follows the current
    stream; the host polls the totals the reduce kernels leave in mapped
    memory) is the same run, with or without timing events."""
    _say("side-stream")
    wl = W.gaussian_d5()
    r0 = ctx.integrate_workload(wl, rel_tol=1e-5)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        r1 = ctx.integrate_workload(wl, rel_tol=1e-5)
        r2 = ctx.integrate_workload(wl, rel_tol=1e-5, timing=2)
    side.synchronize()
    for r in (r1, r2):
        assert (r.status, r.iterations, r.regions_evaluated, r.estimate, r.error) == \
            (r0.status, r0.iterations, r0.regions_evaluated, r0.estimate, r0.error)
    assert all(x > 0 for x in r2.phase_ms) and r2.phase_ms[0] < 1e3


def test_integrate_invalid_arguments(ctx):
    _say("integrate-invalid")
    import paper_2104_06494_amd as pg
    p = W.gaussian_params(3, 1)
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, p, lo=[0, 0, 1], hi=[1, 1, 1])
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, p, rel_tol=0, abs_tol=0)
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, p, init_splits=200)          # 200^3 > cap
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, p, max_regions=1 << 30)      # above capacity
    with pytest.raises(pg.PaganiError):
        ctx.integrate("gaussian", 3, p[:5])                        # wrong params
