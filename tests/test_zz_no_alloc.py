"""pg_filter_split_noalloc, the FILTER + parent update + SPLIT entry point
that allocates nothing (its scratch is a static device array per GPU),
against pg_filter_split, the context entry point it is a variant of.

Both run the same compaction on the same inputs, so their outputs must be
bit-identical (integer and copy work: the survivor count, every child's
corner and width, every parent estimate). Two calls in a row share the
static scratch, the second on a smaller list, then an empty list and a list
with no survivors; the size limit and NULL arrays are refused on the host
before anything runs (checked without a GPU)."""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _random_list(d, n, seed, p_active):
    """A list of dyadic boxes (corners and widths exact in binary), random
    split axes, estimates and active flags."""
    rng = np.random.default_rng(seed)
    level = rng.integers(1, 12, size=(d, n))
    w = np.ldexp(1.0, -level)
    lo = np.floor(rng.uniform(0.0, 1.0, size=(d, n)) / w) * w
    K = rng.integers(0, d, size=n).astype(np.uint8)
    V = rng.normal(size=n)
    A = (rng.uniform(size=n) < p_active).astype(np.uint8)
    dev = torch.device("cuda", 0)
    f64 = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    u8 = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.uint8, device=dev)
    return f64(lo), f64(w), u8(K), f64(V), u8(A)


@pytest.mark.gpu
def test_noalloc_matches_context_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_06494_amd as pg
    torch.cuda.set_device(0)
    cases = [(5, 300_001, 1, 0.6),     # 294 segments, ragged tail
             (3, 70_003, 2, 0.3),      # smaller: the scratch keeps the first
                                       # call's larger contents beyond it
             (4, 1, 3, 1.0),
             (6, 5000, 4, 0.0),        # no survivors
             (2, 0, 5, 0.5)]           # empty list
    with pg.Context(capacity=1 << 19, dim_max=6) as ctx:
        for d, n, seed, p in cases:
            _say("noalloc filter_split", f"d={d} n={n} seed={seed} p_active={p}")
            lo, w, K, V, A = _random_list(d, n, seed, p)
            ld_out = max(2 * n, 2)
            if n == 0:
                # nothing to compact: no survivors and nothing written
                lo_out = torch.full((d, ld_out), np.nan, dtype=torch.float64,
                                    device=lo.device)
                Vp = torch.full((1,), np.nan, dtype=torch.float64, device=lo.device)
                assert pg.filter_split_noalloc(lo, w, K, V, A, lo_out,
                                               lo_out.clone(), Vp) == 0
                assert torch.isnan(lo_out).all() and torch.isnan(Vp).all()
                continue
            ref_lo, ref_w, ref_Vp = ctx.filter_split(lo, w, K, V, A)
            lo_out = torch.full((d, ld_out), np.nan, dtype=torch.float64, device=lo.device)
            w_out = torch.full_like(lo_out, np.nan)
            Vp = torch.full((max(n, 1),), np.nan, dtype=torch.float64, device=lo.device)
            na = pg.filter_split_noalloc(lo, w, K, V, A, lo_out, w_out, Vp)
            torch.cuda.synchronize()
            assert na == int(A.sum().item()) == ref_Vp.numel()
            assert torch.equal(lo_out[:, :2 * na], ref_lo)
            assert torch.equal(w_out[:, :2 * na], ref_w)
            assert torch.equal(Vp[:na], ref_Vp)
            # nothing written beyond the 2 n_active children and n_active parents
            assert torch.isnan(lo_out[:, 2 * na:]).all() and torch.isnan(Vp[na:]).all()


def test_noalloc_refuses_bad_arguments_on_the_host():
    """Refused before any HIP call, so this runs without a GPU: a list above
    PG_NOALLOC_MAX_REGIONS, NULL arrays, a bad dimension, ld < n."""
    from paper_2104_06494_amd import _lib
    lib = _lib.load()
    f = lib.pg_filter_split_noalloc
    buf = (C.c_double * 4)()
    p = C.cast(buf, C.c_void_p)
    na = C.c_int64(-7)
    big = (1 << 26) + 1
    assert f(None, 3, big, p, p, big, p, p, p, p, p, 2 * big, p, C.byref(na)) == -1
    assert na.value == 0
    assert f(None, 3, 4, None, p, 4, p, p, p, p, p, 8, p, C.byref(na)) == -1
    assert f(None, 11, 4, p, p, 4, p, p, p, p, p, 8, p, C.byref(na)) == -1
    assert f(None, 3, 4, p, p, 3, p, p, p, p, p, 8, p, C.byref(na)) == -1
    assert f(None, 3, 4, p, p, 4, p, p, p, p, p, 8, p, None) == -1
