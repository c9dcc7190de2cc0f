"""C-ABI checks that need no GPU: the library loads and exports every entry
point include/pagani.h declares; host-only helpers behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pagani.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pg_integrate", "pg_evaluate", "pg_classify",
                 "pg_threshold_search", "pg_filter_split", "pg_context_create",
                 "pg_context_destroy", "pg_workspace_bytes", "pg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2104_06494_amd as pg
    lib = pg.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2104_06494_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_workspace_bytes():
    import paper_2104_06494_amd as pg
    lib = pg.load()
    b = lib.pg_workspace_bytes(5, 1 << 21)
    # two ping-pong lists of lo and w dominate the part that grows with the
    # capacity (4 d cap doubles); besides it the per-integral tables of the
    # many-integral driver (error histograms and their bound tables, 1024
    # integrals) take a fixed amount, about 100 MB
    fixed = lib.pg_workspace_bytes(5, 2)
    assert 64e6 < fixed < 128e6
    assert b >= 4 * 5 * (1 << 21) * 8 + fixed
    assert b < 1.2 * (4 * 5 + 3) * (1 << 21) * 8 + fixed
    assert lib.pg_workspace_bytes(11, 100) == 0
    assert lib.pg_workspace_bytes(1, 100) == 0
    assert lib.pg_workspace_bytes(5, 1) == 0
    assert lib.pg_workspace_bytes(10, 1 << 20) > lib.pg_workspace_bytes(5, 1 << 20)


def test_default_options():
    from paper_2104_06494_amd import _lib
    lib = _lib.load()
    o = _lib.Options()
    lib.pg_default_options(C.byref(o))
    assert (o.rel_tol, o.abs_tol, o.init_splits, o.max_iters) == (1e-3, 1e-20, 4, 100)
    assert (o.relerr_filter, o.threshold_filter, o.max_regions) == (1, 1, 0)
    assert o.trace_path is None


def test_context_create_rejects_bad_arguments():
    from paper_2104_06494_amd import _lib
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.pg_context_create(0, 11, 1024, None, 0, None, C.byref(h)) == -1
    assert lib.pg_context_create(0, 5, 1, None, 0, None, C.byref(h)) == -1
    # workspace smaller than required
    assert lib.pg_context_create(0, 5, 1024, C.c_void_p(256), 16, None, C.byref(h)) == -2
    assert h.value is None


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle and fails loudly without the
    library."""
    pkg = os.path.join(ROOT, "paper_2104_06494_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src, fn


def test_eval_wave_target_needs_a_context():
    from paper_2104_06494_amd import _lib
    lib = _lib.load()
    assert lib.pg_context_set_eval_waves(None, 2048) == -1
