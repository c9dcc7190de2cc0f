"""PAGANI on MI355X: the data-parallel adaptive integrator of Sakiotis et
al. (SC'21) as hand-written gfx950 HIP kernels behind a C interface
(include/pagani.h), with this thin Python front end.

    import paper_2104_06494_amd as pg
    r = pg.integrate("gaussian", 5, params, rel_tol=1e-6)
"""
from ._lib import FAMILY_ID, STATUS, PG_DIM_MAX, PG_DIM_MIN, LIB_PATH, load  # noqa: F401
from .api import (Context, IntegrateResult, PaganiError, context, filter_split_noalloc,  # noqa: F401
                  integrate)
from .autograd import PaganiIntegral, integral  # noqa: F401
