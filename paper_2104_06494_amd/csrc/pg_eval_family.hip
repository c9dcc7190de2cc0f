// pg_eval_family.hip -- the EVALUATE kernels of one integrand family,
// compiled once per family with -DPG_EVAL_FAMILY=<pg_family>.
#include "pg_eval_kernels.hpp"

#ifndef PG_EVAL_FAMILY
#error "compile with -DPG_EVAL_FAMILY=<family id>"
#endif

namespace pg {
template EvalKernel eval_family<PG_EVAL_FAMILY>(int, bool);
template FvalKernel fval_family<PG_EVAL_FAMILY>(int);
}  // namespace pg
