// dg_solver.hip -- Jacobi-preconditioned CG (FP64) and FP32 CG inside FP64
// iterative refinement.
#include "dg_internal.hpp"

using namespace dgk;

extern "C" dg_status dg_cg_solve(dg_op *, dg_vec, dg_vec, const dg_solve_params *, dg_solve_stats *, void *)
{
  return fail(DG_ERR_UNSUPPORTED, "dg_cg_solve: not built yet");
}
