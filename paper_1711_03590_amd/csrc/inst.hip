// inst.hip -- explicit instantiation of the kernels for one number of 1D
// points, DG_N (compiled once per N = 2..9, i.e. degree 1..8).
#include "kernels.hpp"

#ifndef DG_N
#error "compile with -DDG_N=<points per direction>"
#endif

namespace dgk {
template hipError_t launch_apply<DG_N>(const dg_op *, const void *, void *, bool, hipStream_t, const void *const *);
template hipError_t launch_face_traces<DG_N>(const dg_op *, int, const void *, void *, bool, hipStream_t);
template hipError_t launch_diag<DG_N>(const dg_op *, void *, void *, hipStream_t);
template hipError_t launch_apply_dot<DG_N>(const dg_op *, const void *, void *, bool, void *, hipStream_t);
template int apply_workgroups<DG_N>(const dg_op *);
}  // namespace dgk
