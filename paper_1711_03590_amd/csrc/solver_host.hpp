// solver_host.hpp -- host-side steps of the reliable-update mixed CG that
// the single-solve path and the batched path share, so that a request gets
// the same kernels, in the same order, whichever path runs it.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.hpp"
#include "solver_kernels.hpp"

namespace dgk {

// r64 = b - A x (FP64 apply), dscal[0] = ||r64||^2, r32 = r64 / nb
inline hipError_t rel_residual_async(dg_op *op, const double *b, const double *x, double *r64, double *dpart,
                                     double *dscal, float *r32, double nb, hipStream_t s)
{
  const int64_t n = op->ndofs;
  hipError_t e = launch_apply_any(op, x, r64, false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((sub_kernel<double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, b, r64, r64, n);
  hipLaunchKernelGGL((dot_partial_kernel<double, double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, r64, r64, n,
                     dpart);
  hipLaunchKernelGGL((finalize_kernel<double>), dim3(1), dim3(kRedThreads), 0, s, dpart, kRedBlocks, dscal);
  hipLaunchKernelGGL(scale_to_f32_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, r64, 1.0 / nb, r32, n);
  return hipGetLastError();
}

// e = 0; p = r / d; scal[1] = r.z, scal[2] = r.r  (first iteration uses cur = 1)
inline hipError_t start_direction_async(int64_t n, float *e, const float *r, float *p, const float *d, float *part,
                                        hipStream_t s)
{
  float *rz_part = part + kRedBlocks, *scal = part + 3 * kRedBlocks;
  hipLaunchKernelGGL((fill_kernel<float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, e, 0.0f, n);
  hipLaunchKernelGGL((rz_partial_kernel<float, float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, r, d, n, rz_part);
  hipLaunchKernelGGL((cg_pupdate_kernel<float, float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, p,
                     (float *)nullptr, r, d, n, part, rz_part, scal, 0, 0);
  return hipGetLastError();
}

// x += nb e; e = 0  (flush of the FP32 correction)
inline hipError_t flush_correction_async(int64_t n, double *x, double nb, float *e, hipStream_t s)
{
  hipLaunchKernelGGL(axpy_f32_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, nb, e, n);
  hipLaunchKernelGGL((fill_kernel<float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, e, 0.0f, n);
  return hipGetLastError();
}

// after a residual replacement: scal[cur] = r.z, scal[2] = r.r of the new r
inline hipError_t restart_rz_async(int64_t n, const float *r, const float *d, float *part, int cur, hipStream_t s)
{
  float *rz_part = part + kRedBlocks, *scal = part + 3 * kRedBlocks;
  hipLaunchKernelGGL((rz_partial_kernel<float, float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, r, d, n, rz_part);
  hipLaunchKernelGGL((rz_finalize_kernel<float>), dim3(1), dim3(kRedThreads), 0, s, rz_part, scal, cur);
  return hipGetLastError();
}

}  // namespace dgk
