// solver_kernels.hpp -- BLAS-1 kernels of the CG solvers with deterministic
// reductions (fixed partition, fixed summation order).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "reduce.hpp"

namespace dgk {

constexpr int kRedBlocks = 512;   // fixed partition of every reduction
constexpr int kRedThreads = 256;

// sum over the block in a fixed order (butterfly per wave, then the waves
// in order); every thread gets the result
template <typename Acc>
__device__ __forceinline__ Acc block_sum(Acc v, Acc *sh)
{
  return workgroup_sum<kRedThreads>(v, sh);
}

// the kRedBlocks partials of one reduction, summed in a fixed order
template <typename Acc>
__device__ __forceinline__ Acc reduce_partials(const Acc *part, int stride, Acc *sh)
{
  Acc v = Acc(0);
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) v += part[i * stride];
  return block_sum(v, sh);
}

// The chunk-th piece of a reduction (chunk in [0, kRedBlocks)) covers the
// elements chunk*T + t + j*kRedBlocks*T; the kernels below run one chunk per
// workgroup, the batched kernels one chunk of one request per workgroup, so
// a request's sums do not depend on what else shares the launch.  Each
// thread takes its elements four at a time (loads first, then the
// arithmetic in the same order as one at a time), so that enough loads are
// in flight to keep HBM busy with one workgroup per chunk.
constexpr int kUnroll = 4;
constexpr int64_t kChunkStride = (int64_t)kRedBlocks * kRedThreads;
template <typename Real, typename Acc>
__device__ __forceinline__ void dot_partial_body(const Real *__restrict__ x, const Real *__restrict__ y, int64_t n,
                                                 Acc *__restrict__ part, int chunk, Acc *sh)
{
  if ((int64_t)chunk * kRedThreads >= n) {  // an empty chunk (short vectors): its partial is zero
    if (threadIdx.x == 0) part[chunk] = Acc(0);
    return;
  }
  Acc v = Acc(0);
  int64_t i = (int64_t)chunk * kRedThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * kChunkStride < n; i += kUnroll * kChunkStride) {
    Real a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      a[u] = x[i + u * kChunkStride];
      b[u] = y[i + u * kChunkStride];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v += (Acc)a[u] * (Acc)b[u];
  }
  for (; i < n; i += kChunkStride) v += (Acc)x[i] * (Acc)y[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[chunk] = v;
}

template <typename Real, typename Acc>
__global__ void __launch_bounds__(kRedThreads) dot_partial_kernel(const Real *__restrict__ x, const Real *__restrict__ y,
                                                                  int64_t n, Acc *__restrict__ part)
{
  __shared__ Acc sh[kRedThreads];
  dot_partial_body(x, y, n, part, blockIdx.x, sh);
}

template <typename Acc>
__global__ void __launch_bounds__(kRedThreads) finalize_kernel(const Acc *__restrict__ part, int count, Acc *out)
{
  __shared__ Acc sh[kRedThreads];
  Acc v = Acc(0);
  for (int i = threadIdx.x; i < count; i += kRedThreads) v += part[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[0] = v;
}

// out[0] = the sum of part[0 .. count) in a fixed order: thread t sums the
// entries t, t + T, t + 2T, ... (eight loads issued before their adds), then
// the fixed-order workgroup sum over the T = 1024 threads of the one workgroup
constexpr int kSumThreads = 1024;
template <typename Acc>
__device__ __forceinline__ void sum_shares_body(const Acc *__restrict__ part, int count, Acc *out, Acc *sh)
{
  const int t = threadIdx.x;
  Acc v = Acc(0);
  int i = t;
  for (; i + 7 * kSumThreads < count; i += 8 * kSumThreads) {
    Acc a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = part[i + u * kSumThreads];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += a[u];
  }
  for (; i < count; i += kSumThreads) v += part[i];
  v = workgroup_sum<kSumThreads>(v, sh);
  if (t == 0) out[0] = v;
}

template <typename Acc>
__global__ void __launch_bounds__(kSumThreads) sum_shares_kernel(const Acc *__restrict__ part, int count, Acc *out)
{
  __shared__ Acc sh[kSumThreads];
  sum_shares_body(part, count, out, sh);
}

template <typename Real>
__global__ void copy_kernel(const Real *__restrict__ a, Real *__restrict__ b, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <typename Real>
__global__ void fill_kernel(Real *__restrict__ a, Real v, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// c = a - b (c may alias b)
template <typename Real>
__global__ void sub_kernel(const Real *a, const Real *b, Real *c, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] - b[i];
}

// partials of r.z and r.r with z = r / d, interleaved per block
template <typename Real, typename Acc>
__global__ void __launch_bounds__(kRedThreads) rz_partial_kernel(const Real *__restrict__ r, const Real *__restrict__ d,
                                                                 int64_t n, Acc *__restrict__ part2)
{
  __shared__ Acc sh[kRedThreads];
  Acc rz = Acc(0), rr = Acc(0);
  int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * kChunkStride < n; i += kUnroll * kChunkStride) {
    Real rv[kUnroll], dv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      rv[u] = r[i + u * kChunkStride];
      dv[u] = d[i + u * kChunkStride];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const Acc ri = (Acc)rv[u];
      rz += ri * (ri / (Acc)dv[u]);
      rr += ri * ri;
    }
  }
  for (; i < n; i += kChunkStride) {
    const Acc ri = (Acc)r[i];
    rz += ri * (ri / (Acc)d[i]);
    rr += ri * ri;
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = rz;
    part2[2 * blockIdx.x + 1] = rr;
  }
}

// alpha = rz / (p.q);  r -= alpha q;  partials of r.z, r.r (the solution
// update x += alpha p is left to the direction update, which reads p anyway)
template <typename Real, typename Acc>
__device__ __forceinline__ void cg_update_body(Real *__restrict__ r, const Real *__restrict__ q,
                                               const Real *__restrict__ d, int64_t n,
                                               const Acc *__restrict__ pq_part, const Acc *scal, int cur,
                                               Acc *__restrict__ part2, int chunk, Acc *sh)
{
  if ((int64_t)chunk * kRedThreads >= n) {  // an empty chunk needs no alpha
    if (threadIdx.x == 0) part2[2 * chunk] = part2[2 * chunk + 1] = Acc(0);
    return;
  }
  const Acc pq = reduce_partials(pq_part, 1, sh);
  const Acc alpha = scal[cur] / pq;
  Acc rz = Acc(0), rr = Acc(0);
  auto one = [&](int64_t j, Real rv, Real qv, Real dv) {
    const Acc ri = (Acc)rv - alpha * (Acc)qv;
    r[j] = (Real)ri;
    rz += ri * (ri / (Acc)dv);
    rr += ri * ri;
  };
  int64_t i = (int64_t)chunk * kRedThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * kChunkStride < n; i += kUnroll * kChunkStride) {
    Real rv[kUnroll], qv[kUnroll], dv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t j = i + u * kChunkStride;
      rv[u] = r[j];
      qv[u] = q[j];
      dv[u] = d[j];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) one(i + u * kChunkStride, rv[u], qv[u], dv[u]);
  }
  for (; i < n; i += kChunkStride) one(i, r[i], q[i], d[i]);
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    part2[2 * chunk] = rz;
    part2[2 * chunk + 1] = rr;
  }
}

template <typename Real, typename Acc>
__global__ void __launch_bounds__(kRedThreads) cg_update_kernel(Real *__restrict__ r, const Real *__restrict__ q,
                                                                const Real *__restrict__ d, int64_t n,
                                                                const Acc *__restrict__ pq_part, const Acc *scal,
                                                                int cur, Acc *__restrict__ part2)
{
  __shared__ Acc sh[kRedThreads];
  cg_update_body(r, q, d, n, pq_part, scal, cur, part2, blockIdx.x, sh);
}

// x += alpha p with the same alpha = scal[cur] / (p.q) as cg_update (when x
// is not null), then rz_new = r.z;  p = z + (rz_new / scal[cur]) p  (p = z
// when use_beta == 0); chunk 0 stores rz_new in scal[1 - cur] and r.r in
// scal[2] (the other chunks still read scal[cur], hence the ping-pong)
template <typename Real, typename Acc>
__device__ __forceinline__ void cg_pupdate_body(Real *__restrict__ p, Real *__restrict__ x,
                                                const Real *__restrict__ r, const Real *__restrict__ d, int64_t n,
                                                const Acc *__restrict__ pq_part, const Acc *__restrict__ part2,
                                                Acc *scal, int use_beta, int cur, int chunk, Acc *sh)
{
  if (chunk > 0 && (int64_t)chunk * kRedThreads >= n) return;  // empty; chunk 0 always stores the scalars
  const Acc rz = reduce_partials(part2, 2, sh);
  const Acc rr = reduce_partials(part2 + 1, 2, sh);
  const Acc beta = use_beta ? rz / scal[cur] : Acc(0);
  Acc alpha = Acc(0);
  if (x) alpha = scal[cur] / reduce_partials(pq_part, 1, sh);
  int64_t i = (int64_t)chunk * kRedThreads + threadIdx.x;
  if (x) {
    for (; i + (kUnroll - 1) * kChunkStride < n; i += kUnroll * kChunkStride) {
      Real rv[kUnroll], dv[kUnroll], pv[kUnroll], xv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t j = i + u * kChunkStride;
        rv[u] = r[j];
        dv[u] = d[j];
        pv[u] = p[j];
        xv[u] = x[j];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t j = i + u * kChunkStride;
        x[j] = (Real)((Acc)xv[u] + alpha * (Acc)pv[u]);
        const Acc z = (Acc)rv[u] / (Acc)dv[u];
        p[j] = use_beta ? (Real)(z + beta * (Acc)pv[u]) : (Real)z;
      }
    }
    for (; i < n; i += kChunkStride) {
      const Acc pv = (Acc)p[i];
      x[i] = (Real)((Acc)x[i] + alpha * pv);
      const Acc z = (Acc)r[i] / (Acc)d[i];
      p[i] = use_beta ? (Real)(z + beta * pv) : (Real)z;
    }
  } else {
    for (; i + (kUnroll - 1) * kChunkStride < n; i += kUnroll * kChunkStride) {
      Real rv[kUnroll], dv[kUnroll], pv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t j = i + u * kChunkStride;
        rv[u] = r[j];
        dv[u] = d[j];
        pv[u] = p[j];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const Acc z = (Acc)rv[u] / (Acc)dv[u];
        p[i + u * kChunkStride] = use_beta ? (Real)(z + beta * (Acc)pv[u]) : (Real)z;
      }
    }
    for (; i < n; i += kChunkStride) {
      const Acc z = (Acc)r[i] / (Acc)d[i];
      p[i] = use_beta ? (Real)(z + beta * (Acc)p[i]) : (Real)z;
    }
  }
  if (chunk == 0 && threadIdx.x == 0) {
    scal[1 - cur] = rz;
    scal[2] = rr;
  }
}

template <typename Real, typename Acc>
__global__ void __launch_bounds__(kRedThreads) cg_pupdate_kernel(Real *__restrict__ p, Real *__restrict__ x,
                                                                 const Real *__restrict__ r,
                                                                 const Real *__restrict__ d, int64_t n,
                                                                 const Acc *__restrict__ pq_part,
                                                                 const Acc *__restrict__ part2, Acc *scal, int use_beta,
                                                                 int cur)
{
  __shared__ Acc sh[kRedThreads];
  cg_pupdate_body(p, x, r, d, n, pq_part, part2, scal, use_beta, cur, blockIdx.x, sh);
}

// scal[cur] = r.z, scal[2] = r.r from interleaved partials
template <typename Acc>
__global__ void __launch_bounds__(kRedThreads) rz_finalize_kernel(const Acc *__restrict__ part2, Acc *scal, int cur)
{
  __shared__ Acc sh[kRedThreads];
  const Acc rz = reduce_partials(part2, 2, sh);
  const Acc rr = reduce_partials(part2 + 1, 2, sh);
  if (threadIdx.x == 0) {
    scal[cur] = rz;
    scal[2] = rr;
  }
}

static __global__ void scale_to_f32_kernel(const double *__restrict__ a, double s, float *__restrict__ b, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)(a[i] * s);
}

static __global__ void axpy_f32_kernel(double *__restrict__ x, double a, const float *__restrict__ d, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += a * (double)d[i];
}

}  // namespace dgk
