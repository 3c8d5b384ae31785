// reduce.hpp -- deterministic workgroup sums: a butterfly within each 64-lane
// wave (cross-lane exchanges, no LDS), then the wave partials added in wave
// order.  Every lane of a wave ends the butterfly with the same bits (each
// step adds the same two values, and addition commutes exactly), so the
// result depends on nothing but the values and the fixed order.
#pragma once

#include <hip/hip_runtime.h>

namespace dgk {

constexpr int kWave = 64;

template <typename Real>
__device__ __forceinline__ Real wave_sum(Real v)
{
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// sum over the T threads of a workgroup (T a multiple of 64); sh holds at
// least T / 64 values; every thread gets the result
template <int T, typename Real>
__device__ __forceinline__ Real workgroup_sum(Real v, Real *sh)
{
  static_assert(T % kWave == 0, "whole waves");
  constexpr int NW = T / kWave;
  v = wave_sum(v);
  if constexpr (NW == 1) return v;
  const int t = threadIdx.x;
  if ((t & (kWave - 1)) == 0) sh[t / kWave] = v;
  __syncthreads();
  Real s = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s += sh[w];
  __syncthreads();   // sh is free for the next sum
  return s;
}

}  // namespace dgk
