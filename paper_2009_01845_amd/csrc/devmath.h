// Small device helpers for the kernels outside kernels.hip (density matrices,
// time evolution, reduced density matrices): complex types per precision and
// a fixed-order workgroup sum.  Everything here is internal to each
// translation unit that includes it.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qs_types.h"

namespace qs {
namespace dm {

template <typename R> struct CT;
template <> struct CT<float> {
  using C = float2;
};
template <> struct CT<double> {
  using C = double2;
};

// a complex value widened to float64 and narrowed back
struct Z {
  double x, y;
};
template <typename C> __device__ __forceinline__ Z wide(C a) { return Z{(double)a.x, (double)a.y}; }
template <typename C> __device__ __forceinline__ C narrow(Z a) {
  C r;
  r.x = (decltype(r.x))a.x;
  r.y = (decltype(r.y))a.y;
  return r;
}
__device__ __forceinline__ Z zmul(Z a, Z b) { return Z{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ Z zconj(Z a) { return Z{a.x, -a.y}; }

// Sum of v over a 256-thread workgroup in a fixed order (valid in thread 0).
__device__ __forceinline__ double wg_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(kThreads >> 6); ++i) r += red[i];
  __syncthreads();
  return r;
}

}  // namespace dm
}  // namespace qs
