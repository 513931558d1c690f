// Deterministic reduction helpers shared by the Krylov and pressure kernels.
#pragma once

#include "stk_internal.h"

namespace stk {

// Number of partial sums (one per block) used for a vector of length n.
inline int red_parts(int64_t n) {
  const int64_t p = (n + (int64_t)kRedThreads * 8 - 1) / ((int64_t)kRedThreads * 8);
  return (int)(p < 1 ? 1 : (p > kRedBlocks ? kRedBlocks : p));
}
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sum of part[b*stride + k] over b < nparts by one full wavefront; every lane
// gets the result.
__device__ inline double wave_reduce_parts(const double* __restrict__ part, int nparts, int stride, int k) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nparts; b += 64) s += part[b * stride + k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

}  // namespace stk
