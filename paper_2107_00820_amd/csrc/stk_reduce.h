// Deterministic reduction helpers shared by the Krylov and pressure kernels.
#pragma once

#include "stk_internal.h"

namespace stk {

// Number of partial sums (one per block) used for a vector of length n: one
// element per thread up to kRedBlocks blocks (short vectors then finish in
// one memory round trip), grid-stride beyond.
// Threads per workgroup of the reductions over a vector of length n: 256,
// or kRedThreads (1024) for long vectors, where fewer grid-stride rounds per
// thread pay for the wider block sums.
inline int red_threads(int64_t n) { return n >= kRedLongVector ? kRedThreads : 256; }
inline int red_parts(int64_t n) {
  const int64_t t = red_threads(n);
  const int64_t p = (n + t - 1) / t;
  return (int)(p < 1 ? 1 : (p > kRedBlocks ? kRedBlocks : p));
}

// Sum over the block (kRedThreads threads): butterfly within each wavefront,
// then the wavefront sums in a fixed order. `sh` holds kRedThreads/64 doubles.
// Every thread gets the result.
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r += sh[w];
  return r;
}

// Block sums of v[0..m) (m <= 8) at once: out[k] valid in every thread.
// `sh` holds 8 * kRedThreads/64 doubles.
template <int M>
__device__ inline void block_sum_n(const double (&v)[M], int m, double* sh, double (&out)[M]) {
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double t[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    t[k] = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t[k] += __shfl_xor(t[k], off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (k < m) sh[wave * M + k] = t[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double r = 0.0;
    if (k < m)
      for (int w = 0; w < nw; ++w) r += sh[w * M + k];
    out[k] = r;
  }
}

// Sum of part[b*stride + k] over b < nparts by one full wavefront; every lane
// gets the result.
__device__ inline double wave_reduce_parts(const double* __restrict__ part, int nparts, int stride, int k) {
  const int lane = threadIdx.x & 63;
  // the (at most kRedBlocks / 64) loads of a lane are issued together, then
  // added in index order (the same order as a plain strided loop)
  constexpr int kPer = kRedBlocks / 64;
  double v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int b = lane + 64 * i;
    v[i] = b < nparts ? part[b * stride + k] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) s += v[i];
  for (int b = lane + 64 * kPer; b < nparts; b += 64) s += part[b * stride + k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

}  // namespace stk
