// Vector kernels of the Krylov methods (relaxation GMRES and outer FGMRES).
//
// Reductions are deterministic: a vector of length n is covered by a fixed
// grid of red_parts(n) blocks (grid-stride loops, so block b always owns the
// same indices), each block writes one partial per reduced quantity, and
// every consumer reduces the partials in a fixed order (64 lanes with strided
// sums, then a fixed butterfly). Arnoldi uses classical Gram-Schmidt applied
// twice; the second pass's dot products are formed by the blocks that finish
// the first pass's update of their own indices, so one CGS2 step takes three
// kernels plus the normalisation.
#include "stk_reduce.h"

namespace stk {

// h[k] = sum_b part[b*nk + k] for k < nk, into LDS, by the block's wavefronts.
__device__ inline void reduce_parts_to_lds(const double* __restrict__ part, int nparts, int nk, double* h) {
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = wave; k < nk; k += nw) {
    const double s = wave_reduce_parts(part, nparts, nk, k);
    if ((threadIdx.x & 63) == 0) h[k] = s;
  }
  __syncthreads();
}

// part[b*nk + k] = sum over block b's indices of V_k . w (storage type R,
// accumulation in double)
template <class R>
__global__ void __launch_bounds__(kRedThreads) k_dots(const R* __restrict__ V, int64_t ldv, int nk,
                                                       const R* __restrict__ w, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  for (int k0 = 0; k0 < nk; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const double wi = (double)w[i];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < nk) acc[kk] += (double)V[(int64_t)(k0 + kk) * ldv + i] * wi;
    }
    double tot[8];
    block_sum_n<8>(acc, nk - k0, sh, tot);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < nk) part[blockIdx.x * nk + k0 + kk] = tot[kk];
    }
  }
}

// h = reduce(part_in); Hcol[k*hstride] (+)= h_k (block 0); w -= sum_k h_k V_k on
// this block's indices; then either the next pass's dot partials
// (next_dots = 1: part_out[b*nk+k] = V_k . w) or the squared-norm partial
// (next_dots = 0: part_out[b] = w . w).
template <class R>
__global__ void __launch_bounds__(kRedThreads) k_orth_update(const R* __restrict__ V, int64_t ldv, int nk,
                                                              R* __restrict__ w, int64_t n,
                                                              const double* __restrict__ part_in,
                                                              double* __restrict__ Hcol, int hstride, int accumulate,
                                                              double* __restrict__ part_out, int next_dots) {
  __shared__ double h[64];
  __shared__ double sh[kRedThreads];
  // this thread's first entry of w and of the first KP basis vectors are
  // loaded before the partials are reduced (they do not depend on them), so
  // the two memory round trips overlap; the arithmetic below is unchanged
  constexpr int KP = 4;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const bool has0 = i0 < n;
  const double w0 = has0 ? (double)w[i0] : 0.0;
  double v0[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) v0[k] = (has0 && k < nk) ? (double)V[(int64_t)k * ldv + i0] : 0.0;
  reduce_parts_to_lds(part_in, gridDim.x, nk, h);
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < nk; k += blockDim.x)
      Hcol[k * hstride] = (accumulate ? Hcol[k * hstride] : 0.0) + h[k];
  double nrm = 0.0;
  if (has0) {
    double v = w0;
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (k < nk) v -= h[k] * v0[k];
    for (int k = KP; k < nk; ++k) v -= h[k] * (double)V[(int64_t)k * ldv + i0];
    const R vr = (R)v;
    w[i0] = vr;
    nrm += (double)vr * (double)vr;
  }
  for (int64_t i = i0 + step; i < n; i += step) {
    double v = (double)w[i];
    for (int k = 0; k < nk; ++k) v -= h[k] * (double)V[(int64_t)k * ldv + i];
    const R vr = (R)v;
    w[i] = vr;
    nrm += (double)vr * (double)vr;
  }
  if (next_dots) {
    // second-pass dots over the same indices (each written by this thread above)
    for (int k0 = 0; k0 < nk; k0 += 8) {
      double acc[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
      for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
           i += (int64_t)gridDim.x * blockDim.x) {
        const double wi = (double)w[i];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (k0 + kk < nk) acc[kk] += (double)V[(int64_t)(k0 + kk) * ldv + i] * wi;
      }
      double tot[8];
      block_sum_n<8>(acc, nk - k0, sh, tot);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (k0 + kk < nk) part_out[blockIdx.x * nk + k0 + kk] = tot[kk];
      }
    }
  } else {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
  }
}

// nrm = sqrt(sum part); *hout = nrm (block 0); dst = w / nrm (0 if nrm == 0).
template <class R>
__global__ void __launch_bounds__(kRedThreads) k_normalize(const double* __restrict__ part, int nparts,
                                                            const R* w, int64_t n, R* dst,
                                                            double* __restrict__ hout) {
  __shared__ double nrm;
  // first entry loaded before the norm is reduced (dst may alias w: each
  // entry is read and written by the same thread only)
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const double w0 = i0 < n ? (double)w[i0] : 0.0;
  if (threadIdx.x < 64) {
    const double s = wave_reduce_parts(part, nparts, 1, 0);
    if (threadIdx.x == 0) {
      nrm = sqrt(s);
      if (blockIdx.x == 0 && hout) *hout = nrm;
    }
  }
  __syncthreads();
  const double d = nrm;
  if (i0 < n) dst[i0] = (R)(d > 0.0 ? w0 / d : 0.0);
  for (int64_t i = i0 + step; i < n; i += step)
    dst[i] = (R)(d > 0.0 ? (double)w[i] / d : 0.0);
}

// Least squares min ||beta e1 - Hbar y|| by Givens rotations over NU columns
// (compile-time, so every array stays in registers); columns after an exact
// breakdown (H[j+1][j] == 0) are dropped; entries below the subdiagonal are
// zero by construction and not read.
template <int NU>
__device__ inline void ls_solve(const double* __restrict__ small, double hlast, double* y) {
  const double* Hm = small + kSmallH;
  const double beta = small[kSmallBeta];
  // H[NU][NU-1] from the caller when given (hlast >= 0), else as stored
  auto Hat = [&](int i, int j) { return (i == NU && j == NU - 1 && hlast >= 0.0) ? hlast : Hm[i * kMaxNu + j]; };
  double yr[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) yr[j] = 0.0;
  if (beta > 0.0) {
    int k = NU;
#pragma unroll
    for (int j = NU - 1; j >= 0; --j)
      if (Hat(j + 1, j) == 0.0) k = j + 1;
    double R[NU + 1][NU], g[NU + 1];
#pragma unroll
    for (int i = 0; i <= NU; ++i) {
      g[i] = 0.0;
#pragma unroll
      for (int j = 0; j < NU; ++j) R[i][j] = i <= j + 1 ? Hat(i, j) : 0.0;
    }
    g[0] = beta;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      if (j < k) {
        const double a = R[j][j], b = R[j + 1][j];
        double c = 1.0, s = 0.0;
        if (b != 0.0) {
          const double r = hypot(a, b);
          c = a / r;
          s = b / r;
        }
#pragma unroll
        for (int t = j; t < NU; ++t) {
          if (t < k) {
            const double u = R[j][t], v = R[j + 1][t];
            R[j][t] = c * u + s * v;
            R[j + 1][t] = -s * u + c * v;
          }
        }
        const double gu = g[j], gv = g[j + 1];
        g[j] = c * gu + s * gv;
        g[j + 1] = -s * gu + c * gv;
      }
    }
#pragma unroll
    for (int j = NU - 1; j >= 0; --j) {
      if (j < k) {
        double s = g[j];
#pragma unroll
        for (int t = j + 1; t < NU; ++t)
          if (t < k) s -= R[j][t] * yr[t];
        yr[j] = s / R[j][j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NU; ++j) y[j] = yr[j];
}

// x = (x_zero ? 0 : x) + sum_k y_k Z_k with y solved from the relaxation's
// Hessenberg system (every block solves the tiny system redundantly). The
// last subdiagonal entry ||w|| is reduced here from the norm partials of the
// final Gram-Schmidt pass, so the last Arnoldi vector is never normalised.
template <class R, int NU>
__global__ void k_relax_update(const R* __restrict__ Z, int64_t ldz, const double* __restrict__ small,
                               const double* __restrict__ norm_part, int nparts, R* __restrict__ x, int64_t n,
                               int x_zero) {
  __shared__ double y[NU];
  __shared__ double hl;
  // this thread's x and Z entries are loaded before the reduction and the
  // small least-squares solve, which they do not depend on
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = i < n;
  const double x0 = (in && !x_zero) ? (double)x[i] : 0.0;
  double zk[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) zk[k] = in ? (double)Z[(int64_t)k * ldz + i] : 0.0;
  if (threadIdx.x < 64) {
    const double s = wave_reduce_parts(norm_part, nparts, 1, 0);
    if (threadIdx.x == 0) hl = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) ls_solve<NU>(small, hl, y);
  __syncthreads();
  if (!in) return;
  double v = x0;
#pragma unroll
  for (int k = 0; k < NU; ++k) v += y[k] * zk[k];
  x[i] = (R)v;
}

__global__ void k_combine(const double* __restrict__ Z, int64_t ldz, int nk, const double* __restrict__ y,
                          double* __restrict__ x, int64_t n, int x_zero) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = x_zero ? 0.0 : x[i];
  for (int k = 0; k < nk; ++k) v += y[k] * Z[(int64_t)k * ldz + i];
  x[i] = v;
}

template <class R>
__global__ void k_axpby(double a, const R* x, double b, const R* y, R* out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (R)(a * (double)x[i] + b * (double)y[i]);
}

template <class A, class B>
__global__ void k_convert(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (B)x[i];
}

template <class R>
__global__ void k_fill(R* __restrict__ x, double v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = (R)v;
}

__global__ void k_fill_int(int* __restrict__ x, int v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class R>
void launch_dots(const R* V, int64_t ldv, int nk, const R* w, int64_t n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dots<R>, dim3(red_parts(n)), dim3(red_threads(n)), 0, s, V, ldv, nk, w, n, partials);
}

template <class R>
void launch_orth_update(const R* V, int64_t ldv, int nk, R* w, int64_t n, const double* part_in, double* Hcol,
                        int hstride, bool accumulate, double* part_out, bool next_dots, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_update<R>, dim3(red_parts(n)), dim3(red_threads(n)), 0, s, V, ldv, nk, w, n, part_in,
                     Hcol, hstride, accumulate ? 1 : 0, part_out, next_dots ? 1 : 0);
}

template <class R>
void launch_normalize(const double* norm_partials, R* w, int64_t n, R* dst, double* hout, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<R>, dim3(red_parts(n)), dim3(red_threads(n)), 0, s, norm_partials, red_parts(n), w, n,
                     dst, hout);
}

template <class R>
void launch_relax_update(const R* Z, int64_t ldz, int nu, const double* small, const double* norm_part, R* x,
                         int64_t n, bool x_zero, hipStream_t s) {
  const dim3 g(nblk(n, 256)), b(256);
  const int xz = x_zero ? 1 : 0;
  const int np = red_parts(n);
  switch (nu) {
    case 1: hipLaunchKernelGGL((k_relax_update<R, 1>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 2: hipLaunchKernelGGL((k_relax_update<R, 2>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 3: hipLaunchKernelGGL((k_relax_update<R, 3>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 4: hipLaunchKernelGGL((k_relax_update<R, 4>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 5: hipLaunchKernelGGL((k_relax_update<R, 5>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 6: hipLaunchKernelGGL((k_relax_update<R, 6>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    case 7: hipLaunchKernelGGL((k_relax_update<R, 7>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
    default: hipLaunchKernelGGL((k_relax_update<R, 8>), g, b, 0, s, Z, ldz, small, norm_part, np, x, n, xz); break;
  }
}

void launch_combine(const double* Z, int64_t ldz, int nk, const double* y, double* x, int64_t n, bool x_zero,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(nblk(n, 256)), dim3(256), 0, s, Z, ldz, nk, y, x, n, x_zero ? 1 : 0);
}

template <class R>
void launch_axpby(double a, const R* x, double b, const R* y, R* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<R>, dim3(nblk(n, 256)), dim3(256), 0, s, a, x, b, y, out, n);
}

template <class R>
void launch_fill(R* x, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<R>, dim3(nblk(n, 256)), dim3(256), 0, s, x, v, n);
}

template <class A, class B>
void launch_convert(const A* x, B* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<A, B>), dim3(nblk(n, 256)), dim3(256), 0, s, x, y, n);
}

void launch_fill_int(int* x, int v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_copy(const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, s, x, y, n);
}

#define STK_INST(R)                                                                                         \
  template void launch_dots<R>(const R*, int64_t, int, const R*, int64_t, double*, hipStream_t);           \
  template void launch_orth_update<R>(const R*, int64_t, int, R*, int64_t, const double*, double*, int, bool, \
                                      double*, bool, hipStream_t);                                          \
  template void launch_normalize<R>(const double*, R*, int64_t, R*, double*, hipStream_t);                 \
  template void launch_relax_update<R>(const R*, int64_t, int, const double*, const double*, R*, int64_t, bool,  \
                                       hipStream_t);                                                           \
  template void launch_axpby<R>(double, const R*, double, const R*, R*, int64_t, hipStream_t);             \
  template void launch_fill<R>(R*, double, int64_t, hipStream_t);
STK_INST(double)
STK_INST(float)
#undef STK_INST
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace stk
