// Vector kernels of the Krylov methods (relaxation GMRES and outer FGMRES).
// Reductions are deterministic: a fixed grid of kRedBlocks blocks writes one
// partial per block, and every consumer sums the partials in block order.
// Arnoldi uses classical Gram-Schmidt applied twice (dots of all basis
// vectors against the same w, then one combined update).
#include "stk_internal.h"

namespace stk {

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

// partials[b*nk + k] = sum over block b's share of V_k . w
__global__ void __launch_bounds__(kRedThreads) k_dots(const double* __restrict__ V, int64_t ldv, int nk,
                                                       const double* __restrict__ w, int64_t n,
                                                       double* __restrict__ partials) {
  __shared__ double sh[kRedThreads];
  for (int k0 = 0; k0 < nk; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const double wi = w[i];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < nk) acc[kk] += V[(int64_t)(k0 + kk) * ldv + i] * wi;
    }
    for (int kk = 0; kk < 8 && k0 + kk < nk; ++kk) {
      const double s = block_sum(acc[kk], sh);
      if (threadIdx.x == 0) partials[blockIdx.x * nk + k0 + kk] = s;
    }
  }
}

// h_k = sum_b partials[b*nk+k];  w -= sum_k h_k V_k;  Hcol[k*hstride] += h_k
// (block 0); norm partial of the updated w per block.
__global__ void __launch_bounds__(kRedThreads) k_orth_update(const double* __restrict__ V, int64_t ldv, int nk,
                                                              double* __restrict__ w, int64_t n,
                                                              const double* __restrict__ partials,
                                                              double* __restrict__ Hcol, int hstride,
                                                              double* __restrict__ norm_partials) {
  __shared__ double h[64];
  __shared__ double sh[kRedThreads];
  for (int k = threadIdx.x; k < nk; k += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += partials[b * nk + k];
    h[k] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < nk; k += blockDim.x) Hcol[k * hstride] += h[k];
  double nrm = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = w[i];
    for (int k = 0; k < nk; ++k) v -= h[k] * V[(int64_t)k * ldv + i];
    w[i] = v;
    nrm += v * v;
  }
  const double s = block_sum(nrm, sh);
  if (threadIdx.x == 0) norm_partials[blockIdx.x] = s;
}

// nrm = sqrt(sum partials); *hout = nrm (block 0); dst = w / nrm (0 if nrm == 0).
__global__ void __launch_bounds__(kRedThreads) k_normalize(const double* __restrict__ part, int nparts,
                                                            const double* w, int64_t n, double* dst,
                                                            double* __restrict__ hout) {
  __shared__ double nrm;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[b];
    nrm = sqrt(s);
    if (blockIdx.x == 0 && hout) *hout = nrm;
  }
  __syncthreads();
  const double d = nrm;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = d > 0.0 ? w[i] / d : 0.0;
}

// Least squares min ||beta e1 - Hbar y|| by Givens rotations (one thread).
// Columns after an exact breakdown (H[j+1][j] == 0) are dropped.
__global__ void k_ls_solve(double* __restrict__ small, int nu) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double* Hm = small + kSmallH;
  double* y = small + kSmallY;
  const double beta = small[kSmallBeta];
  for (int j = 0; j < kMaxNu; ++j) y[j] = 0.0;
  if (!(beta > 0.0)) return;
  int k = nu;
  for (int j = 0; j < nu; ++j)
    if (Hm[(j + 1) * kMaxNu + j] == 0.0) { k = j + 1; break; }
  double R[kMaxNu + 1][kMaxNu];
  double g[kMaxNu + 1];
  for (int i = 0; i <= k; ++i) {
    g[i] = 0.0;
    for (int j = 0; j < k; ++j) R[i][j] = Hm[i * kMaxNu + j];
  }
  g[0] = beta;
  for (int j = 0; j < k; ++j) {
    const double a = R[j][j], b = R[j + 1][j];
    double c = 1.0, s = 0.0;
    if (b != 0.0) {
      const double r = hypot(a, b);
      c = a / r;
      s = b / r;
    }
    for (int t = j; t < k; ++t) {
      const double u = R[j][t], v = R[j + 1][t];
      R[j][t] = c * u + s * v;
      R[j + 1][t] = -s * u + c * v;
    }
    const double gu = g[j], gv = g[j + 1];
    g[j] = c * gu + s * gv;
    g[j + 1] = -s * gu + c * gv;
  }
  for (int j = k - 1; j >= 0; --j) {
    double s = g[j];
    for (int t = j + 1; t < k; ++t) s -= R[j][t] * y[t];
    y[j] = s / R[j][j];
  }
}

__global__ void k_combine(const double* __restrict__ Z, int64_t ldz, int nk, const double* __restrict__ y,
                          double* __restrict__ x, int64_t n, int x_zero) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = x_zero ? 0.0 : x[i];
  for (int k = 0; k < nk; ++k) v += y[k] * Z[(int64_t)k * ldz + i];
  x[i] = v;
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + b * y[i];
}

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
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

void launch_dots(const double* V, int64_t ldv, int nk, const double* w, int64_t n, double* partials,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks), dim3(kRedThreads), 0, s, V, ldv, nk, w, n, partials);
}

void launch_orth_update(const double* V, int64_t ldv, int nk, double* w, int64_t n, const double* partials,
                        double* Hcol, int hstride, double* norm_partials, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, V, ldv, nk, w, n, partials, Hcol,
                     hstride, norm_partials);
}

void launch_normalize(const double* norm_partials, double* w, int64_t n, double* dst, double* hout,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(kRedBlocks), dim3(kRedThreads), 0, s, norm_partials, kRedBlocks, w, n, dst,
                     hout);
}

void launch_ls_solve(double* small, int nu, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(64), 0, s, small, nu);
}

void launch_combine(const double* Z, int64_t ldz, int nk, const double* y, double* x, int64_t n, bool x_zero,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(nblk(n, 256)), dim3(256), 0, s, Z, ldz, nk, y, x, n, x_zero ? 1 : 0);
}

void launch_axpby(double a, const double* x, double b, const double* y, double* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 256)), dim3(256), 0, s, a, x, b, y, out, n);
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_fill_int(int* x, int v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n, 256)), dim3(256), 0, s, x, v, n);
}

void launch_copy(const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, s, x, y, n);
}

}  // namespace stk
