// Coarsest level: dense A_0,gamma over the interior unknowns, its explicit
// inverse by blocked in-place Gauss-Jordan elimination, and the solve as one
// dense GEMV. The paper solves the coarsest level with a sparse direct solver
// (Section 5.1); the coarse systems here (<= ~10^4 unknowns) fit HBM as dense
// matrices, and an explicit inverse turns every coarse solve into one fully
// parallel, coalesced pass instead of two sequential triangular sweeps.
//
// Block Gauss-Jordan step on pivot block k (P = A_kk, SPD for an SPD matrix):
//   A_kk <- P^{-1};  A_kj <- P^{-1} A_kj;  A_ik <- -A_ik P^{-1};
//   A_ij <- A_ij - A_ik P^{-1} A_kj          (i, j outside block k).
// After all blocks the array holds A^{-1}. With R' = [P^{-1} A_k,: whose pivot
// columns are replaced by P^{-1}] and C = A_:,k (old), every step is
//   rows i in k:      A_i,: = R'_{i-k0},:
//   other rows:       A_ij = (j in k ? 0 : A_ij) - C_i,: R'_:,j
#include "stk_dev.h"

namespace stk {

constexpr int kGJB = 32;   // pivot block width

// Interior unknown i (component-major over the (2N-1)^d interior nodes) ->
// (component, node coordinates).
template <int D>
__device__ inline int interior_dof(const LevelGeo& g, int64_t i, int nd[3]) {
  const int ni = 2 * g.N - 1;
  const int64_t nin = D == 2 ? (int64_t)ni * ni : (int64_t)ni * ni * ni;
  const int comp = (int)(i / nin);
  int64_t b = i - comp * nin;
  nd[0] = 1 + (int)(b % ni);
  b /= ni;
  nd[1] = 1 + (int)(b % ni);
  nd[2] = D == 3 ? 1 + (int)(b / ni) : 0;
  return comp;
}

template <int D>
__global__ void k_coarse_assemble(LevelGeo g, const double* __restrict__ mu, const double* __restrict__ cw,
                                  double gamma, int64_t n, double* __restrict__ A) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  int ni[3], nj[3];
  const int ci = interior_dof<D>(g, i, ni);
  const int cj = interior_dof<D>(g, j, nj);
  A[idx] = global_entry<D>(g, mu, cw, gamma, ci, ni, cj, nj);
}

// Pivot block inverse (single workgroup).
__global__ void k_gj_pivot(double* __restrict__ A, int64_t n, int64_t k0, int nb, double* __restrict__ Pinv,
                           int* __restrict__ flag) {
  __shared__ double a[kGJB * (kGJB + 1)];
  __shared__ double tmp[kGJB];
  __shared__ int bad;
  const int ld = nb + 1;
  if (threadIdx.x == 0) bad = 0;
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    const int i = t / nb, j = t % nb;
    a[i * ld + j] = A[(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  spd_invert_lds(a, nb, ld, tmp, &bad);
  __syncthreads();
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    const int i = t / nb, j = t % nb;
    Pinv[i * nb + j] = i >= j ? a[i * ld + j] : a[j * ld + i];
  }
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// R'[t][j] and C[i][t].
__global__ void k_gj_panels(const double* __restrict__ A, int64_t n, int64_t k0, int nb,
                            const double* __restrict__ Pinv, double* __restrict__ R, double* __restrict__ C) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nb) return;
  {
    const int t = (int)(idx / n);
    const int64_t j = idx - (int64_t)t * n;
    double v;
    if (j >= k0 && j < k0 + nb) {
      v = Pinv[t * nb + (j - k0)];
    } else {
      v = 0.0;
      for (int s = 0; s < nb; ++s) v += Pinv[t * nb + s] * A[(k0 + s) * n + j];
    }
    R[t * n + j] = v;
  }
  {
    const int64_t i = idx / nb;
    const int t = (int)(idx - i * nb);
    C[i * nb + t] = A[i * n + k0 + t];
  }
}

// Tiled update: 64x64 outputs per workgroup of 256 threads, 4x4 per thread.
__global__ void __launch_bounds__(256) k_gj_update(double* __restrict__ A, int64_t n, int64_t k0, int nb,
                                                    const double* __restrict__ R, const double* __restrict__ C) {
  __shared__ double Ct[64][kGJB + 1];
  __shared__ double Rt[kGJB][64 + 1];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  for (int t = threadIdx.x; t < 64 * nb; t += 256) {
    const int r = t / nb, c = t % nb;
    const int64_t gi = i0 + r;
    Ct[r][c] = gi < n ? C[gi * nb + c] : 0.0;
  }
  for (int t = threadIdx.x; t < nb * 64; t += 256) {
    const int r = t / 64, c = t % 64;
    const int64_t gj = j0 + c;
    Rt[r][c] = gj < n ? R[(int64_t)r * n + gj] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int t = 0; t < nb; ++t) {
    double cv[4], rv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) cv[a] = Ct[ty + 16 * a][t];
#pragma unroll
    for (int b = 0; b < 4; ++b) rv[b] = Rt[t][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += cv[a] * rv[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t i = i0 + ty + 16 * a;
    if (i >= n) continue;
    const bool prow = i >= k0 && i < k0 + nb;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t j = j0 + tx + 16 * b;
      if (j >= n) continue;
      if (prow) {
        A[i * n + j] = R[(i - k0) * n + j];
      } else {
        const bool pcol = j >= k0 && j < k0 + nb;
        const double old = pcol ? 0.0 : A[i * n + j];
        A[i * n + j] = old - acc[a][b];
      }
    }
  }
}

// x = Ainv b on interior unknowns: one wavefront per row.
template <int D, class R>
__global__ void __launch_bounds__(256) k_coarse_gemv(LevelGeo g, const double* __restrict__ Ainv, int64_t n,
                                                      const R* __restrict__ b, R* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) {
    int nd[3];
    const int c = interior_dof<D>(g, j, nd);
    s += Ainv[row * n + j] * (double)b[c * g.nnodes + node_index<D>(g, nd[0], nd[1], nd[2])];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    int nd[3];
    const int c = interior_dof<D>(g, row, nd);
    x[c * g.nnodes + node_index<D>(g, nd[0], nd[1], nd[2])] = (R)s;
  }
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_coarse_assemble(const Hier& H, const Level& l, double* A, hipStream_t s) {
  const int64_t n = H.n0;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_coarse_assemble<2>, dim3(nblk(n * n, 256)), dim3(256), 0, s, l.g, l.mu, l.cw, H.gamma, n, A);
  else
    hipLaunchKernelGGL(k_coarse_assemble<3>, dim3(nblk(n * n, 256)), dim3(256), 0, s, l.g, l.mu, l.cw, H.gamma, n, A);
}

// work needs kGJB*kGJB + 2*n*kGJB doubles.
int launch_coarse_invert(const Hier& H, double* A, int64_t n, double* work, hipStream_t s) {
  double* Pinv = work;
  double* R = work + kGJB * kGJB;
  double* C = R + (int64_t)kGJB * n;
  for (int64_t k0 = 0; k0 < n; k0 += kGJB) {
    const int nb = (int)((n - k0) < kGJB ? (n - k0) : kGJB);
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, A, n, k0, nb, Pinv, H.flag);
    hipLaunchKernelGGL(k_gj_panels, dim3(nblk(n * nb, 256)), dim3(256), 0, s, A, n, k0, nb, Pinv, R, C);
    const unsigned t = nblk(n, 64);
    hipLaunchKernelGGL(k_gj_update, dim3(t, t), dim3(256), 0, s, A, n, k0, nb, R, C);
  }
  return 0;
}

// The coarse solve is FP64 in both forms; R only selects the vector storage.
template <class R>
void launch_coarse_apply(const Hier& H, const Level& l, const R* b, R* x, hipStream_t s) {
  launch_fill<R>(x, 0.0, (int64_t)H.dim * l.g.nnodes, s);
  if (H.dim == 2)
    hipLaunchKernelGGL((k_coarse_gemv<2, R>), dim3(nblk(H.n0, 4)), dim3(256), 0, s, l.g, H.Ainv0, H.n0, b, x);
  else
    hipLaunchKernelGGL((k_coarse_gemv<3, R>), dim3(nblk(H.n0, 4)), dim3(256), 0, s, l.g, H.Ainv0, H.n0, b, x);
}

template void launch_coarse_apply<double>(const Hier&, const Level&, const double*, double*, hipStream_t);
template void launch_coarse_apply<float>(const Hier&, const Level&, const float*, float*, hipStream_t);

}  // namespace stk
