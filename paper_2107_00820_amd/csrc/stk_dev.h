// Device helpers shared by the patch, transfer and coarse kernels: reference
// tables in constant memory (for runtime-indexed access), patch geometry,
// Gauss-point entries of A_gamma, and the in-LDS SPD inversion.
#pragma once

#include "stk_internal.h"
#include "stk_asm_sum.h"

namespace stk {

static __constant__ RefTab<2> cT2 = RefTab<2>();
static __constant__ RefTab<3> cT3 = RefTab<3>();

template <int D>
__device__ inline const RefTab<D>& ctab();
template <>
__device__ inline const RefTab<2>& ctab<2>() { return cT2; }
template <>
__device__ inline const RefTab<3>& ctab<3>() { return cT3; }

// Node box of the patch of vertex v: per axis first node and extent (1 or 3).
template <int D>
__device__ inline void patch_box(const LevelGeo& g, int vert, int lo[3], int ext[3], int vc[3]) {
  const int nv = g.N + 1;
  vc[0] = vert % nv;
  vc[1] = (vert / nv) % nv;
  vc[2] = D == 3 ? vert / (nv * nv) : 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { lo[k] = 0; ext[k] = 1; continue; }
    if (vc[k] == 0) { lo[k] = 1; ext[k] = 1; }
    else if (vc[k] == g.N) { lo[k] = 2 * g.N - 1; ext[k] = 1; }
    else { lo[k] = 2 * vc[k] - 1; ext[k] = 3; }
  }
}

// Patch unknown i -> (component, node coordinates).
template <int D>
__device__ inline int patch_dof(int i, const int lo[3], const int ext[3], int nd[3]) {
  const int nbox = ext[0] * ext[1] * ext[2];
  const int comp = i / nbox;
  int b = i - comp * nbox;
  nd[0] = lo[0] + b % ext[0];
  b /= ext[0];
  nd[1] = lo[1] + b % ext[1];
  nd[2] = lo[2] + b / ext[1];
  return comp;
}

// Contribution of cell `cell` to the (comp ci, local node na; comp cj, local
// node nb) entry of A_gamma:  h^{d-2} [ sum_q w_q mu_q (delta_{ci,cj} grad phi_a .
// grad phi_b + d_{cj} phi_a d_{ci} phi_b) + gamma sum_m Bhat_m,a Bhat_m,b / Mhat_m ].
// With the tensor law (cw != NULL) each Gauss point also subtracts
// w_q (w_ci,: . grad phi_a)(w_cj,: . grad phi_b), the (w:eps_i)(w:eps_j) part of
// (C:eps_j):eps_i.
// With W = M_p(1/mu) (winv != NULL) the augmented term uses the cell's
// inverse weighted mass winv[cell] in place of Mhat^{-1}.
template <int D>
__device__ inline double cell_entry(const double* __restrict__ mu, const double* __restrict__ cw,
                                    const double* __restrict__ winv, int64_t ncell, int64_t cell, double h,
                                    double gamma, int ci, int na, int cj, int nb) {
  constexpr int NN = Dims<D>::NN, NP = Dims<D>::NP, NS = SymIdx<D>::NS;
  const RefTab<D>& T = ctab<D>();
  double s = 0.0;
  for (int q = 0; q < NN; ++q) {
    double gg = T.dphi[q][na][cj] * T.dphi[q][nb][ci];
    if (ci == cj) {
#pragma unroll
      for (int k = 0; k < D; ++k) gg += T.dphi[q][na][k] * T.dphi[q][nb][k];
    }
    s += T.w[q] * mu[cell * NN + q] * gg;
    if (cw) {
      double wi = 0.0, wj = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        wi += cw[(cell * NS + SymIdx<D>::at(ci, k)) * NN + q] * T.dphi[q][na][k];
        wj += cw[(cell * NS + SymIdx<D>::at(cj, k)) * NN + q] * T.dphi[q][nb][k];
      }
      s -= T.w[q] * wi * wj;
    }
  }
  double al = 0.0;
  if (winv) {
    const double* W = winv + cell * NP * NP;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) t += W[m * NP + k] * T.bhat[k][cj * NN + nb];
      al += T.bhat[m][ci * NN + na] * t;
    }
  } else {
#pragma unroll
    for (int m = 0; m < NP; ++m) al += T.bhat[m][ci * NN + na] * T.bhat[m][cj * NN + nb] * kInvMhat[m];
  }
  const double sc = D == 2 ? 1.0 : h;
  return sc * (s + gamma * al);
}

// Entry of A_gamma between (ci, node ni) and (cj, node nj): sum over the cells
// that contain both nodes.
template <int D>
__device__ inline double global_entry(const LevelGeo& g, const double* __restrict__ mu, const double* __restrict__ cw,
                                      const double* __restrict__ winv, double gamma, int ci, const int ni[3], int cj,
                                      const int nj[3]) {
  int clo[3], chi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { clo[k] = 0; chi[k] = 0; continue; }
    const int alo = (ni[k] - 1) >> 1 > 0 ? (ni[k] - 1) >> 1 : 0;   // cells containing node ni: floor((m-1)/2)..floor(m/2)
    const int ahi = (ni[k] >> 1) < g.N - 1 ? (ni[k] >> 1) : g.N - 1;
    const int blo = (nj[k] - 1) >> 1 > 0 ? (nj[k] - 1) >> 1 : 0;
    const int bhi = (nj[k] >> 1) < g.N - 1 ? (nj[k] >> 1) : g.N - 1;
    clo[k] = alo > blo ? alo : blo;
    chi[k] = ahi < bhi ? ahi : bhi;
    if (clo[k] > chi[k]) return 0.0;
  }
  double s = 0.0;
  for (int c2 = clo[2]; c2 <= chi[2]; ++c2)
    for (int c1 = clo[1]; c1 <= chi[1]; ++c1)
      for (int c0 = clo[0]; c0 <= chi[0]; ++c0) {
        const int64_t cell = cell_index<D>(g, c0, c1, c2);
        const int na = (ni[0] - 2 * c0) + 3 * (ni[1] - 2 * c1) + (D == 3 ? 9 * (ni[2] - 2 * c2) : 0);
        const int nb = (nj[0] - 2 * c0) + 3 * (nj[1] - 2 * c1) + (D == 3 ? 9 * (nj[2] - 2 * c2) : 0);
        s += cell_entry<D>(mu, cw, winv, g.ncell, cell, g.h, gamma, ci, na, cj, nb);
      }
  return s;
}

// In-LDS dense SPD inversion: a[n x ld] holds the full symmetric matrix on
// entry and the lower triangle of its inverse on exit. tmp has n entries.
// Sets *bad if a pivot is not positive.
__device__ inline void spd_invert_lds(double* a, int n, int ld, double* tmp, int* bad) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // Cholesky, right-looking: L overwrites the lower triangle
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      double d = a[k * ld + k];
      if (!(d > 0.0)) { *bad = 1; d = 1.0; }
      a[k * ld + k] = sqrt(d);
    }
    __syncthreads();
    const double lkk = a[k * ld + k];
    for (int i = k + 1 + tid; i < n; i += nt) a[i * ld + k] /= lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += nt) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) a[i * ld + j] -= a[i * ld + k] * a[j * ld + k];
    }
    __syncthreads();
  }
  // L^{-1} in place, columns right to left: column j of the inverse is
  // -Linv[j+1:, j+1:] L[j+1:, j] / L_jj, using the trailing inverse already formed
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = 1.0 / a[j * ld + j];
    for (int i = j + 1 + tid; i < n; i += nt) tmp[i] = a[i * ld + j];
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += nt) {
      double s = 0.0;
      for (int k = j + 1; k <= i; ++k) s += a[i * ld + k] * tmp[k];
      a[i * ld + j] = -s * ljj;
    }
    if (tid == 0) a[j * ld + j] = ljj;
    __syncthreads();
  }
  // A^{-1} = X^T X with X = L^{-1} (lower), row by row: (X^T X)_ij = sum_{k>=i} X_ki X_kj
  for (int i = 0; i < n; ++i) {
    for (int j = tid; j <= i; j += nt) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += a[k * ld + i] * a[k * ld + j];
      tmp[j] = s;
    }
    __syncthreads();
    for (int j = tid; j <= i; j += nt) a[i * ld + j] = tmp[j];
    __syncthreads();
  }
}

}  // namespace stk
