// Device helpers shared by the patch, transfer and coarse kernels: reference
// tables in constant memory (for runtime-indexed access), patch geometry,
// Gauss-point entries of A_gamma, and the in-LDS SPD inversion.
#pragma once

#include "stk_internal.h"

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

// ---------------------------------------------------------------------------
// Dense SPD inversion with FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l
// holds A[l%16][l/16] and B[l/16][l%16] of the 16 x 4 and 4 x 16 operands;
// result register r of lane l is D[l/16 + 4r][l%16]).
typedef double d4 __attribute__((ext_vector_type(4)));

// Orders the LDS accesses of one wavefront's lanes around this point (an
// exchange among the lanes of a single wavefront needs no workgroup barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront: the 16 x 16 SPD block p (row stride 17, full on entry) is
// replaced by X = L^{-1}, L L^T = p (lower triangle; zeros above). Sets *bad
// on a non-positive pivot (taken as 1 so the arithmetic stays finite).
__device__ inline void chol_inv16_wave(double* p, int lane, int* bad) {
  constexpr int ld = 17;
  for (int k = 0; k < 16; ++k) {
    double d = p[k * ld + k];
    if (!(d > 0.0)) {
      if (lane == 0) *bad = 1;
      d = 1.0;
    }
    const double lkk = sqrt(d);
    wave_lds_sync();   // every lane has read the pivot before it is replaced
    if (lane == k) p[k * ld + k] = lkk;
    if (lane > k && lane < 16) p[lane * ld + k] /= lkk;
    wave_lds_sync();
    const int m = 15 - k;
    for (int t = lane; t < m * m; t += 64) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) p[i * ld + j] -= p[i * ld + k] * p[j * ld + k];
    }
    wave_lds_sync();
  }
  for (int j = 15; j >= 0; --j) {
    // column j of L^{-1} below the diagonal: -X[j+1:, j+1:] L[j+1:, j] / L_jj
    const double ljj = p[j * ld + j];
    double s = 0.0;
    if (lane > j && lane < 16)
      for (int k = j + 1; k <= lane; ++k) s += p[lane * ld + k] * p[k * ld + j];
    wave_lds_sync();
    if (lane > j && lane < 16) p[lane * ld + j] = -s / ljj;
    if (lane == j) p[j * ld + j] = 1.0 / ljj;
    wave_lds_sync();
  }
  for (int t = lane; t < 256; t += 64)
    if (t % 16 > t / 16) p[(t / 16) * ld + t % 16] = 0.0;
  wave_lds_sync();
}

// acc += X Y for 16 x 16 tiles in LDS (row stride 17); X read transposed when
// tx, Y likewise when ty.
__device__ inline d4 tile17_mma(const double* X, bool tx, const double* Y, bool ty, d4 acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const int kk = k0 + lk;
    const double x = tx ? X[kk * 17 + li] : X[li * 17 + kk];
    const double y = ty ? Y[li * 17 + kk] : Y[kk * 17 + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
  }
  return acc;
}

// Stores the 16 x 16 result acc (times sign) into a stride-17 tile.
__device__ inline void tile17_store(double* T, d4 acc, double sign) {
  const int lane = threadIdx.x & 63, li = lane & 15, lr = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(lr + 4 * r) * 17 + li] = sign * acc[r];
}

// Lower 16 x 16 tiles of a symmetric matrix: tile (I, J), I >= J, at
// L + (I(I+1)/2 + J) * 272 with row stride 17; diagonal tiles kept in full.
constexpr int kTile17 = 16 * 17;
__device__ inline int ltile(int I, int J) { return I * (I + 1) / 2 + J; }

// In-LDS inverse of the SPD matrix held in the lower tiles L (nb block rows;
// rows and columns past the operator's size hold the identity), through its
// Cholesky factor, in three blocked phases whose tile products run on the
// FP64 matrix cores:
//   1. right-looking block Cholesky: X_kk = L_kk^{-1} by wavefront 0 (kept in
//      the diagonal tile), panel L_Ik = A_Ik X_kk^T, update A_IJ -= L_Ik L_Jk^T;
//   2. X = L^{-1} in place, columns left to right, rows downward:
//      X_IJ = -X_II sum_{m=J}^{I-1} L_Im X_mJ (wavefront 0);
//   3. A^{-1} = X^T X by block rows: (A^{-1})_IJ = sum_{m>=I} X_mI^T X_mJ.
// On exit the lower tiles hold A^{-1} (diagonal tiles in full). W is LDS
// scratch of nb tiles. Sets *bad on a non-positive pivot. All threads of the
// workgroup must call this.
__device__ inline void spd_invert_lower16(double* L, int nb, double* W, int* bad) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  for (int k = 0; k < nb; ++k) {
    double* tkk = L + ltile(k, k) * kTile17;
    if (w == 0) chol_inv16_wave(tkk, lane, bad);
    __syncthreads();
    for (int I = k + 1 + w; I < nb; I += nw) {
      double* T = L + ltile(I, k) * kTile17;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = tile17_mma(T, false, tkk, true, acc);
      tile17_store(T, acc, 1.0);
    }
    __syncthreads();
    const int m = nb - k - 1;
    for (int t = w; t < m * (m + 1) / 2; t += nw) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= t) ++i;
      const int I = k + 1 + i, J = k + 1 + (t - i * (i + 1) / 2);
      double* T = L + ltile(I, J) * kTile17;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = tile17_mma(L + ltile(I, k) * kTile17, false, L + ltile(J, k) * kTile17, true, acc);
      const int li = lane & 15, lr = lane >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(lr + 4 * r) * 17 + li] -= acc[r];
    }
    __syncthreads();
  }
  if (w == 0) {
    for (int J = 0; J < nb; ++J)
      for (int I = J + 1; I < nb; ++I) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int mm = J; mm < I; ++mm)
          acc = tile17_mma(L + ltile(I, mm) * kTile17, false, L + ltile(mm, J) * kTile17, false, acc);
        tile17_store(W, acc, 1.0);
        wave_lds_sync();
        d4 acc2 = {0.0, 0.0, 0.0, 0.0};
        acc2 = tile17_mma(L + ltile(I, I) * kTile17, false, W, false, acc2);
        wave_lds_sync();   // W and L_IJ are read before L_IJ is replaced
        tile17_store(L + ltile(I, J) * kTile17, acc2, -1.0);
        wave_lds_sync();
      }
  }
  __syncthreads();
  for (int I = 0; I < nb; ++I) {
    for (int J = w; J <= I; J += nw) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int mm = I; mm < nb; ++mm)
        acc = tile17_mma(L + ltile(mm, I) * kTile17, true, L + ltile(mm, J) * kTile17, false, acc);
      tile17_store(W + J * kTile17, acc, 1.0);
    }
    __syncthreads();
    for (int e = tid; e < (I + 1) * 256; e += blockDim.x) {
      const int J = e / 256, r = (e % 256) / 16, c = e % 16;
      L[ltile(I, J) * kTile17 + r * 17 + c] = W[J * kTile17 + r * 17 + c];
    }
    __syncthreads();
  }
}

}  // namespace stk
