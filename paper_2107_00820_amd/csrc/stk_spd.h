// Dense SPD inversion in LDS on the FP64 matrix cores, for the setup of the
// star-patch inverses and the pivot blocks of the coarse inverse.
#pragma once

#include "stk_dev.h"

namespace stk {

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
// workgroup must call this. Phases 1-2 are spd_cholinv_lower16 (on exit the
// lower tiles hold X = L^{-1}), phase 3 is spd_xtx_lower16.
__device__ inline void spd_cholinv_lower16(double* L, int nb, double* W, int* bad) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
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
}

// Lower tiles of X^T X for X = L^{-1} held in the lower tiles (in place).
__device__ inline void spd_xtx_lower16(double* L, int nb, double* W) {
  const int tid = threadIdx.x, w = tid >> 6, nw = blockDim.x >> 6;
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

__device__ inline void spd_invert_lower16(double* L, int nb, double* W, int* bad) {
  spd_cholinv_lower16(L, nb, W, bad);
  spd_xtx_lower16(L, nb, W);
}

}  // namespace stk
