// [Q3]^3 x P2disc on axis-aligned cubes (Section 4, V_h^k and Q_h^{k-1} with
// k = 3, d = 3): tensor-product tables and device helpers of the 3D degree-3
// kernels. The 3D tables are products of 1D ones and are formed on the fly:
//   phi_n(x) = l_a(x0) l_b(x1) l_c(x2),   n = a + 4b + 16c,
//   psi_m = (x0 - 1/2)^e0 (x1 - 1/2)^e1 (x2 - 1/2)^e2, total degree <= 2, in
//   the order 1, x, y, z, x^2, xy, xz, y^2, yz, z^2,
//   Gauss points q = i + 4j + 16k of the 4-point rule per axis,
// so Bhat[m][c, n] = prod_k (k == c ? M1 : M0)[e_k][n_k] with the 1D moments
// M0[e][a] = sum_i w_i (x_i - 1/2)^e l_a(x_i), M1[e][a] = sum_i w_i (x_i - 1/2)^e l_a'(x_i),
// and Mhat[m][m'] = prod_k P[e_k + e'_k], P[e] = sum_i w_i (x_i - 1/2)^e.
//
// Cell operator (3D, so the viscous and augmented terms carry h^{d-2} = h):
//   A_K u = h sum_q w_q mu_q [(G + G^T) : dphi],  G_K u = gamma h Bhat^T W^{-1} Bhat u,
//   (B u)_K = -h^2 Bhat u,  (B^T p)_K = -h^2 Bhat^T p.
#pragma once

#include "stk_q3.h"

namespace stk {
namespace q3d {

constexpr int NA = 4;
constexpr int NN = 64;                 // nodes (and Gauss points) per cell
constexpr int NQ = 64;
constexpr int NL = 192;                // velocity unknowns per cell
constexpr int NP = 10;                 // pressure unknowns per cell
constexpr int PA = 5;                  // star-interior nodes per axis
constexpr int PN = 125;
constexpr int PU = 375;                // unknowns of a star patch (padded at the boundary)
constexpr int TB = 6;                  // 64-wide tile rows of a patch (384 padded)
constexpr int TT = 21;                 // lower tiles of a patch
constexpr int64_t TS = (int64_t)TT * 4096;   // doubles per patch in the full-tile layout (setup)
// Stored inverses: the 15 off-diagonal tiles full, the 6 diagonal tiles as
// their lower 4 x 4 blocks in row bands (band b = rows 4b..4b+3, columns
// 0..4b+3, row-major; band b starts at 8 b (b + 1)), so a tile takes 2,176
// doubles instead of 4,096.
constexpr int DS = 2176;
constexpr int64_t PS = (int64_t)(TT - TB) * 4096 + (int64_t)TB * DS;   // doubles per stored patch inverse
// offset of tile tt = I (I + 1) / 2 + J (J <= I) in a stored inverse: the
// I diagonal tiles of the rows above are the short ones
__host__ __device__ constexpr int64_t tile_off(int tt, int I) { return (int64_t)tt * 4096 - (int64_t)I * (4096 - DS); }
// patches assembled and inverted per setup pass (the full-tile staging)
constexpr int kPatchBatch = 2048;

constexpr int kPe[NP][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                            {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};

struct Tab1 {
  double gx[NA], gw[NA];
  double L[NA][NA];      // [point i][basis a] = l_a(x_i)
  double D[NA][NA];      // [point i][basis a] = l_a'(x_i)
  double M0[3][NA], M1[3][NA];
  double P[5];
  double mhinv[NP][NP];
  constexpr Tab1() : gx(), gw(), L(), D(), M0(), M1(), P(), mhinv() {
    for (int i = 0; i < NA; ++i) {
      gx[i] = q3::kGx[i];
      gw[i] = q3::kGw[i];
      for (int a = 0; a < NA; ++a) {
        L[i][a] = q3::lag(a, gx[i]);
        D[i][a] = q3::dlag(a, gx[i]);
      }
    }
    for (int e = 0; e < 3; ++e)
      for (int a = 0; a < NA; ++a) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < NA; ++i) {
          s0 += gw[i] * q3::ipow_c(gx[i] - 0.5, e) * L[i][a];
          s1 += gw[i] * q3::ipow_c(gx[i] - 0.5, e) * D[i][a];
        }
        M0[e][a] = s0;
        M1[e][a] = s1;
      }
    for (int e = 0; e < 5; ++e) {
      double s = 0.0;
      for (int i = 0; i < NA; ++i) s += gw[i] * q3::ipow_c(gx[i] - 0.5, e);
      P[e] = s;
    }
    double a[NP][2 * NP] = {};
    for (int m = 0; m < NP; ++m)
      for (int k = 0; k < NP; ++k) {
        a[m][k] = P[kPe[m][0] + kPe[k][0]] * P[kPe[m][1] + kPe[k][1]] * P[kPe[m][2] + kPe[k][2]];
        a[m][NP + k] = m == k ? 1.0 : 0.0;
      }
    for (int k = 0; k < NP; ++k) {
      const double p = a[k][k];
      for (int j = 0; j < 2 * NP; ++j) a[k][j] /= p;
      for (int i = 0; i < NP; ++i) {
        if (i == k) continue;
        const double f = a[i][k];
        for (int j = 0; j < 2 * NP; ++j) a[i][j] -= f * a[k][j];
      }
    }
    for (int m = 0; m < NP; ++m)
      for (int k = 0; k < NP; ++k) mhinv[m][k] = a[m][NP + k];
  }
};

static __constant__ Tab1 cT1 = Tab1();

// Reference gradient of basis n at Gauss point q.
__device__ inline void grad_phi(int q, int n, double g[3]) {
  const Tab1& T = cT1;
  const int qi = q & 3, qj = (q >> 2) & 3, qk = q >> 4;
  const int a = n & 3, b = (n >> 2) & 3, c = n >> 4;
  const double l0 = T.L[qi][a], l1 = T.L[qj][b], l2 = T.L[qk][c];
  g[0] = T.D[qi][a] * l1 * l2;
  g[1] = l0 * T.D[qj][b] * l2;
  g[2] = l0 * l1 * T.D[qk][c];
}

__device__ inline double phi(int q, int n) {
  const Tab1& T = cT1;
  return T.L[q & 3][n & 3] * T.L[(q >> 2) & 3][(n >> 2) & 3] * T.L[q >> 4][n >> 4];
}

__device__ inline double gauss_w(int q) {
  const Tab1& T = cT1;
  return T.gw[q & 3] * T.gw[(q >> 2) & 3] * T.gw[q >> 4];
}

// Bhat[m][comp * 64 + n]
__device__ inline double bhat(int m, int comp, int n) {
  const Tab1& T = cT1;
  const int nn[3] = {n & 3, (n >> 2) & 3, n >> 4};
  double v = 1.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) v *= (k == comp ? T.M1[kPe[m][k]][nn[k]] : T.M0[kPe[m][k]][nn[k]]);
  return v;
}

// psi_m at Gauss point q
__device__ inline double psi(int m, int q) {
  const Tab1& T = cT1;
  const double x0 = T.gx[q & 3] - 0.5, x1 = T.gx[(q >> 2) & 3] - 0.5, x2 = T.gx[q >> 4] - 0.5;
  double v = 1.0;
  for (int e = 0; e < kPe[m][0]; ++e) v *= x0;
  for (int e = 0; e < kPe[m][1]; ++e) v *= x1;
  for (int e = 0; e < kPe[m][2]; ++e) v *= x2;
  return v;
}

__device__ inline bool bnd_node3(const LevelGeo& g, int i0, int i1, int i2) {
  const int e = 3 * g.N;
  return i0 == 0 || i1 == 0 || i2 == 0 || i0 == e || i1 == e || i2 == e;
}

}  // namespace q3d
}  // namespace stk

namespace stk {
// Host launchers of the 3D degree-3 pieces (k_q3d.hip, k_coarse.hip).
// Cell matrices of A_gamma on level l: CM[cell][192][192] (full).
void q3d_cell_matrices(const Hier& H, const Level& l, double* CM, hipStream_t s);
// In-place -A^{-1} of `count` SPD matrices of nb x nb 64-wide tiles.
void launch_tile_invert_batched(const Hier& H, double* A, int nb, int64_t count, int64_t as, double* work,
                                int64_t ws, hipStream_t s);
void q3d_mu_sinker(const Hier& H, const Level& l, double* out, hipStream_t s);
void q3d_rhs_elem(const Hier& H, const Level& l, hipStream_t s);
void q3d_elem(const Hier& H, const Level& l, int mode, const double* u, const double* p, double* pout,
              hipStream_t s);
void q3d_gather(const Hier& H, const Level& l, const double* base, double alpha, double* out, hipStream_t s);
void q3d_winv_setup(const Hier& H, const Level& l, hipStream_t s);
void q3d_schur_setup(const Hier& H, const Level& l, hipStream_t s);
void q3d_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp, hipStream_t s);
void q3d_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s);
void q3d_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s);
void q3d_asm_solves(const Hier& H, const Level& l, const double* r, double* zbuf, hipStream_t s);
void q3d_asm_gather(const Hier& H, const Level& l, const double* zbuf, double* y, hipStream_t s);
void q3d_center_solve(const Hier& H, const Level& fine, const double* in, double* out, double alpha,
                      bool accumulate, hipStream_t s);
void q3d_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const double* xc, double* xf,
                     hipStream_t s);
void q3d_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const double* rf, double* rc,
                      hipStream_t s);
}  // namespace stk
