// [Q3]^2 x P2disc on axis-aligned squares (Section 4, definition of V_h^k
// and Q_h^{k-1} with k = 3): reference tables evaluated at compile time, and
// the device helpers shared by the degree-3 kernels.
//
// Velocity basis: tensor products of the cubic Lagrange polynomials on the
// equispaced nodes {0, 1/3, 2/3, 1}; local node n = a + 4b (x fastest), local
// unknown j = comp * 16 + n. Pressure basis on a cell: the monomials 1, x, y,
// x^2, xy, y^2 of (xi - 1/2) in reference coordinates (total degree <= 2,
// discontinuous; with x = (x_phys - c_K)/h on the physical cell). Quadrature:
// tensor 4-point Gauss-Legendre, exact through degree 7 per axis.
//
// Level layout (as for Q2, with 3N + 1 nodes per axis): the stored velocity
// vector is the full node grid, component-major, x fastest, zero on the
// Dirichlet boundary; pressure unknowns are cell-major, 6 per cell.
//
// Cell operator (2D, so the h^{d-2} factor of the viscous and augmented terms
// is 1):
//   A_K u = sum_q w_q mu_q [(G + G^T) : dphi],   G = reference gradient of u
//   G_K u = gamma Bhat^T W^{-1} Bhat u,  W^{-1} = Mhat^{-1} (W = M_p) or the
//           cell's inverse reference weighted mass (W = M_p(1/mu))
//   (B u)_K = -h Bhat u,   (B^T p)_K = -h Bhat^T p,
// with Bhat[m][j] = sum_q w_q psi_m div(phi_j) and Mhat[m][n] = sum_q w_q psi_m psi_n.
#pragma once

#include "stk_internal.h"

namespace stk {
namespace q3 {

constexpr int NA = 4;                 // nodes (and Gauss points) per axis of a cell
constexpr int NN = 16;                // nodes per cell
constexpr int NQ = 16;                // Gauss points per cell
constexpr int NL = 32;                // velocity unknowns per cell
constexpr int NP = 6;                 // pressure unknowns per cell
constexpr int PA = 5;                 // star-interior nodes per axis (2k - 1)
constexpr int PN = PA * PA;           // star-interior nodes
constexpr int PU = 2 * PN;            // unknowns of a star patch (padded at the boundary)
constexpr int PP = PU * (PU + 1) / 2; // packed lower triangle

// Gauss-Legendre 4-point rule on [0, 1]
constexpr double kGx[4] = {0.069431844202973712388, 0.33000947820757186760, 0.66999052179242813240,
                           0.93056815579702628761};
constexpr double kGw[4] = {0.17392742256872692869, 0.32607257743127307131, 0.32607257743127307131,
                           0.17392742256872692869};
constexpr double kNd[4] = {0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0};

// Lagrange cubic l_a on kNd (product formula) and its derivative.
constexpr double lag(int a, double x) {
  double v = 1.0;
  for (int b = 0; b < NA; ++b)
    if (b != a) v *= (x - kNd[b]) / (kNd[a] - kNd[b]);
  return v;
}
constexpr double dlag(int a, double x) {
  double den = 1.0;
  for (int b = 0; b < NA; ++b)
    if (b != a) den *= kNd[a] - kNd[b];
  double s = 0.0;
  for (int skip = 0; skip < NA; ++skip) {
    if (skip == a) continue;
    double p = 1.0;
    for (int b = 0; b < NA; ++b)
      if (b != a && b != skip) p *= x - kNd[b];
    s += p;
  }
  return s / den;
}

// exponents of the pressure monomials
constexpr int kPe[NP][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}};

constexpr double ipow_c(double x, int e) {
  double v = 1.0;
  for (int i = 0; i < e; ++i) v *= x;
  return v;
}

struct Tab {
  double w[NQ];             // Gauss weight of point q = a + 4b
  double phi[NQ][NN];       // [q][n] basis value
  double dphi[NQ][NN][2];   // [q][n][k] reference gradient
  double psi[NQ][NP];       // [q][m] pressure basis
  double bhat[NP][NL];      // [m][j] reference divergence moments
  double mhat[NP][NP];      // reference pressure mass
  double mhinv[NP][NP];     // its inverse
  double prol[7][NA];       // l_a(r / 6): coarse basis a at fine offset r of a coarse cell
  constexpr Tab() : w(), phi(), dphi(), psi(), bhat(), mhat(), mhinv(), prol() {
    for (int q = 0; q < NQ; ++q) {
      const int qa = q % NA, qb = q / NA;
      w[q] = kGw[qa] * kGw[qb];
      const double x = kGx[qa], y = kGx[qb];
      for (int m = 0; m < NP; ++m) psi[q][m] = ipow_c(x - 0.5, kPe[m][0]) * ipow_c(y - 0.5, kPe[m][1]);
      for (int n = 0; n < NN; ++n) {
        const int a = n % NA, b = n / NA;
        phi[q][n] = lag(a, x) * lag(b, y);
        dphi[q][n][0] = dlag(a, x) * lag(b, y);
        dphi[q][n][1] = lag(a, x) * dlag(b, y);
      }
    }
    for (int m = 0; m < NP; ++m) {
      for (int c = 0; c < 2; ++c)
        for (int n = 0; n < NN; ++n) {
          double s = 0.0;
          for (int q = 0; q < NQ; ++q) s += w[q] * psi[q][m] * dphi[q][n][c];
          bhat[m][c * NN + n] = s;
        }
      for (int k = 0; k < NP; ++k) {
        double s = 0.0;
        for (int q = 0; q < NQ; ++q) s += w[q] * psi[q][m] * psi[q][k];
        mhat[m][k] = s;
      }
    }
    // Gauss-Jordan inverse of the SPD reference mass (no pivoting needed)
    double a[NP][2 * NP] = {};
    for (int i = 0; i < NP; ++i)
      for (int j = 0; j < NP; ++j) {
        a[i][j] = mhat[i][j];
        a[i][NP + j] = i == j ? 1.0 : 0.0;
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
    for (int i = 0; i < NP; ++i)
      for (int j = 0; j < NP; ++j) mhinv[i][j] = a[i][NP + j];
    for (int r = 0; r <= 6; ++r)
      for (int c = 0; c < NA; ++c) prol[r][c] = lag(c, (double)r / 6.0);
  }
};

struct RefQ3 {
  static constexpr Tab T{};
};

// 1D restriction stencils of a coarse node of local index a = j mod 3 in its
// cell: the fine offsets from 6 C (C = j / 3) with nonzero prolongation
// weight, in 7 slots (a = 0: a cell vertex, weights from both neighbouring
// cells; a = 1, 2: four entries, the remaining slots weight 0 at a valid
// offset).
struct RestrictTab {
  int n[3];
  int off[3][7];
  double w[3][7];
  constexpr RestrictTab() : n(), off(), w() {
    constexpr const Tab& T = RefQ3::T;
    for (int a = 0; a < 3; ++a) {
      int k = 0;
      for (int t = -5; t <= 5; ++t) {
        double wt = 0.0;
        if (a == 0) wt = t < 0 ? T.prol[6 + t][3] : T.prol[t][0];
        else if (t >= 1) wt = T.prol[t][a];
        if (wt == 0.0) continue;
        off[a][k] = t;
        w[a][k] = wt;
        ++k;
      }
      n[a] = k;
      for (int q = k; q < 7; ++q) {
        off[a][q] = off[a][0];
        w[a][q] = 0.0;
      }
    }
  }
};
constexpr RestrictTab kRT{};

// Runtime-indexed copy in constant memory.
static __constant__ Tab cQ3 = Tab();

// Cells containing node i along one axis (one cell for a node inside a cell,
// two at a vertex, clipped to the mesh), lowest first; returns the count.
__host__ __device__ inline int node_cells(int i, int N, int cell[2], int loc[2]) {
  if (i % 3) {
    cell[0] = cell[1] = i / 3;
    loc[0] = loc[1] = i % 3;
    return 1;
  }
  const int v = i / 3;
  int n = 0;
  if (v > 0) { cell[n] = v - 1; loc[n] = 3; ++n; }
  if (v < N) { cell[n] = v; loc[n] = 0; ++n; }
  if (n == 1) { cell[1] = cell[0]; loc[1] = loc[0]; }
  return n;
}

// Contribution of `cell` to the A_gamma entry between (ci, local node na)
// and (cj, local node nb): sum_q w_q mu_q [delta_{ci,cj} grad phi_a . grad
// phi_b + d_cj phi_a d_ci phi_b] + gamma sum_{m,k} Bhat[m][ci,na] W^{-1}[m][k] Bhat[k][cj,nb].
__device__ inline double cell_entry(const double* __restrict__ mu, const double* __restrict__ winv, int64_t cell,
                                    double gamma, int ci, int na, int cj, int nb) {
  const Tab& T = cQ3;
  double s = 0.0;
  for (int q = 0; q < NQ; ++q) {
    double gg = T.dphi[q][na][cj] * T.dphi[q][nb][ci];
    if (ci == cj) gg += T.dphi[q][na][0] * T.dphi[q][nb][0] + T.dphi[q][na][1] * T.dphi[q][nb][1];
    s += T.w[q] * mu[cell * NQ + q] * gg;
  }
  double al = 0.0;
  for (int m = 0; m < NP; ++m) {
    double t = 0.0;
    for (int k = 0; k < NP; ++k)
      t += (winv ? winv[cell * NP * NP + m * NP + k] : T.mhinv[m][k]) * T.bhat[k][cj * NN + nb];
    al += T.bhat[m][ci * NN + na] * t;
  }
  return s + gamma * al;
}

// A_gamma entry between (ci, node (i0, i1)) and (cj, node (j0, j1)) of the
// level: the sum over the cells that contain both nodes (ascending y, then x).
__device__ inline double global_entry(const LevelGeo& g, const double* __restrict__ mu,
                                      const double* __restrict__ winv, double gamma, int ci, int i0, int i1, int cj,
                                      int j0, int j1) {
  int ca0[2], la0[2], ca1[2], la1[2], cb0[2], lb0[2], cb1[2], lb1[2];
  const int na0 = node_cells(i0, g.N, ca0, la0), na1 = node_cells(i1, g.N, ca1, la1);
  const int nb0 = node_cells(j0, g.N, cb0, lb0), nb1 = node_cells(j1, g.N, cb1, lb1);
  double s = 0.0;
  for (int t1 = 0; t1 < na1; ++t1)
    for (int u1 = 0; u1 < nb1; ++u1) {
      if (ca1[t1] != cb1[u1]) continue;
      for (int t0 = 0; t0 < na0; ++t0)
        for (int u0 = 0; u0 < nb0; ++u0) {
          if (ca0[t0] != cb0[u0]) continue;
          const int64_t cell = (int64_t)ca0[t0] + (int64_t)g.N * ca1[t1];
          s += cell_entry(mu, winv, cell, gamma, ci, la0[t0] + NA * la1[t1], cj, lb0[u0] + NA * lb1[u1]);
        }
    }
  return s;
}

}  // namespace q3
}  // namespace stk
