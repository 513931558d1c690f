// Reference-cell tables for [Q2]^d x P1disc on axis-aligned cells, evaluated
// at compile time so that fully unrolled kernels see them as immediates.
//
// Velocity basis: tensor products of the quadratic Lagrange polynomials on the
// nodes {0, 1/2, 1} (Section 4, definition of V_h^k with k = 2):
//   l0 = 2(x-1/2)(x-1),  l1 = 4x(1-x),  l2 = 2x(x-1/2).
// Pressure basis on a cell (total degree 1, discontinuous; Section 4,
// definition of Q_h^{k-1}): psi_0 = 1, psi_k = xi_k - 1/2 in reference
// coordinates (= (x_k - c_k)/h on the physical cell).
// Quadrature: tensor 3-point Gauss-Legendre on [0,1]: 1/2 -+ sqrt(3/5)/2,
// 1/2 with weights 5/18, 8/18, 5/18 (exact through degree 5 per axis).
//
// Local numbering: node n = a + 3b + 9c (x fastest), quadrature point q
// likewise, element unknown j = comp * 3^d + n.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stk {

constexpr double kHalfSqrt35 = 0.38729833462074168852;   // sqrt(3/5)/2
constexpr double kGaussX[3] = {0.5 - kHalfSqrt35, 0.5, 0.5 + kHalfSqrt35};
constexpr double kGaussW[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

constexpr double lag(int a, double x) {
  return a == 0 ? 2.0 * (x - 0.5) * (x - 1.0) : (a == 1 ? 4.0 * x * (1.0 - x) : 2.0 * x * (x - 0.5));
}
constexpr double dlag(int a, double x) {
  return a == 0 ? 4.0 * x - 3.0 : (a == 1 ? 4.0 - 8.0 * x : 4.0 * x - 1.0);
}

template <int D>
struct Dims {
  static constexpr int NN = D == 2 ? 9 : 27;   // nodes (and Gauss points) per cell
  static constexpr int NQ = NN;
  static constexpr int NL = D * NN;            // velocity unknowns per cell
  static constexpr int NP = D + 1;             // pressure unknowns per cell
  static constexpr int NN5 = D == 2 ? 25 : 125;  // fine nodes of a coarse cell
};

constexpr int digit(int n, int k) { return k == 0 ? n % 3 : (k == 1 ? (n / 3) % 3 : n / 9); }

// Storage index of entry (a, b) of a symmetric d x d tensor: the diagonal
// first, then (0,1) [, (0,2), (1,2)].
template <int D>
struct SymIdx {
  static constexpr int NS = D * (D + 1) / 2;
  static constexpr int at(int a, int b) {
    return a == b ? a : (D == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
  }
};

// Reference tables for dimension D.
template <int D>
struct RefTab {
  static constexpr int NN = Dims<D>::NN;
  static constexpr int NL = Dims<D>::NL;
  static constexpr int NP = Dims<D>::NP;
  double w[NN];             // quadrature weight of point q
  double phi[NN][NN];       // [q][n] basis value
  double dphi[NN][NN][D];   // [q][n][k] reference gradient
  double psi[NN][NP];       // [q][m] pressure basis
  double bhat[NP][NL];      // [m][j] = sum_q w psi_m dphi_j(comp)  (reference divergence moments)
  double mhat[NP];          // reference pressure mass (diagonal): 1, 1/12, ..
  constexpr RefTab() : w(), phi(), dphi(), psi(), bhat(), mhat() {
    for (int q = 0; q < NN; ++q) {
      double wq = 1.0;
      for (int k = 0; k < D; ++k) wq *= kGaussW[digit(q, k)];
      w[q] = wq;
      psi[q][0] = 1.0;
      for (int k = 0; k < D; ++k) psi[q][k + 1] = kGaussX[digit(q, k)] - 0.5;
      for (int n = 0; n < NN; ++n) {
        double v = 1.0;
        for (int k = 0; k < D; ++k) v *= lag(digit(n, k), kGaussX[digit(q, k)]);
        phi[q][n] = v;
        for (int j = 0; j < D; ++j) {
          double g = 1.0;
          for (int k = 0; k < D; ++k) {
            const double x = kGaussX[digit(q, k)];
            g *= (k == j) ? dlag(digit(n, k), x) : lag(digit(n, k), x);
          }
          dphi[q][n][j] = g;
        }
      }
    }
    mhat[0] = 1.0;
    for (int k = 1; k < NP; ++k) mhat[k] = 1.0 / 12.0;
    for (int m = 0; m < NP; ++m)
      for (int c = 0; c < D; ++c)
        for (int n = 0; n < NN; ++n) {
          double s = 0.0;
          for (int q = 0; q < NN; ++q) s += w[q] * psi[q][m] * dphi[q][n][c];
          bhat[m][c * NN + n] = s;
        }
  }
};

template <int D>
struct Ref {
  static constexpr RefTab<D> T{};
};

// Exact 1D prolongation weights: value of coarse l_a at fine offset r/4 of a
// coarse cell, r = 0..4.
constexpr double kProlW[5][3] = {
    {1.0, 0.0, 0.0}, {0.375, 0.75, -0.125}, {0.0, 1.0, 0.0}, {-0.125, 0.75, 0.375}, {0.0, 0.0, 1.0}};

// ---------------------------------------------------------------------------
// Level geometry (index arithmetic only; no stored connectivity).
struct LevelGeo {
  int N;          // cells per axis
  int n1;         // nodes per axis = 2N+1
  int64_t nnodes; // n1^d
  int64_t ncell;  // N^d
  double h;       // 1/N
};

template <int D>
__host__ __device__ inline int64_t node_index(const LevelGeo& g, int i0, int i1, int i2) {
  return D == 2 ? (int64_t)i0 + (int64_t)g.n1 * i1
                : (int64_t)i0 + (int64_t)g.n1 * ((int64_t)i1 + (int64_t)g.n1 * i2);
}

template <int D>
__host__ __device__ inline int64_t cell_index(const LevelGeo& g, int c0, int c1, int c2) {
  return D == 2 ? (int64_t)c0 + (int64_t)g.N * c1
                : (int64_t)c0 + (int64_t)g.N * ((int64_t)c1 + (int64_t)g.N * c2);
}

}  // namespace stk
