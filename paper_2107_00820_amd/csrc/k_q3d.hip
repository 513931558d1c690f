// Kernels of [Q3]^3 x P2disc (velocity degree 3 on hexahedra), on the same
// level layout and with the same semantics as the Q2 launchers that route
// to them: the cell kernel of A_gamma / B / B^T and its node gather, the
// cellwise W and Schur blocks, the cell matrices, the vertex-star patch
// inverses (Section 4.1, eq. (viim): 375 unknowns at an interior vertex)
// and their solves, the local solves of the robust prolongation on
// coarse-cell interiors (Section 4.2, eq. (Ptilde)) and the standard Q3
// prolongation and its transpose.
//
// A 375-unknown star does not fit a workgroup's LDS, so its matrix is
// assembled from the cell matrices into 64 x 64 tiles in device memory and
// inverted there by the coarse level's symmetric sweep, batched over the
// patches; a patch solve is a tile GEMV of one workgroup. Every output is a
// fixed-order sum (no atomics): repeated calls are bit-identical.
#include "stk_dev.h"
#include "stk_q3d.h"
#include "stk_reduce.h"

namespace stk {
namespace q3d {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
constexpr int64_t kCM = (int64_t)NL * NL;   // doubles per cell matrix

__device__ inline void cell3(const LevelGeo& g, int64_t cell, int c[3]) {
  c[0] = (int)(cell % g.N);
  c[1] = (int)((cell / g.N) % g.N);
  c[2] = (int)(cell / ((int64_t)g.N * g.N));
}

__device__ inline int64_t node3(const LevelGeo& g, int i0, int i1, int i2) {
  return (int64_t)i0 + (int64_t)g.n1 * ((int64_t)i1 + (int64_t)g.n1 * i2);
}

// ---------------------------------------------------------------------------
// Cell kernel: one 64-lane workgroup per cell, by sum factorisation over the
// tensor-product basis. Forward: the reference gradient of each component at
// the 64 Gauss points from the 64 nodal values in three 1D contractions
// (z, then y, then x; lane t owns one point of each intermediate tensor).
// Lane q then forms the weighted stress at Gauss point q, and the pressure
// moments (B-hat u)_m = sum_q w_q psi_m(q) div u(q) (the 4-point rule is
// exact for these products, so this equals B-hat u) by butterfly sums that
// leave the same value in every lane. The augmented and B^T terms enter as
// pi(q) = w_q sum_m psi_m(q) t_m on the stress diagonal, since
// sum_m Bhat[m][c, n] t_m = sum_q d_c phi_n(q) pi(q). Backward: the
// transposed contractions (x, then y, then z) give the outputs of node t.
// Two LDS regions of 9 x 64 doubles alternate between the stages.
template <int MODE>
__global__ void __launch_bounds__(64) k3d_elem(LevelGeo g, const double* __restrict__ mu,
                                               const double* __restrict__ winv, double gamma,
                                               const double* __restrict__ u, const double* __restrict__ p,
                                               double* __restrict__ E, double* __restrict__ pout) {
  const Tab1& T = cT1;
  __shared__ double R0[9 * 64];
  __shared__ double R1[9 * 64];
  __shared__ double sT[40];   // L[4][4], D[4][4], gx[4], gw[4]
  const int64_t cell = blockIdx.x;
  const int t = threadIdx.x;
  const int t0 = t & 3, t1 = (t >> 2) & 3, t2 = t >> 4;
  if (t < 16) {
    sT[t] = T.L[t >> 2][t & 3];
    sT[16 + t] = T.D[t >> 2][t & 3];
  } else if (t < 20) {
    sT[32 + (t - 16)] = T.gx[t - 16];
    sT[36 + (t - 16)] = T.gw[t - 16];
  }
  __syncthreads();
  const double* Lt = sT;         // Lt[4 * point + basis]
  const double* Dt = sT + 16;
  const double* gxt = sT + 32;
  const double* gwt = sT + 36;
  constexpr bool NEED_U = (MODE & (EL_VISC | EL_AUG | EL_BOUT)) != 0;
  constexpr bool NEED_T = (MODE & (EL_AUG | EL_BT)) != 0;
  double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double tm[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) tm[m] = 0.0;
  if (NEED_U) {
    int c[3];
    cell3(g, cell, c);
    {
      const int i0 = 3 * c[0] + t0, i1 = 3 * c[1] + t1, i2 = 3 * c[2] + t2;
      const bool b = bnd_node3(g, i0, i1, i2);
      const int64_t nd = node3(g, i0, i1, i2);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) R0[comp * 64 + t] = b ? 0.0 : u[comp * g.nnodes + nd];
    }
    __syncthreads();
    // z: lane (a, b, k); AL = sum_c L[k][c] u, AD = sum_c D[k][c] u
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      double al = 0.0, ad = 0.0;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const double v = R0[comp * 64 + t0 + 4 * t1 + 16 * cc];
        al += Lt[4 * t2 + cc] * v;
        ad += Dt[4 * t2 + cc] * v;
      }
      R1[(2 * comp) * 64 + t] = al;
      R1[(2 * comp + 1) * 64 + t] = ad;
    }
    __syncthreads();
    // y: lane (a, j, k); LL = sum_b L[j][b] AL, DL = sum_b D[j][b] AL, LD = sum_b L[j][b] AD
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      double ll = 0.0, dl = 0.0, ld = 0.0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const double al = R1[(2 * comp) * 64 + t0 + 4 * bb + 16 * t2];
        const double ad = R1[(2 * comp + 1) * 64 + t0 + 4 * bb + 16 * t2];
        ll += Lt[4 * t1 + bb] * al;
        dl += Dt[4 * t1 + bb] * al;
        ld += Lt[4 * t1 + bb] * ad;
      }
      R0[(3 * comp) * 64 + t] = ll;
      R0[(3 * comp + 1) * 64 + t] = dl;
      R0[(3 * comp + 2) * 64 + t] = ld;
    }
    __syncthreads();
    // x: lane q = (i, j, k); G[comp][dir]
    double G[3][3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const int o = aa + 4 * t1 + 16 * t2;
        g0 += Dt[4 * t0 + aa] * R0[(3 * comp) * 64 + o];
        g1 += Lt[4 * t0 + aa] * R0[(3 * comp + 1) * 64 + o];
        g2 += Lt[4 * t0 + aa] * R0[(3 * comp + 2) * 64 + o];
      }
      G[comp][0] = g0;
      G[comp][1] = g1;
      G[comp][2] = g2;
    }
    const double wq = gwt[t0] * gwt[t1] * gwt[t2];
    if (MODE & EL_VISC) {
      const double wm = wq * mu[cell * NQ + t] * g.h;
      S[0] = 2.0 * wm * G[0][0];
      S[1] = 2.0 * wm * G[1][1];
      S[2] = 2.0 * wm * G[2][2];
      S[3] = wm * (G[0][1] + G[1][0]);
      S[4] = wm * (G[0][2] + G[2][0]);
      S[5] = wm * (G[1][2] + G[2][1]);
    }
    if (MODE & (EL_AUG | EL_BOUT)) {
      const double dq = wq * (G[0][0] + G[1][1] + G[2][2]);
      const double x0 = gxt[t0] - 0.5, x1 = gxt[t1] - 0.5, x2 = gxt[t2] - 0.5;
      const double ps[NP] = {1.0, x0, x1, x2, x0 * x0, x0 * x1, x0 * x2, x1 * x1, x1 * x2, x2 * x2};
      double sp[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        double v = dq * ps[m];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        sp[m] = v;
      }
      if (MODE & EL_BOUT) {
#pragma unroll
        for (int m = 0; m < NP; ++m)
          if (t == m) pout[cell * NP + m] = -g.h * g.h * sp[m];
      }
      if (MODE & EL_AUG) {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) s += (winv ? winv[cell * NP * NP + m * NP + k] : T.mhinv[m][k]) * sp[k];
          tm[m] = gamma * g.h * s;
        }
      }
    }
  }
  if (MODE & EL_BT) {
#pragma unroll
    for (int m = 0; m < NP; ++m) tm[m] -= g.h * g.h * p[cell * NP + m];
  }
  if (NEED_T) {
    const double x0 = gxt[t0] - 0.5, x1 = gxt[t1] - 0.5, x2 = gxt[t2] - 0.5;
    const double ps[NP] = {1.0, x0, x1, x2, x0 * x0, x0 * x1, x0 * x2, x1 * x1, x1 * x2, x2 * x2};
    double pi = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) pi += ps[m] * tm[m];
    pi *= gwt[t0] * gwt[t1] * gwt[t2];
    S[0] += pi;
    S[1] += pi;
    S[2] += pi;
  }
  // weighted stress rows at Gauss point t: comp 0 (S0 S3 S4), 1 (S3 S1 S5), 2 (S4 S5 S2)
#pragma unroll
  for (int k = 0; k < 6; ++k) R1[k * 64 + t] = S[k];
  __syncthreads();
  constexpr int kRow[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  // x: lane (a, j, k); X0 = sum_i D[i][a] F0, X1 = sum_i L[i][a] F1, X2 = sum_i L[i][a] F2
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int o = ii + 4 * t1 + 16 * t2;
      x0 += Dt[4 * ii + t0] * R1[kRow[comp][0] * 64 + o];
      x1 += Lt[4 * ii + t0] * R1[kRow[comp][1] * 64 + o];
      x2 += Lt[4 * ii + t0] * R1[kRow[comp][2] * 64 + o];
    }
    R0[(3 * comp) * 64 + t] = x0;
    R0[(3 * comp + 1) * 64 + t] = x1;
    R0[(3 * comp + 2) * 64 + t] = x2;
  }
  __syncthreads();
  // y: lane (a, b, k); Y0 = sum_j L[j][b] X0 + D[j][b] X1, Y2 = sum_j L[j][b] X2
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    double y0 = 0.0, y2 = 0.0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int o = t0 + 4 * jj + 16 * t2;
      y0 += Lt[4 * jj + t1] * R0[(3 * comp) * 64 + o] + Dt[4 * jj + t1] * R0[(3 * comp + 1) * 64 + o];
      y2 += Lt[4 * jj + t1] * R0[(3 * comp + 2) * 64 + o];
    }
    R1[(2 * comp) * 64 + t] = y0;
    R1[(2 * comp + 1) * 64 + t] = y2;
  }
  __syncthreads();
  // z: lane n = (a, b, c); e = sum_k L[k][c] Y0 + D[k][c] Y2
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    double e = 0.0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int o = t0 + 4 * t1 + 16 * kk;
      e += Lt[4 * kk + t2] * R1[(2 * comp) * 64 + o] + Dt[4 * kk + t2] * R1[(2 * comp + 1) * 64 + o];
    }
    E[cell * NL + comp * NN + t] = e;
  }
}

// out[idx] = base[idx] + alpha * sum over the cells containing the node
// (ascending z, y, x); 0 on Dirichlet nodes.
__global__ void k3d_gather(LevelGeo g, const double* __restrict__ E, const double* __restrict__ base, double alpha,
                           double* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 3 * g.nnodes) return;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  const int i0 = (int)(nd % g.n1), i1 = (int)((nd / g.n1) % g.n1), i2 = (int)(nd / ((int64_t)g.n1 * g.n1));
  if (bnd_node3(g, i0, i1, i2)) {
    out[idx] = 0.0;
    return;
  }
  int ca[3][2], la[3][2], na[3];
  na[0] = q3::node_cells(i0, g.N, ca[0], la[0]);
  na[1] = q3::node_cells(i1, g.N, ca[1], la[1]);
  na[2] = q3::node_cells(i2, g.N, ca[2], la[2]);
  double s = 0.0;
  for (int t2 = 0; t2 < na[2]; ++t2)
    for (int t1 = 0; t1 < na[1]; ++t1)
      for (int t0 = 0; t0 < na[0]; ++t0) {
        const int64_t cell = (int64_t)ca[0][t0] + (int64_t)g.N * ((int64_t)ca[1][t1] + (int64_t)g.N * ca[2][t2]);
        s += E[cell * NL + comp * NN + la[0][t0] + 4 * la[1][t1] + 16 * la[2][t2]];
      }
  out[idx] = (base ? base[idx] : 0.0) + alpha * s;
}

// ---------------------------------------------------------------------------
template <int N>
__device__ inline void small_inverse_n(double (&M)[N][N], double (&X)[N][N]) {
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) X[a][b] = a == b ? 1.0 : 0.0;
  for (int k = 0; k < N; ++k) {
    const double piv = 1.0 / M[k][k];
    for (int b = 0; b < N; ++b) {
      M[k][b] *= piv;
      X[k][b] *= piv;
    }
    for (int a = 0; a < N; ++a) {
      if (a == k) continue;
      const double f = M[a][k];
      for (int b = 0; b < N; ++b) {
        M[a][b] -= f * M[k][b];
        X[a][b] -= f * X[k][b];
      }
    }
  }
}

__device__ inline void weighted_mass3(const double* __restrict__ mu, int64_t cell, double (&M)[NP][NP]) {
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) M[a][b] = 0.0;
  for (int q = 0; q < NQ; ++q) {
    const double wq = gauss_w(q) / mu[cell * NQ + q];
    double ps[NP];
    for (int m = 0; m < NP; ++m) ps[m] = psi(m, q);
    for (int a = 0; a < NP; ++a)
      for (int b = 0; b < NP; ++b) M[a][b] += wq * ps[a] * ps[b];
  }
}

__global__ void k3d_winv_setup(LevelGeo g, const double* __restrict__ mu, double* __restrict__ winv) {
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double M[NP][NP], X[NP][NP];
  weighted_mass3(mu, cell, M);
  small_inverse_n<NP>(M, X);
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) winv[cell * NP * NP + a * NP + b] = X[a][b];
}

__global__ void k3d_schur_setup(LevelGeo g, const double* __restrict__ mu, double gamma, int p2,
                                double* __restrict__ Sinv) {
  const Tab1& T = cT1;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double M[NP][NP], X[NP][NP];
  weighted_mass3(mu, cell, M);
  small_inverse_n<NP>(M, X);
  const double ivol = 1.0 / (g.h * g.h * g.h);
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) {
      double v = ivol * X[a][b];
      if (p2) v *= 1.0 + gamma;
      else v += gamma * ivol * T.mhinv[a][b];
      Sinv[cell * NP * NP + a * NP + b] = v;
    }
}

// z_p = -Sinv (v_p - B y) per cell (y == NULL: z_p = -Sinv v_p).
__global__ void k3d_schur_apply(LevelGeo g, const double* __restrict__ Sinv, const double* __restrict__ y,
                                const double* __restrict__ vp, double* __restrict__ zp) {
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  int c[3];
  cell3(g, cell, c);
  double bu[NP];
  for (int m = 0; m < NP; ++m) bu[m] = 0.0;
  if (y) {
    for (int n = 0; n < NN; ++n) {
      const int i0 = 3 * c[0] + (n & 3), i1 = 3 * c[1] + ((n >> 2) & 3), i2 = 3 * c[2] + (n >> 4);
      if (bnd_node3(g, i0, i1, i2)) continue;
      const int64_t nd = node3(g, i0, i1, i2);
      const double v0 = y[nd], v1 = y[g.nnodes + nd], v2 = y[2 * g.nnodes + nd];
      for (int m = 0; m < NP; ++m) bu[m] += bhat(m, 0, n) * v0 + bhat(m, 1, n) * v1 + bhat(m, 2, n) * v2;
    }
  }
  double t[NP];
  for (int m = 0; m < NP; ++m) t[m] = vp[cell * NP + m] + g.h * g.h * bu[m];
  for (int a = 0; a < NP; ++a) {
    double s = 0.0;
    for (int b = 0; b < NP; ++b) s += Sinv[cell * NP * NP + a * NP + b] * t[b];
    zp[cell * NP + a] = -s;
  }
}

// Zero mean: int_K p = h^3 (p_0 + (p_x2 + p_y2 + p_z2) / 12).
__global__ void k3d_pmean_partials(int64_t ncell, const double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x)
    s += p[c * NP] + (p[c * NP + 4] + p[c * NP + 7] + p[c * NP + 9]) * (1.0 / 12.0);
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k3d_pmean_subtract(int64_t ncell, const double* __restrict__ part, int nparts,
                                   double* __restrict__ p) {
  __shared__ double mean;
  if (threadIdx.x < 64) {
    const double s = wave_reduce_parts(part, nparts, 1, 0);
    if (threadIdx.x == 0) mean = s / (double)ncell;
  }
  __syncthreads();
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x)
    p[c * NP] -= mean;
}

// ---------------------------------------------------------------------------
// Cell matrices CM[cell][i][j] of A_gamma (i, j = comp * 64 + node): h sum_q
// w_q mu_q [delta_{ci,cj} grad phi_a . grad phi_b + d_cj phi_a d_ci phi_b] +
// gamma h sum_m Bhat[m][i] (W^{-1} Bhat)[m][j]. One workgroup per cell; the
// Gauss points go in four groups of 16 whose basis gradients are staged in
// LDS, each group's terms added to the entries in place (fixed order).
__global__ void __launch_bounds__(256) k3d_cellmat(LevelGeo g, const double* __restrict__ mu,
                                                   const double* __restrict__ winv, double gamma,
                                                   double* __restrict__ CM) {
  const Tab1& T = cT1;
  constexpr int QG = 16;
  __shared__ double gr[QG][NN][3];
  __shared__ double wmu[NQ];
  __shared__ double Bh[NP][NL];
  __shared__ double WB[NP][NL];
  const int64_t cell = blockIdx.x;
  for (int q = threadIdx.x; q < NQ; q += blockDim.x) wmu[q] = gauss_w(q) * mu[cell * NQ + q] * g.h;
  for (int e = threadIdx.x; e < NP * NL; e += blockDim.x) {
    const int m = e / NL, j = e % NL;
    Bh[m][j] = bhat(m, j / NN, j % NN);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NP * NL; e += blockDim.x) {
    const int m = e / NL, j = e % NL;
    double t = 0.0;
    for (int k = 0; k < NP; ++k) t += (winv ? winv[cell * NP * NP + m * NP + k] : T.mhinv[m][k]) * Bh[k][j];
    WB[m][j] = t;
  }
  double* out = CM + cell * kCM;
  for (int qg = 0; qg < NQ / QG; ++qg) {
    __syncthreads();
    for (int e = threadIdx.x; e < QG * NN; e += blockDim.x) {
      const int q = e / NN, n = e % NN;
      double v[3];
      grad_phi(QG * qg + q, n, v);
      gr[q][n][0] = v[0];
      gr[q][n][1] = v[1];
      gr[q][n][2] = v[2];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NL * NL; e += blockDim.x) {
      const int i = e / NL, j = e % NL;
      const int ci = i / NN, a = i % NN, cj = j / NN, b = j % NN;
      double s;
      if (qg == 0) {
        double al = 0.0;
        for (int m = 0; m < NP; ++m) al += Bh[m][i] * WB[m][j];
        s = gamma * g.h * al;
      } else {
        s = out[(int64_t)i * NL + j];
      }
      for (int q = 0; q < QG; ++q) {
        double gg = gr[q][a][cj] * gr[q][b][ci];
        if (ci == cj) gg += gr[q][a][0] * gr[q][b][0] + gr[q][a][1] * gr[q][b][1] + gr[q][a][2] * gr[q][b][2];
        s += wmu[QG * qg + q] * gg;
      }
      out[(int64_t)i * NL + j] = s;
    }
  }
}

// Star patches: the patch of vertex v holds the 5^3 nodes 3v - 2 .. 3v + 2
// per axis, three components (unknown i = comp * 125 + a0 + 5 a1 + 25 a2),
// padded to 384 unknowns; nodes outside the domain interior and the padding
// keep an identity row.
__device__ inline bool patch_node3(const LevelGeo& g, int vert, int i, int& comp, int nd[3]) {
  if (i >= PU) return false;
  const int nv = g.N + 1;
  const int v0 = vert % nv, v1 = (vert / nv) % nv, v2 = vert / (nv * nv);
  comp = i / PN;
  const int a = i - comp * PN;
  nd[0] = 3 * v0 - 2 + a % PA;
  nd[1] = 3 * v1 - 2 + (a / PA) % PA;
  nd[2] = 3 * v2 - 2 + a / (PA * PA);
  const int e = 3 * g.N - 1;
  return nd[0] >= 1 && nd[1] >= 1 && nd[2] >= 1 && nd[0] <= e && nd[1] <= e && nd[2] <= e;
}

__device__ inline void tile_of(int t, int& I, int& J) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// Patch matrices in the tile layout of the coarse inverse (lower tiles,
// diagonal tiles full): grid (21 tiles, patches); entries are sums of the
// cell-matrix entries of the cells that contain both nodes.
__global__ void __launch_bounds__(256) k3d_patch_assemble(LevelGeo g, const double* __restrict__ CM,
                                                          const int* __restrict__ verts, double* __restrict__ A) {
  const int t = blockIdx.x, s = blockIdx.y;
  int I, J;
  tile_of(t, I, J);
  const int vert = verts[s];
  double* T = A + (int64_t)s * TS + (int64_t)t * 4096;
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int i = 64 * I + e / 64, j = 64 * J + e % 64;
    int ci = 0, cj = 0, ni[3], nj[3];
    const bool vi = patch_node3(g, vert, i, ci, ni);
    const bool vj = patch_node3(g, vert, j, cj, nj);
    double v = i == j ? 1.0 : 0.0;
    if (vi && vj) {
      int ca[3][2], la[3][2], cb[3][2], lb[3][2], na[3], nb[3];
      for (int k = 0; k < 3; ++k) {
        na[k] = q3::node_cells(ni[k], g.N, ca[k], la[k]);
        nb[k] = q3::node_cells(nj[k], g.N, cb[k], lb[k]);
      }
      v = 0.0;
      for (int t2 = 0; t2 < na[2]; ++t2)
        for (int u2 = 0; u2 < nb[2]; ++u2) {
          if (ca[2][t2] != cb[2][u2]) continue;
          for (int t1 = 0; t1 < na[1]; ++t1)
            for (int u1 = 0; u1 < nb[1]; ++u1) {
              if (ca[1][t1] != cb[1][u1]) continue;
              for (int t0 = 0; t0 < na[0]; ++t0)
                for (int u0 = 0; u0 < nb[0]; ++u0) {
                  if (ca[0][t0] != cb[0][u0]) continue;
                  const int64_t cell =
                      (int64_t)ca[0][t0] + (int64_t)g.N * ((int64_t)ca[1][t1] + (int64_t)g.N * ca[2][t2]);
                  const int a = la[0][t0] + 4 * la[1][t1] + 16 * la[2][t2];
                  const int b = lb[0][u0] + 4 * lb[1][u1] + 16 * lb[2][u2];
                  v += CM[cell * kCM + (int64_t)(ci * NN + a) * NL + cj * NN + b];
                }
            }
        }
    }
    T[e] = v;
  }
}

// The full-tile inverses of `n` patches (A, TS apart; grid (21 tiles, n))
// into the stored layout of patches s0, s0 + 1, ..: off-diagonal tiles as
// they are, diagonal tiles as their lower 4 x 4 blocks in row bands.
__global__ void __launch_bounds__(256) k3d_patch_pack(const double* __restrict__ A, int64_t s0,
                                                      double* __restrict__ inv) {
  const int tt = blockIdx.x, s = blockIdx.y;
  int I, J;
  tile_of(tt, I, J);
  const double* src = A + (int64_t)s * TS + (int64_t)tt * 4096;
  double* dst = inv + (s0 + s) * PS + tile_off(tt, I);
  if (I != J) {
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) dst[e] = src[e];
    return;
  }
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int row = e >> 6, col = e & 63, b = row >> 2, r = row & 3;
    if (col < 4 * b + 4) dst[8 * b * (b + 1) + r * 4 * (b + 1) + col] = src[e];
  }
}

// y = A_s^{-1} x for the patch's stored -A_s^{-1} (21 tiles, the diagonal
// ones as lower 4 x 4 blocks), one 256-lane workgroup: tile by tile in a
// fixed order, thread (tr, tc) = (t / 16, t % 16) multiplies its 4 x 4 block
// (in a diagonal tile only tc <= tr, whose diagonal block is stored whole and
// used by rows only); row sums meet over the 16 lanes of a row band
// (shuffles), column sums (the transposed use of a lower block) over the 16
// bands (shuffles, then the four wavefronts through LDS in order), and one
// thread per row adds them to y: in an off-diagonal tile the row sums go to
// band I and the column sums to band J, in a diagonal tile both to band I,
// added together by one thread per row. The next tile's block is loaded
// before the current one is reduced, so its loads are in flight across the
// barrier; the partials alternate between two LDS buffers, so one barrier
// per tile separates both the partials and the updates of y of consecutive
// tiles. `part` holds 2 x 320 doubles; y is complete after the caller's next
// barrier.
__device__ inline void load_block(const double* __restrict__ T, bool diag, int tr, int tc, double m[4][4]) {
  if (diag && tc > tr) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) m[r][c] = 0.0;
    return;
  }
  const int base = diag ? 8 * tr * (tr + 1) + 4 * tc : 256 * tr + 4 * tc;
  const int stride = diag ? 4 * (tr + 1) : 64;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) m[r][c] = T[base + r * stride + c];
}

__device__ inline void patch_tile_gemv(const double* __restrict__ Ainv, const double* x, double* y, double* part) {
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15, wave = t >> 6, lane = t & 63;
  double m[4][4], mn[4][4];
  load_block(Ainv, true, tr, tc, m);
  for (int tt = 0; tt < TT; ++tt) {
    int I, J;
    tile_of(tt, I, J);
    const bool diag = I == J;
    if (tt + 1 < TT) {
      int In, Jn;
      tile_of(tt + 1, In, Jn);
      load_block(Ainv + tile_off(tt + 1, In), In == Jn, tr, tc, mn);
    }
    double rs[4], cs[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) v += m[r][c] * x[64 * J + 4 * tc + c];
      rs[r] = v;
    }
    // the column use of a diagonal tile's blocks: strictly below the diagonal only
    const bool cuse = !diag || tc < tr;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double v = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) v += m[r][c] * x[64 * I + 4 * tr + r];
      cs[c] = cuse ? v : 0.0;
    }
    // row sums over the 16 lanes of the band
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) rs[r] += __shfl_xor(rs[r], off, 64);
    // column sums over the 4 bands of the wavefront
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int off = 32; off >= 16; off >>= 1) cs[c] += __shfl_xor(cs[c], off, 64);
    double* pb = part + (tt & 1) * 320;
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < 4; ++c) pb[wave * 64 + 4 * lane + c] = cs[c];
    }
    if (diag && tc == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) pb[256 + 4 * tr + r] = rs[r];
    }
    __syncthreads();
    if (diag) {
      if (t < 64) y[64 * I + t] -= pb[256 + t] + (pb[t] + pb[64 + t] + pb[128 + t] + pb[192 + t]);
    } else {
      if (tc == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) y[64 * I + 4 * tr + r] -= rs[r];
      }
      if (t < 64) y[64 * J + t] -= pb[t] + pb[64 + t] + pb[128 + t] + pb[192 + t];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) m[r][c] = mn[r][c];
  }
}

// MODE 0: patch solves of an ASM application (residual r, outputs
// zbuf[i * nvert + vert]); MODE 1 / 2: local solves of the robust transfer
// on coarse cell s (the star of its centre vertex, patch slot s), out|_K =
// alpha z (1) or out|_K + alpha z (2).
template <int MODE>
__global__ void __launch_bounds__(256) k3d_patch_solve(LevelGeo g, const int* __restrict__ verts,
                                                       const double* __restrict__ inv, const double* __restrict__ in,
                                                       double* __restrict__ out, int nvert, double alpha) {
  __shared__ double x[64 * TB];
  __shared__ double y[64 * TB];
  __shared__ double part[2 * 320];
  const int s = blockIdx.x;
  const int vert = verts[s];
  for (int i = threadIdx.x; i < 64 * TB; i += blockDim.x) {
    int c, nd[3];
    const bool v = patch_node3(g, vert, i, c, nd);
    x[i] = v ? in[c * g.nnodes + node3(g, nd[0], nd[1], nd[2])] : 0.0;
    y[i] = 0.0;
  }
  __syncthreads();
  patch_tile_gemv(inv + (int64_t)s * PS, x, y, part);
  __syncthreads();
  for (int i = threadIdx.x; i < PU; i += blockDim.x) {
    int c, nd[3];
    const bool v = patch_node3(g, vert, i, c, nd);
    if (MODE == 0) {
      out[(int64_t)i * nvert + vert] = v ? y[i] : 0.0;
    } else if (v) {
      const int64_t idx = c * g.nnodes + node3(g, nd[0], nd[1], nd[2]);
      out[idx] = MODE == 2 ? out[idx] + alpha * y[i] : alpha * y[i];
    }
  }
}

// y[idx] = sum over the patches containing the node of their results
// (ascending vertex z, y, x); 0 on Dirichlet nodes.
__global__ void k3d_asm_gather(LevelGeo g, const double* __restrict__ zbuf, int nvert, double* __restrict__ y) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 3 * g.nnodes) return;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  const int i[3] = {(int)(nd % g.n1), (int)((nd / g.n1) % g.n1), (int)(nd / ((int64_t)g.n1 * g.n1))};
  if (bnd_node3(g, i[0], i[1], i[2])) {
    y[idx] = 0.0;
    return;
  }
  const int nv = g.N + 1;
  int lo[3], cnt[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = i[k] / 3;
    cnt[k] = i[k] % 3 ? 2 : 1;
  }
  double s = 0.0;
  for (int t2 = 0; t2 < cnt[2]; ++t2)
    for (int t1 = 0; t1 < cnt[1]; ++t1)
      for (int t0 = 0; t0 < cnt[0]; ++t0) {
        const int v0 = lo[0] + t0, v1 = lo[1] + t1, v2 = lo[2] + t2;
        const int a = (i[0] - (3 * v0 - 2)) + PA * (i[1] - (3 * v1 - 2)) + PA * PA * (i[2] - (3 * v2 - 2));
        s += zbuf[(int64_t)(comp * PN + a) * nvert + v0 + nv * (v1 + nv * v2)];
      }
  y[idx] = s;
}

// ---------------------------------------------------------------------------
// 1D weight l_a(r / 6) of the coarse cubic basis a (compile-time) at a
// lane-dependent fine offset r = 0..6, chosen among constants.
template <int A>
__device__ inline double prol3_w(int r) {
  constexpr const q3::Tab& T = q3::RefQ3::T;
  return r == 0 ? T.prol[0][A] : r == 1 ? T.prol[1][A] : r == 2 ? T.prol[2][A] : r == 3 ? T.prol[3][A]
         : r == 4 ? T.prol[4][A] : r == 5 ? T.prol[5][A] : T.prol[6][A];
}

// P_H x_c, six fine nodes per thread: the nodes 6C .. 6C+5 of one fine row
// (i1, i2) along x, at offsets r = 0..5 in coarse cell C (thread C = N_c
// owns the last node 6 N_c, a Dirichlet node). The coarse values of the
// row's (y, z) stencil (at most 4 x 4 entries, shared by the six nodes) are
// summed per coarse x-node 3C .. 3C+3 first; each output then takes its
// compile-time x weights. Coarse Dirichlet nodes contribute nothing, fine
// Dirichlet nodes are written as 0.
__global__ void k3d_prolong_std(LevelGeo gc, LevelGeo gf, const double* __restrict__ xc, double* __restrict__ xf) {
  constexpr const q3::Tab& T = q3::RefQ3::T;
  const int Nc = gc.N, nf1 = gf.n1;
  const int64_t nc1 = gc.n1;
  const int64_t per = (int64_t)nf1 * nf1 * (Nc + 1);
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 3 * per) return;
  const int comp = (int)(idx / per);
  const int64_t rem = idx - (int64_t)comp * per;
  const int C = (int)(rem % (Nc + 1));
  const int64_t row = rem / (Nc + 1);
  const int i1 = (int)(row % nf1), i2 = (int)(row / nf1);
  double* out = xf + (int64_t)comp * gf.nnodes + (int64_t)nf1 * (i1 + (int64_t)nf1 * i2) + 6 * C;
  const int e = 3 * gf.N;
  if (C == Nc || i1 == 0 || i1 == e || i2 == 0 || i2 == e) {
    const int nout = C == Nc ? 1 : 6;
    for (int k = 0; k < nout; ++k) out[k] = 0.0;
    return;
  }
  int cl1 = i1 / 6, r1 = i1 % 6, cl2 = i2 / 6, r2 = i2 % 6;
  if (cl1 == Nc) { cl1 = Nc - 1; r1 = 6; }
  if (cl2 == Nc) { cl2 = Nc - 1; r2 = 6; }
  const double w1[4] = {prol3_w<0>(r1), prol3_w<1>(r1), prol3_w<2>(r1), prol3_w<3>(r1)};
  const double w2[4] = {prol3_w<0>(r2), prol3_w<1>(r2), prol3_w<2>(r2), prol3_w<3>(r2)};
  const int ec = 3 * Nc;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  const double* src0 = xc + (int64_t)comp * gc.nnodes + 3 * C;
#pragma unroll
  for (int a2 = 0; a2 < 4; ++a2) {
    const int j2 = 3 * cl2 + a2;
    if (w2[a2] == 0.0 || j2 == 0 || j2 == ec) continue;
#pragma unroll
    for (int a1 = 0; a1 < 4; ++a1) {
      const int j1 = 3 * cl1 + a1;
      if (w1[a1] == 0.0 || j1 == 0 || j1 == ec) continue;
      const double w = w1[a1] * w2[a2];
      const double* src = src0 + nc1 * (j1 + nc1 * j2);
      t[0] += w * (C > 0 ? src[0] : 0.0);        // x-node 3C is Dirichlet for C = 0
      t[1] += w * src[1];
      t[2] += w * src[2];
      t[3] += w * (C < Nc - 1 ? src[3] : 0.0);   // x-node 3C+3 is Dirichlet for C = Nc - 1
    }
  }
#pragma unroll
  for (int r0 = 0; r0 < 6; ++r0) {
    double y = 0.0;
#pragma unroll
    for (int a0 = 0; a0 < 4; ++a0)
      if (T.prol[r0][a0] != 0.0) y += T.prol[r0][a0] * t[a0];
    out[r0] = (C == 0 && r0 == 0) ? 0.0 : y;    // fine node 0 is Dirichlet
  }
}

// rc = P^T rf for the standard prolongation: for an interior coarse node
// every fine node of its stencil is interior (a vertex has 1 <= C <= N - 1,
// the others 0 <= C <= N - 1, and the offsets lie in [-5, 5] and [1, 5]), so
// the sum runs over the tensor product of the three 1D stencils; its weights
// and offsets are compile-time constants selected by a (fixed slots, guarded
// by the stencil length), so no table is read with a lane-dependent index.
__global__ void k3d_restrict_std(LevelGeo gf, LevelGeo gc, const double* __restrict__ rf, double* __restrict__ rc) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 3 * gc.nnodes) return;
  const int comp = (int)(idx / gc.nnodes);
  const int64_t nd = idx - (int64_t)comp * gc.nnodes;
  const int j[3] = {(int)(nd % gc.n1), (int)((nd / gc.n1) % gc.n1), (int)(nd / ((int64_t)gc.n1 * gc.n1))};
  if (bnd_node3(gc, j[0], j[1], j[2])) {
    rc[idx] = 0.0;
    return;
  }
  int len[3];
  int64_t off[3][7];
  double w[3][7];
  const int64_t stride[3] = {1, gf.n1, (int64_t)gf.n1 * gf.n1};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = j[k] % 3, base = 6 * (j[k] / 3);
    len[k] = a == 0 ? q3::kRT.n[0] : (a == 1 ? q3::kRT.n[1] : q3::kRT.n[2]);
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) {
      const int o = a == 0 ? q3::kRT.off[0][sl] : (a == 1 ? q3::kRT.off[1][sl] : q3::kRT.off[2][sl]);
      off[k][sl] = (int64_t)(base + o) * stride[k];
      w[k][sl] = a == 0 ? q3::kRT.w[0][sl] : (a == 1 ? q3::kRT.w[1][sl] : q3::kRT.w[2][sl]);
    }
  }
  const double* src = rf + comp * gf.nnodes;
  double s = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < 7; ++s2) {
    if (s2 >= len[2]) break;
    double s1v = 0.0;
#pragma unroll
    for (int s1 = 0; s1 < 7; ++s1) {
      if (s1 >= len[1]) break;
      const double* row = src + off[2][s2] + off[1][s1];
      double s0v = 0.0;
#pragma unroll
      for (int s0 = 0; s0 < 7; ++s0) s0v += w[0][s0] * row[off[0][s0]];
      s1v += w[1][s1] * s0v;
    }
    s += w[2][s2] * s1v;
  }
  rc[idx] = s;
}

}  // namespace q3d

// ---------------------------------------------------------------------------
using namespace q3d;

void q3d_elem(const Hier& H, const Level& l, int mode, const double* u, const double* p, double* pout,
              hipStream_t s) {
  const dim3 grid((unsigned)l.g.ncell), blk(64);
  switch (mode) {
    case EL_VISC | EL_AUG:
      hipLaunchKernelGGL(k3d_elem<EL_VISC | EL_AUG>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_AUG:
      hipLaunchKernelGGL(k3d_elem<EL_AUG>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_BT:
      hipLaunchKernelGGL(k3d_elem<EL_BT>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_VISC | EL_AUG | EL_BT | EL_BOUT:
      hipLaunchKernelGGL(k3d_elem<EL_VISC | EL_AUG | EL_BT | EL_BOUT>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma,
                         u, p, l.E, pout);
      break;
    default:
      break;
  }
}

void q3d_gather(const Hier& H, const Level& l, const double* base, double alpha, double* out, hipStream_t s) {
  (void)H;
  hipLaunchKernelGGL(k3d_gather, dim3(nblk(3 * l.g.nnodes, 256)), dim3(256), 0, s, l.g, (const double*)l.E, base,
                     alpha, out);
}

void q3d_winv_setup(const Hier& H, const Level& l, hipStream_t s) {
  (void)H;
  hipLaunchKernelGGL(k3d_winv_setup, dim3(nblk(l.g.ncell, 64)), dim3(64), 0, s, l.g, (const double*)l.mu, l.winv);
}

void q3d_schur_setup(const Hier& H, const Level& l, hipStream_t s) {
  hipLaunchKernelGGL(k3d_schur_setup, dim3(nblk(l.g.ncell, 64)), dim3(64), 0, s, l.g, (const double*)l.mu, H.gamma,
                     H.schur == 2 ? 1 : 0, H.Sinv);
}

void q3d_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp, hipStream_t s) {
  hipLaunchKernelGGL(k3d_schur_apply, dim3(nblk(l.g.ncell, 64)), dim3(64), 0, s, l.g, (const double*)H.Sinv, y, vp,
                     zp);
}

void q3d_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s) {
  const int np = red_parts(l.g.ncell);
  hipLaunchKernelGGL(k3d_pmean_partials, dim3(np), dim3(red_threads(l.g.ncell)), 0, s, l.g.ncell, (const double*)p,
                     H.partials);
  hipLaunchKernelGGL(k3d_pmean_subtract, dim3(nblk(l.g.ncell, 256)), dim3(256), 0, s, l.g.ncell,
                     (const double*)H.partials, np, p);
}

void q3d_cell_matrices(const Hier& H, const Level& l, double* CM, hipStream_t s) {
  hipLaunchKernelGGL(k3d_cellmat, dim3((unsigned)l.g.ncell), dim3(256), 0, s, l.g, (const double*)l.mu,
                     (const double*)l.winv, H.gamma, CM);
}

// Patch inverses of a level in passes of up to kPatchBatch patches: each
// pass assembles full tiles into the staging area behind the level's cell
// matrices, inverts them in place by the batched sweep (its work, 7 tiles per
// patch, behind the staging) and packs them into the stored layout.
void q3d_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s) {
  if (pc.count == 0) return;
  q3d_cell_matrices(H, l, H.q3cm, s);
  const int64_t pass = std::min<int64_t>(pc.count, kPatchBatch);
  double* stage = H.q3cm + l.g.ncell * kCM;
  double* work = stage + pass * TS;
  for (int64_t s0 = 0; s0 < pc.count; s0 += pass) {
    const int n = (int)std::min<int64_t>(pass, pc.count - s0);
    hipLaunchKernelGGL(k3d_patch_assemble, dim3(TT, (unsigned)n), dim3(256), 0, s, l.g, (const double*)H.q3cm,
                       (const int*)pc.verts + s0, stage);
    launch_tile_invert_batched(H, stage, TB, n, TS, work, 7 * 4096, s);
    hipLaunchKernelGGL(k3d_patch_pack, dim3(TT, (unsigned)n), dim3(256), 0, s, (const double*)stage, s0, pc.inv);
  }
}

void q3d_asm_solves(const Hier& H, const Level& l, const double* r, double* zbuf, hipStream_t s) {
  (void)H;
  const PatchClass& pc = l.cls[0];
  hipLaunchKernelGGL(k3d_patch_solve<0>, dim3((unsigned)pc.count), dim3(256), 0, s, l.g, (const int*)pc.verts,
                     (const double*)pc.inv, r, zbuf, l.nvert, 1.0);
}

void q3d_asm_gather(const Hier& H, const Level& l, const double* zbuf, double* y, hipStream_t s) {
  (void)H;
  hipLaunchKernelGGL(k3d_asm_gather, dim3(nblk(3 * l.g.nnodes, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
}

void q3d_center_solve(const Hier& H, const Level& fine, const double* in, double* out, double alpha,
                      bool accumulate, hipStream_t s) {
  (void)H;
  const int nc = fine.g.N / 2;
  const unsigned ncc = (unsigned)(nc * nc * nc);
  const PatchClass& pc = fine.cls[0];
  if (accumulate)
    hipLaunchKernelGGL(k3d_patch_solve<2>, dim3(ncc), dim3(256), 0, s, fine.g, (const int*)pc.verts,
                       (const double*)pc.inv, in, out, fine.nvert, alpha);
  else
    hipLaunchKernelGGL(k3d_patch_solve<1>, dim3(ncc), dim3(256), 0, s, fine.g, (const int*)pc.verts,
                       (const double*)pc.inv, in, out, fine.nvert, alpha);
}

void q3d_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const double* xc, double* xf,
                     hipStream_t s) {
  (void)H;
  // threads: components x fine rows x (coarse cells along x + 1)
  const int64_t nf1 = fine.g.n1;
  hipLaunchKernelGGL(k3d_prolong_std, dim3(nblk(3 * nf1 * nf1 * (coarse.g.N + 1), 256)), dim3(256), 0, s, coarse.g,
                     fine.g, xc, xf);
}

void q3d_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const double* rf, double* rc,
                      hipStream_t s) {
  (void)H;
  hipLaunchKernelGGL(k3d_restrict_std, dim3(nblk(3 * coarse.g.nnodes, 256)), dim3(256), 0, s, fine.g, coarse.g, rf,
                     rc);
}

}  // namespace stk
