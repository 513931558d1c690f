// Kernels of the [Q3]^2 x P2disc discretisation (velocity degree k = 3; the
// discretisation of the paper's main Q3 experiments, Sections 3, 4 and
// 5.2.1), on the same level layout and with the same semantics as the Q2
// launchers that route to them: the cell kernel of A_gamma / B / B^T and its
// node gather, the cellwise W and Schur blocks, the vertex-star patch
// inverses and solves (Section 4.1, eq. (viim): 50 unknowns at an interior
// vertex, (2k-1)^d nodes), the local solves of the robust prolongation on
// coarse-cell interiors (Section 4.2, eq. (Ptilde)) and the standard Q3
// prolongation and its transpose.
//
// Every output is a fixed-order sum with no atomics, so repeated calls give
// bit-identical results.
#include "stk_dev.h"
#include "stk_q3d.h"
#include "stk_reduce.h"

namespace stk {
namespace q3 {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__device__ inline bool bnd_node(const LevelGeo& g, int i0, int i1) {
  return i0 == 0 || i1 == 0 || i0 == 3 * g.N || i1 == 3 * g.N;
}

// ---------------------------------------------------------------------------
// Cell kernel: element vectors E[cell][comp * 16 + n] of the terms in MODE
// (EL_VISC, EL_AUG, EL_BT) and, with EL_BOUT, (B u)_K into pout. Four cells
// per 64-lane workgroup, 16 lanes per cell, by sum factorisation: the
// gradients at the 16 Gauss points in two 1D contractions (y, then x; lane t
// owns one point of each intermediate), the weighted stress at Gauss point t,
// the pressure moments (B-hat u)_m = sum_q w_q psi_m(q) div u(q) (B-hat is
// this Gauss sum) by butterflies over the cell's 16 lanes, the augmented and
// B^T terms as pi(q) = w_q sum_m psi_m(q) t_m on the stress diagonal, and the
// transposed contractions (x, then y) back to node t. The 1D tables are copied
// to LDS first (no constant-table read with a lane-dependent row).
template <int MODE>
__global__ void __launch_bounds__(64) k3_elem(LevelGeo g, const double* __restrict__ mu,
                                              const double* __restrict__ winv, double gamma,
                                              const double* __restrict__ u, const double* __restrict__ p,
                                              double* __restrict__ E, double* __restrict__ pout) {
  const Tab& T = cQ3;
  const q3d::Tab1& T1 = q3d::cT1;
  __shared__ double R0[4][4 * NN];
  __shared__ double R1[4][4 * NN];
  __shared__ double sT[40];   // L[4][4], D[4][4], gx[4], gw[4]
  const int c = threadIdx.x >> 4, t = threadIdx.x & 15, t0 = t & 3, t1 = t >> 2;
  const int64_t cell0 = (int64_t)blockIdx.x * 4 + c;
  const bool valid = cell0 < g.ncell;
  const int64_t cell = valid ? cell0 : g.ncell - 1;   // lanes past the end take part in the barriers
  const int c0 = (int)(cell % g.N), c1 = (int)(cell / g.N);
  if (threadIdx.x < 16) {
    sT[threadIdx.x] = T1.L[threadIdx.x >> 2][threadIdx.x & 3];
    sT[16 + threadIdx.x] = T1.D[threadIdx.x >> 2][threadIdx.x & 3];
  } else if (threadIdx.x < 20) {
    sT[32 + threadIdx.x - 16] = T1.gx[threadIdx.x - 16];
    sT[36 + threadIdx.x - 16] = T1.gw[threadIdx.x - 16];
  }
  constexpr bool NEED_U = (MODE & (EL_VISC | EL_AUG | EL_BOUT)) != 0;
  constexpr bool NEED_T = (MODE & (EL_AUG | EL_BT)) != 0;
  if (NEED_U) {
    const int i0 = 3 * c0 + t0, i1 = 3 * c1 + t1;
    const bool b = bnd_node(g, i0, i1);
    const int64_t nd = (int64_t)i0 + (int64_t)g.n1 * i1;
    R0[c][t] = b ? 0.0 : u[nd];
    R0[c][NN + t] = b ? 0.0 : u[g.nnodes + nd];
  }
  __syncthreads();
  const double* Lt = sT;         // Lt[4 * point + basis]
  const double* Dt = sT + 16;
  const double x0 = sT[32 + t0] - 0.5, x1 = sT[32 + t1] - 0.5;
  const double wq = sT[36 + t0] * sT[36 + t1];
  const double ps[NP] = {1.0, x0, x1, x0 * x0, x0 * x1, x1 * x1};
  double S[3] = {0.0, 0.0, 0.0};   // weighted stress at Gauss point t: (0,0), (1,1), (0,1)
  double tm[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) tm[m] = 0.0;
  if (NEED_U) {
    // y: lane (a, j) = (t0, t1); AL = sum_b L[j][b] u(a, b), AD = sum_b D[j][b] u(a, b)
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      double al = 0.0, ad = 0.0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const double v = R0[c][comp * NN + t0 + 4 * bb];
        al += Lt[4 * t1 + bb] * v;
        ad += Dt[4 * t1 + bb] * v;
      }
      R1[c][(2 * comp) * NN + t] = al;
      R1[c][(2 * comp + 1) * NN + t] = ad;
    }
    __syncthreads();
    // x: lane (i, j) = (t0, t1); G[comp][0] = sum_a D[i][a] AL(a, j), G[comp][1] = sum_a L[i][a] AD(a, j)
    double G[2][2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      double g0 = 0.0, g1 = 0.0;
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        g0 += Dt[4 * t0 + aa] * R1[c][(2 * comp) * NN + aa + 4 * t1];
        g1 += Lt[4 * t0 + aa] * R1[c][(2 * comp + 1) * NN + aa + 4 * t1];
      }
      G[comp][0] = g0;
      G[comp][1] = g1;
    }
    if (MODE & EL_VISC) {
      const double wm = wq * mu[cell * NQ + t];
      S[0] = wm * 2.0 * G[0][0];
      S[1] = wm * 2.0 * G[1][1];
      S[2] = wm * (G[0][1] + G[1][0]);
    }
    if (MODE & (EL_AUG | EL_BOUT)) {
      const double dq = wq * (G[0][0] + G[1][1]);
      double sp[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        double v = dq * ps[m];
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        sp[m] = v;
      }
      if (MODE & EL_BOUT) {
#pragma unroll
        for (int m = 0; m < NP; ++m)
          if (t == m && valid) pout[cell * NP + m] = -g.h * sp[m];
      }
      if (MODE & EL_AUG) {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) s += (winv ? winv[cell * NP * NP + m * NP + k] : T.mhinv[m][k]) * sp[k];
          tm[m] = gamma * s;
        }
      }
    }
  }
  if (MODE & EL_BT) {
#pragma unroll
    for (int m = 0; m < NP; ++m) tm[m] -= g.h * p[cell * NP + m];
  }
  if (NEED_T) {
    double pi = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) pi += ps[m] * tm[m];
    pi *= wq;
    S[0] += pi;
    S[1] += pi;
  }
  // stress rows: comp 0 (S0, S2), comp 1 (S2, S1); R0 is free (the y stage read it)
#pragma unroll
  for (int k = 0; k < 3; ++k) R0[c][k * NN + t] = S[k];
  __syncthreads();
  constexpr int kRow[2][2] = {{0, 2}, {2, 1}};
  // x: lane (a, j) = (t0, t1); X0 = sum_i D[i][a] F0(i, j), X1 = sum_i L[i][a] F1(i, j)
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int o = ii + 4 * t1;
      v0 += Dt[4 * ii + t0] * R0[c][kRow[comp][0] * NN + o];
      v1 += Lt[4 * ii + t0] * R0[c][kRow[comp][1] * NN + o];
    }
    R1[c][(2 * comp) * NN + t] = v0;
    R1[c][(2 * comp + 1) * NN + t] = v1;
  }
  __syncthreads();
  // y: lane n = (a, b) = (t0, t1); e = sum_j L[j][b] X0(a, j) + D[j][b] X1(a, j)
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    double e = 0.0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int o = t0 + 4 * jj;
      e += Lt[4 * jj + t1] * R1[c][(2 * comp) * NN + o] + Dt[4 * jj + t1] * R1[c][(2 * comp + 1) * NN + o];
    }
    if (valid) E[cell * NL + comp * NN + t] = e;
  }
}

// out[idx] = base[idx] + alpha * sum of the element outputs of the cells
// containing the node (ascending y, then x); 0 on Dirichlet nodes.
__global__ void k3_gather(LevelGeo g, const double* __restrict__ E, const double* __restrict__ base, double alpha,
                          double* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 2 * g.nnodes) return;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  const int i0 = (int)(nd % g.n1), i1 = (int)(nd / g.n1);
  if (bnd_node(g, i0, i1)) {
    out[idx] = 0.0;
    return;
  }
  int ca0[2], la0[2], ca1[2], la1[2];
  const int n0 = node_cells(i0, g.N, ca0, la0), n1 = node_cells(i1, g.N, ca1, la1);
  double s = 0.0;
  for (int t1 = 0; t1 < n1; ++t1)
    for (int t0 = 0; t0 < n0; ++t0) {
      const int64_t cell = (int64_t)ca0[t0] + (int64_t)g.N * ca1[t1];
      s += E[cell * NL + comp * NN + la0[t0] + NA * la1[t1]];
    }
  out[idx] = (base ? base[idx] : 0.0) + alpha * s;
}

// ---------------------------------------------------------------------------
// In-register Gauss-Jordan inverse of a small SPD matrix.
__device__ inline void small_inverse(double (&M)[NP][NP], double (&X)[NP][NP]) {
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) X[a][b] = a == b ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double piv = 1.0 / M[k][k];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      M[k][b] *= piv;
      X[k][b] *= piv;
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      if (a == k) continue;
      const double f = M[a][k];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        M[a][b] -= f * M[k][b];
        X[a][b] -= f * X[k][b];
      }
    }
  }
}

// Reference weighted pressure mass sum_q w_q / mu_q psi psi^T of a cell.
__device__ inline void weighted_mass(const double* __restrict__ mu, int64_t cell, double (&M)[NP][NP]) {
  constexpr const Tab& T = RefQ3::T;
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) M[a][b] = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double wq = T.w[q] / mu[cell * NQ + q];
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
      for (int b = 0; b < NP; ++b) M[a][b] += wq * T.psi[q][a] * T.psi[q][b];
  }
}

// W = M_p(1/mu): per cell the inverse reference weighted mass (M_K(1/mu) = h^2 times it).
__global__ void k3_winv_setup(LevelGeo g, const double* __restrict__ mu, double* __restrict__ winv) {
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double M[NP][NP], X[NP][NP];
  weighted_mass(mu, cell, M);
  small_inverse(M, X);
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) winv[cell * NP * NP + a * NP + b] = X[a][b];
}

// Schur blocks (eq. (P1P2)): P1 M_K(1/mu)^{-1} + gamma M_K^{-1}, P2 (1 + gamma) M_K(1/mu)^{-1}.
__global__ void k3_schur_setup(LevelGeo g, const double* __restrict__ mu, double gamma, int p2,
                               double* __restrict__ Sinv) {
  constexpr const Tab& T = RefQ3::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double M[NP][NP], X[NP][NP];
  weighted_mass(mu, cell, M);
  small_inverse(M, X);
  const double ivol = 1.0 / (g.h * g.h);
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      double v = ivol * X[a][b];
      if (p2) v *= 1.0 + gamma;
      else v += gamma * ivol * T.mhinv[a][b];
      Sinv[cell * NP * NP + a * NP + b] = v;
    }
}

// z_p = -Sinv (v_p - B y) per cell (y == NULL: z_p = -Sinv v_p).
__global__ void k3_schur_apply(LevelGeo g, const double* __restrict__ Sinv, const double* __restrict__ y,
                               const double* __restrict__ vp, double* __restrict__ zp) {
  constexpr const Tab& T = RefQ3::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const int c0 = (int)(cell % g.N), c1 = (int)(cell / g.N);
  double bu[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) bu[m] = 0.0;
  if (y) {
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      const int i0 = 3 * c0 + n % NA, i1 = 3 * c1 + n / NA;
      if (bnd_node(g, i0, i1)) continue;
      const int64_t nd = (int64_t)i0 + (int64_t)g.n1 * i1;
      const double v0 = y[nd], v1 = y[g.nnodes + nd];
#pragma unroll
      for (int m = 0; m < NP; ++m) bu[m] += T.bhat[m][n] * v0 + T.bhat[m][NN + n] * v1;
    }
  }
  double t[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) t[m] = vp[cell * NP + m] + g.h * bu[m];
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b) s += Sinv[cell * NP * NP + a * NP + b] * t[b];
    zp[cell * NP + a] = -s;
  }
}

// Zero mean: int_K p = h^2 (p_0 + (p_x2 + p_y2) / 12); the mean is removed
// from the constant coefficients. Deterministic partials, then every block
// reduces them in the same order.
__global__ void k3_pmean_partials(int64_t ncell, const double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x)
    s += p[c * NP] + (p[c * NP + 3] + p[c * NP + 5]) * (1.0 / 12.0);
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k3_pmean_subtract(int64_t ncell, const double* __restrict__ part, int nparts, double* __restrict__ p) {
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
// Star patches. The patch of vertex (v0, v1) holds the 5 x 5 nodes 3v - 2 ..
// 3v + 2 per axis, both components (unknown i = comp * 25 + a0 + 5 a1); at
// the boundary the nodes outside the domain interior keep an identity row,
// so every patch has 50 unknowns and their solves leave those entries zero.
__device__ inline bool patch_node(const LevelGeo& g, int vert, int i, int& comp, int& n0, int& n1) {
  const int nv = g.N + 1;
  const int v0 = vert % nv, v1 = vert / nv;
  comp = i / PN;
  const int a = i - comp * PN;
  n0 = 3 * v0 - 2 + a % PA;
  n1 = 3 * v1 - 2 + a / PA;
  return n0 >= 1 && n1 >= 1 && n0 <= 3 * g.N - 1 && n1 <= 3 * g.N - 1;
}

// One workgroup per patch: the patch matrix (entries of the assembled
// A_gamma) in LDS, inverted through its Cholesky factor, stored as a packed
// lower triangle interleaved in blocks of 64 patches (element k of patch s
// at ((s/64) * PP + k) * 64 + s % 64).
__global__ void __launch_bounds__(64) k3_patch_setup(LevelGeo g, const double* __restrict__ mu,
                                                     const double* __restrict__ winv, double gamma,
                                                     const int* __restrict__ verts, int count,
                                                     double* __restrict__ inv, int* __restrict__ flag) {
  constexpr int ld = PU + 1;
  __shared__ double a[PU * ld];
  __shared__ double tmp[PU];
  __shared__ int bad;
  const int s = blockIdx.x;
  if (s >= count) return;
  if (threadIdx.x == 0) bad = 0;
  const int vert = verts[s];
  for (int t = threadIdx.x; t < PU * PU; t += blockDim.x) {
    const int i = t / PU, j = t % PU;
    if (j > i) continue;
    int ci, i0, i1, cj, j0, j1;
    const bool vi = patch_node(g, vert, i, ci, i0, i1);
    const bool vj = patch_node(g, vert, j, cj, j0, j1);
    const double v = (vi && vj) ? global_entry(g, mu, winv, gamma, ci, i0, i1, cj, j0, j1) : (i == j ? 1.0 : 0.0);
    a[i * ld + j] = v;
    a[j * ld + i] = v;
  }
  __syncthreads();
  spd_invert_lds(a, PU, ld, tmp, &bad);
  double* dst = inv + ((int64_t)(s / 64) * PP) * 64 + (s % 64);
  for (int i = 0; i < PU; ++i)
    for (int j = threadIdx.x; j <= i; j += blockDim.x) dst[((int64_t)i * (i + 1) / 2 + j) * 64] = a[i * ld + j];
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// y = A_s^{-1} x for patch s from the packed interleaved lower triangle:
// row i takes a_ij x_j for j <= i and column j < i takes a_ij x_i, in the
// order the packed entries are read.
__device__ inline void patch_symv(const double* __restrict__ inv, int s, const double (&x)[PU], double (&y)[PU]) {
  const double* A = inv + ((int64_t)(s / 64) * PP) * 64 + (s % 64);
#pragma unroll
  for (int i = 0; i < PU; ++i) y[i] = 0.0;
  int k = 0;
#pragma unroll
  for (int i = 0; i < PU; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const double aij = A[(int64_t)k * 64];
      ++k;
      y[i] += aij * x[j];
      if (j < i) y[j] += aij * x[i];
    }
  }
}

// Patch solves of one ASM application: zbuf[i * nvert + vert] = (A_s^{-1} r_s)_i.
__global__ void __launch_bounds__(64) k3_asm_solves(LevelGeo g, const int* __restrict__ verts, int count,
                                                    const double* __restrict__ inv, const double* __restrict__ r,
                                                    double* __restrict__ zbuf, int nvert) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= count) return;
  const int vert = verts[s];
  double x[PU], y[PU];
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    int c, n0, n1;
    const bool v = patch_node(g, vert, i, c, n0, n1);
    x[i] = v ? r[c * g.nnodes + (int64_t)n0 + (int64_t)g.n1 * n1] : 0.0;
  }
  patch_symv(inv, s, x, y);
#pragma unroll
  for (int i = 0; i < PU; ++i) zbuf[(int64_t)i * nvert + vert] = y[i];
}

// y[idx] = sum over the patches containing the node of their results
// (ascending vertex y, then x); 0 on Dirichlet nodes.
__global__ void k3_asm_gather(LevelGeo g, const double* __restrict__ zbuf, int nvert, double* __restrict__ y) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 2 * g.nnodes) return;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  const int i0 = (int)(nd % g.n1), i1 = (int)(nd / g.n1);
  if (bnd_node(g, i0, i1)) {
    y[idx] = 0.0;
    return;
  }
  // vertices v with |3v - i| <= 2: one for i = 3m, two (m, m + 1) otherwise
  const int lo0 = i0 / 3, lo1 = i1 / 3;
  const int cnt0 = i0 % 3 ? 2 : 1, cnt1 = i1 % 3 ? 2 : 1;
  const int nv = g.N + 1;
  double s = 0.0;
  for (int t1 = 0; t1 < cnt1; ++t1)
    for (int t0 = 0; t0 < cnt0; ++t0) {
      const int v0 = lo0 + t0, v1 = lo1 + t1;
      const int a0 = i0 - (3 * v0 - 2), a1 = i1 - (3 * v1 - 2);
      s += zbuf[(int64_t)(comp * PN + a0 + PA * a1) * nvert + v0 + nv * v1];
    }
  y[idx] = s;
}

// Local solves of the robust transfer: for every coarse cell K (lex order),
// z = A_K^{-1} in|_K with A_K the star patch of the fine vertex 2K + 1
// (patch slot lex(K): the centre vertices come first in the patch list);
// out|_K = (ACC ? out|_K : 0) + alpha z. The coarse-cell interiors are
// disjoint, so each node is written by one lane.
template <bool ACC>
__global__ void __launch_bounds__(64) k3_center_solve(LevelGeo g, const double* __restrict__ inv,
                                                      const double* __restrict__ in, double* __restrict__ out,
                                                      double alpha) {
  const int nc = g.N / 2;
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= nc * nc) return;
  const int k0 = s % nc, k1 = s / nc;
  double x[PU], y[PU];
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    const int c = i / PN, a = i % PN;
    const int64_t nd = (int64_t)(6 * k0 + 1 + a % PA) + (int64_t)g.n1 * (6 * k1 + 1 + a / PA);
    x[i] = in[c * g.nnodes + nd];
  }
  patch_symv(inv, s, x, y);
  // with ACC, all 50 old values are loaded before the first store (loads and
  // stores interleaved per entry would each wait for the previous store)
  if (ACC) {
#pragma unroll
    for (int i = 0; i < PU; ++i) {
      const int c = i / PN, a = i % PN;
      x[i] = out[c * g.nnodes + (int64_t)(6 * k0 + 1 + a % PA) + (int64_t)g.n1 * (6 * k1 + 1 + a / PA)];
    }
  }
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    const int c = i / PN, a = i % PN;
    const int64_t idx = c * g.nnodes + (int64_t)(6 * k0 + 1 + a % PA) + (int64_t)g.n1 * (6 * k1 + 1 + a / PA);
    out[idx] = ACC ? x[i] + alpha * y[i] : alpha * y[i];
  }
}

// ---------------------------------------------------------------------------
// Standard prolongation: the coarse Q3 field at the fine nodes. Fine node i
// lies in coarse cell i / 6 at offset r = i mod 6 (r = 6 at the last node).
__global__ void k3_prolong_std(LevelGeo gc, LevelGeo gf, const double* __restrict__ xc, double* __restrict__ xf) {
  constexpr const Tab& T = RefQ3::T;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 2 * gf.nnodes) return;
  const int comp = (int)(idx / gf.nnodes);
  const int64_t nd = idx - (int64_t)comp * gf.nnodes;
  const int i0 = (int)(nd % gf.n1), i1 = (int)(nd / gf.n1);
  if (bnd_node(gf, i0, i1)) {
    xf[idx] = 0.0;
    return;
  }
  int C0 = i0 / 6, r0 = i0 % 6, C1 = i1 / 6, r1 = i1 % 6;
  if (C0 == gc.N) { C0 = gc.N - 1; r0 = 6; }
  if (C1 == gc.N) { C1 = gc.N - 1; r1 = 6; }
  double s = 0.0;
  for (int a1 = 0; a1 < NA; ++a1)
    for (int a0 = 0; a0 < NA; ++a0) {
      const double w = T.prol[r0][a0] * T.prol[r1][a1];
      const int j0 = 3 * C0 + a0, j1 = 3 * C1 + a1;
      if (w == 0.0 || bnd_node(gc, j0, j1)) continue;
      s += w * xc[comp * gc.nnodes + (int64_t)j0 + (int64_t)gc.n1 * j1];
    }
  xf[idx] = s;
}

// rc = P^T rf: for an interior coarse node every fine node of its stencil is
// interior, so the sum runs over the product of the two 1D stencils (kRT:
// compile-time offsets and weights selected by j mod 3, 7 slots per axis).
__global__ void k3_restrict_std(LevelGeo gf, LevelGeo gc, const double* __restrict__ rf, double* __restrict__ rc) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= 2 * gc.nnodes) return;
  const int comp = (int)(idx / gc.nnodes);
  const int64_t nd = idx - (int64_t)comp * gc.nnodes;
  const int j[2] = {(int)(nd % gc.n1), (int)(nd / gc.n1)};
  if (bnd_node(gc, j[0], j[1])) {
    rc[idx] = 0.0;
    return;
  }
  int len[2];
  int64_t off[2][7];
  double w[2][7];
  const int64_t stride[2] = {1, gf.n1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int a = j[k] % 3, base = 6 * (j[k] / 3);
    len[k] = a == 0 ? kRT.n[0] : (a == 1 ? kRT.n[1] : kRT.n[2]);
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) {
      const int o = a == 0 ? kRT.off[0][sl] : (a == 1 ? kRT.off[1][sl] : kRT.off[2][sl]);
      off[k][sl] = (int64_t)(base + o) * stride[k];
      w[k][sl] = a == 0 ? kRT.w[0][sl] : (a == 1 ? kRT.w[1][sl] : kRT.w[2][sl]);
    }
  }
  const double* src = rf + comp * gf.nnodes;
  double s = 0.0;
#pragma unroll
  for (int s1 = 0; s1 < 7; ++s1) {
    if (s1 >= len[1]) break;
    const double* row = src + off[1][s1];
    double s0v = 0.0;
#pragma unroll
    for (int s0 = 0; s0 < 7; ++s0) s0v += w[0][s0] * row[off[0][s0]];
    s += w[1][s1] * s0v;
  }
  rc[idx] = s;
}

}  // namespace q3

// ---------------------------------------------------------------------------
using namespace q3;

void q3_elem(const Hier& H, const Level& l, int mode, const double* u, const double* p, double* pout,
             hipStream_t s) {
  if (H.dim == 3) return q3d_elem(H, l, mode, u, p, pout, s);
  const dim3 grid(nblk(l.g.ncell, 4)), blk(64);
  switch (mode) {
    case EL_VISC | EL_AUG:
      hipLaunchKernelGGL(k3_elem<EL_VISC | EL_AUG>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_AUG:
      hipLaunchKernelGGL(k3_elem<EL_AUG>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_BT:
      hipLaunchKernelGGL(k3_elem<EL_BT>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma, u, p, l.E, pout);
      break;
    case EL_VISC | EL_AUG | EL_BT | EL_BOUT:
      hipLaunchKernelGGL(k3_elem<EL_VISC | EL_AUG | EL_BT | EL_BOUT>, grid, blk, 0, s, l.g, l.mu, l.winv, H.gamma,
                         u, p, l.E, pout);
      break;
    default:
      break;
  }
}

void q3_gather(const Hier& H, const Level& l, const double* base, double alpha, double* out, hipStream_t s) {
  if (H.dim == 3) return q3d_gather(H, l, base, alpha, out, s);
  (void)H;
  hipLaunchKernelGGL(k3_gather, dim3(nblk(2 * l.g.nnodes, 256)), dim3(256), 0, s, l.g, (const double*)l.E, base,
                     alpha, out);
}

void q3_winv_setup(const Hier& H, const Level& l, hipStream_t s) {
  if (H.dim == 3) return q3d_winv_setup(H, l, s);
  (void)H;
  hipLaunchKernelGGL(k3_winv_setup, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, (const double*)l.mu, l.winv);
}

void q3_schur_setup(const Hier& H, const Level& l, hipStream_t s) {
  if (H.dim == 3) return q3d_schur_setup(H, l, s);
  hipLaunchKernelGGL(k3_schur_setup, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, (const double*)l.mu, H.gamma,
                     H.schur == 2 ? 1 : 0, H.Sinv);
}

void q3_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp, hipStream_t s) {
  if (H.dim == 3) return q3d_schur_apply(H, l, y, vp, zp, s);
  hipLaunchKernelGGL(k3_schur_apply, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, (const double*)H.Sinv, y, vp,
                     zp);
}

void q3_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s) {
  if (H.dim == 3) return q3d_project_mean(H, l, p, s);
  const int np = red_parts(l.g.ncell);
  hipLaunchKernelGGL(k3_pmean_partials, dim3(np), dim3(red_threads(l.g.ncell)), 0, s, l.g.ncell, (const double*)p,
                     H.partials);
  hipLaunchKernelGGL(k3_pmean_subtract, dim3(nblk(l.g.ncell, 256)), dim3(256), 0, s, l.g.ncell,
                     (const double*)H.partials, np, p);
}

void q3_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s) {
  if (H.dim == 3) return q3d_patch_setup(H, l, pc, s);
  if (pc.count == 0) return;
  hipLaunchKernelGGL(k3_patch_setup, dim3(pc.count), dim3(64), 0, s, l.g, (const double*)l.mu,
                     (const double*)l.winv, H.gamma, (const int*)pc.verts, pc.count, pc.inv, H.flag);
}

void q3_asm_solves(const Hier& H, const Level& l, const double* r, double* zbuf, hipStream_t s) {
  if (H.dim == 3) return q3d_asm_solves(H, l, r, zbuf, s);
  (void)H;
  const PatchClass& pc = l.cls[0];
  hipLaunchKernelGGL(k3_asm_solves, dim3(nblk(pc.count, 64)), dim3(64), 0, s, l.g, (const int*)pc.verts, pc.count,
                     (const double*)pc.inv, r, zbuf, l.nvert);
}

void q3_asm_gather(const Hier& H, const Level& l, const double* zbuf, double* y, hipStream_t s) {
  if (H.dim == 3) return q3d_asm_gather(H, l, zbuf, y, s);
  (void)H;
  hipLaunchKernelGGL(k3_asm_gather, dim3(nblk(2 * l.g.nnodes, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
}

void q3_center_solve(const Hier& H, const Level& fine, const double* in, double* out, double alpha,
                     bool accumulate, hipStream_t s) {
  if (H.dim == 3) return q3d_center_solve(H, fine, in, out, alpha, accumulate, s);
  (void)H;
  const int nc = fine.g.N / 2;
  const dim3 grid(nblk((int64_t)nc * nc, 64)), blk(64);
  const double* inv = fine.cls[0].inv;
  if (accumulate) hipLaunchKernelGGL(k3_center_solve<true>, grid, blk, 0, s, fine.g, inv, in, out, alpha);
  else hipLaunchKernelGGL(k3_center_solve<false>, grid, blk, 0, s, fine.g, inv, in, out, alpha);
}

void q3_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const double* xc, double* xf,
                    hipStream_t s) {
  if (H.dim == 3) return q3d_prolong_std(H, coarse, fine, xc, xf, s);
  (void)H;
  hipLaunchKernelGGL(k3_prolong_std, dim3(nblk(2 * fine.g.nnodes, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
}

void q3_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const double* rf, double* rc,
                     hipStream_t s) {
  if (H.dim == 3) return q3d_restrict_std(H, fine, coarse, rf, rc, s);
  (void)H;
  hipLaunchKernelGGL(k3_restrict_std, dim3(nblk(2 * coarse.g.nnodes, 256)), dim3(256), 0, s, fine.g, coarse.g, rf,
                     rc);
}

}  // namespace stk
