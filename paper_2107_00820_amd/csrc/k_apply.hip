// Matrix-free operator kernels: coefficients at Gauss points, the cell kernel
// of A_gamma / B / B^T, the deterministic node gather, the right-hand side,
// and the cellwise Schur-complement blocks.
//
// Operator (Section 2, entries after eq. (stokessys); Section 3, eq.
// (augstokessys)): on each cell K of width h
//   A_K u = h^{d-2} sum_q w_q mu_q [ (G + G^T) : dphi ]      (G = reference gradient of u)
//   G_K u = gamma h^{d-2} Bhat^T Mhat^{-1} Bhat u             (gamma B^T M_p^{-1} B, cell-local)
//   (B u)_K = -h^{d-1} Bhat u,   (B^T p)_K = -h^{d-1} Bhat^T p
// with Bhat[m][j] = int_ref psi_m div(phi_j) and Mhat = diag(1, 1/12, ..) the
// reference pressure mass matrix (W = M_p; preconditioner P1 of eq. (P1P2)).
//
// Determinism: the cell kernel writes element vectors E[cell][j]; a node
// kernel sums the <= 2^d cell contributions of each node in a fixed order.
// No atomics, so repeated applications give bit-identical results.
#include <type_traits>

#include "stk_asm_sum.h"
#include "stk_q3d.h"
#include "stk_reduce.h"

namespace stk {

// The coefficient kernels (Fourier gradients at Gauss points) keep 256-thread
// workgroups: their register use would spill at the reductions' 1024.
constexpr int kCoefThreads = 256;
inline int coef_parts(int64_t n) {
  const int64_t p = (n + kCoefThreads - 1) / kCoefThreads;
  return (int)(p < 1 ? 1 : (p > kRedBlocks ? kRedBlocks : p));
}

template <int D>
__device__ inline void cell_coords(const LevelGeo& g, int64_t cell, int c[3]) {
  c[0] = (int)(cell % g.N);
  c[1] = (int)((cell / g.N) % g.N);
  c[2] = D == 3 ? (int)(cell / ((int64_t)g.N * g.N)) : 0;
}

// chi(x) of the multi-sinker field (reading: squared Gaussian).
template <int D>
__device__ inline double sinker_chi(const double* __restrict__ ctr, int ns, double omega, double delta,
                                    const double x[D]) {
  double out = 1.0;
  for (int i = 0; i < ns; ++i) {
    double s2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double dx = x[k] - ctr[i * D + k];
      s2 += dx * dx;
    }
    const double s = fmax(0.0, sqrt(s2) - 0.5 * omega);
    out *= (1.0 - exp(-delta * s * s));
  }
  return out;
}

// ---------------------------------------------------------------------------
template <int D>
__global__ void k_mu_sinker(LevelGeo g, const double* __restrict__ ctr, int ns, double omega,
                            double delta, double mu_min, double mu_max, double* __restrict__ mu) {
  constexpr int NQ = Dims<D>::NQ;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)NQ * g.ncell) return;
  const int64_t cell = idx / NQ;
  const int q = (int)(idx - cell * NQ);
  int c[3];
  cell_coords<D>(g, cell, c);
  double x[D];
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = g.h * ((double)c[k] + kGaussX[digit(q, k)]);
  const double chi = sinker_chi<D>(ctr, ns, omega, delta, x);
  mu[idx] = (mu_max - mu_min) * (1.0 - chi) + mu_min;
}

// ---------------------------------------------------------------------------
// Viscoplastic Newton tensor (Section 5.3.1; reading for the synthetic
// workload): mu0 = sinker field, eps = strain rate of the Fourier velocity
//   u_c = s sum_m amp[c][m] / (1 + |m|^2) prod_j sin(pi m_j x_j),  m in {1..M}^d,
// eps_II = (eps:eps/2)^(1/2), mu_eff = mu_floor + min(mu0 - mu_floor, tau_y/(2 eps_II)),
// C = 2 mu_eff I - w (x) w with w = (2 (mu_eff - mu_floor) [yielded])^(1/2) eps/|eps|_F.

// Gradient G[c][k] = d u_c / d x_k of the unscaled velocity (s = 1) at x,
// by partial sums over the tensor-product modes (x_{d-1} innermost).
template <int D>
__device__ inline void fourier_grad(const double* __restrict__ amp, int M, const double x[D], double G[D][D]) {
  constexpr double kPi = 3.141592653589793;
  double sn[3][8], cs[3][8];
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      double sv = 0.0, cv = 0.0;
      if (m < M) sincospi((double)(m + 1) * x[j], &sv, &cv);
      sn[j][m] = sv;
      cs[j][m] = kPi * (double)(m + 1) * cv;
    }
  for (int c = 0; c < D; ++c) {
    if constexpr (D == 3) {
      double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
      for (int m0 = 0; m0 < 8; ++m0) {
        if (m0 >= M) break;
        double qss = 0.0, qcs = 0.0, qsc = 0.0;
#pragma unroll
        for (int m1 = 0; m1 < 8; ++m1) {
          if (m1 >= M) break;
          double ps = 0.0, pc = 0.0;
          const double* a = amp + ((int64_t)(c * M + m0) * M + m1) * M;
#pragma unroll
          for (int m2 = 0; m2 < 8; ++m2) {
            if (m2 >= M) break;
            const double msq = (double)((m0 + 1) * (m0 + 1) + (m1 + 1) * (m1 + 1) + (m2 + 1) * (m2 + 1));
            const double av = a[m2] / (1.0 + msq);
            ps += av * sn[2][m2];
            pc += av * cs[2][m2];
          }
          qss += ps * sn[1][m1];
          qcs += ps * cs[1][m1];
          qsc += pc * sn[1][m1];
        }
        g0 += qss * cs[0][m0];
        g1 += qcs * sn[0][m0];
        g2 += qsc * sn[0][m0];
      }
      G[c][0] = g0;
      G[c][1] = g1;
      G[c][2] = g2;
    } else {
      double g0 = 0.0, g1 = 0.0;
#pragma unroll
      for (int m0 = 0; m0 < 8; ++m0) {
        if (m0 >= M) break;
        double ps = 0.0, pc = 0.0;
        const double* a = amp + (int64_t)(c * M + m0) * M;
#pragma unroll
        for (int m1 = 0; m1 < 8; ++m1) {
          if (m1 >= M) break;
          const double msq = (double)((m0 + 1) * (m0 + 1) + (m1 + 1) * (m1 + 1));
          const double av = a[m1] / (1.0 + msq);
          ps += av * sn[1][m1];
          pc += av * cs[1][m1];
        }
        g0 += ps * cs[0][m0];
        g1 += pc * sn[0][m0];
      }
      G[c][0] = g0;
      G[c][1] = g1;
    }
  }
}

template <int D>
__device__ inline void gauss_point(const LevelGeo& g, int64_t cell, int q, double x[D]) {
  int c[3];
  cell_coords<D>(g, cell, c);
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = g.h * ((double)c[k] + kGaussX[digit(q, k)]);
}

// The capped viscoplastic law at a physical strain rate e: returns
//   mu_eff = mu_f + min(mu0 - mu_f, tau_y / (2 eps_II)),  eps_II = (e:e/2)^(1/2),
// and sets w = (2 (mu_eff - mu_f) [yielded])^(1/2) e / |e|_F in symmetric
// storage, so that the derivative of tau(e) = 2 mu_eff(eps_II) e is
// C:x = 2 mu_eff x - (w:x) w (yielded: the cap below mu0 - mu_f; e = 0
// never yields).
template <int D>
__device__ inline double capped_law(const double (&e)[D][D], double mu0, double tau_y, double mu_f,
                                    double (&w)[SymIdx<D>::NS]) {
  double ee = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) ee += e[a][b] * e[a][b];
  const double eii = sqrt(0.5 * ee);
  const double cap = eii > 0.0 ? tau_y / (2.0 * eii) : INFINITY;
  const bool yielded = cap < mu0 - mu_f;
  const double meff = mu_f + fmin(mu0 - mu_f, cap);
  const double nrm = sqrt(ee);
  const double ws = (yielded && nrm > 0.0) ? sqrt(2.0 * (meff - mu_f)) / nrm : 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) w[SymIdx<D>::at(a, b)] = ws * e[a][b];
  return meff;
}

// The effective viscosity of the capped law alone (no tensor), for a
// strain rate given as a reference gradient G (physical: sym G / h).
template <int D, class R>
__device__ inline R capped_mu_ref(const R (&G)[D][D], R h, double mu0, double tau_y, double mu_f) {
  double ee = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double e = 0.5 * ((double)G[a][b] + (double)G[b][a]) / (double)h;
      ee += e * e;
    }
  const double eii = sqrt(0.5 * ee);
  const double cap = eii > 0.0 ? tau_y / (2.0 * eii) : INFINITY;
  return (R)(mu_f + fmin(mu0 - mu_f, cap));
}

// eps:eps of the unscaled strain rate (eps = sym G).
template <int D>
__device__ inline double strain_sq(const double G[D][D]) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double e = 0.5 * (G[a][b] + G[b][a]);
      s += e * e;
    }
  return s;
}

// part[b] = sum of eps_II^2 = eps:eps / 2 (s = 1) over block b's Gauss points
// of the finest level (fixed grid-stride partition).
template <int D>
__global__ void __launch_bounds__(kCoefThreads) k_eps_partials(LevelGeo g, const double* __restrict__ amp, int M,
                                                               double* __restrict__ part) {
  constexpr int NQ = Dims<D>::NQ;
  __shared__ double sh[kCoefThreads];
  double acc = 0.0;
  const int64_t n = (int64_t)NQ * g.ncell;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = i / NQ;
    double x[D], G[D][D];
    gauss_point<D>(g, cell, (int)(i - cell * NQ), x);
    fourier_grad<D>(amp, M, x, G);
    acc += 0.5 * strain_sq<D>(G);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// mu_eff and w at the Gauss points of one level. The velocity scale is
// `scale` if positive, else 1/sqrt(mean eps_II^2) from the fine-level
// partial sums (reduced identically by every block).
template <int D>
__global__ void __launch_bounds__(kCoefThreads)
k_coef_tensor(LevelGeo g, const double* __restrict__ ctr, int ns, double omega, double delta, double mu_min,
              double mu_max, double mu_floor, const double* __restrict__ amp, int M, double tau_y, double scale,
              const double* __restrict__ part, int nparts, int64_t nfine_pts, double* __restrict__ mu,
              double* __restrict__ cw) {
  constexpr int NQ = Dims<D>::NQ, NS = SymIdx<D>::NS;
  __shared__ double s_sh;
  if (threadIdx.x < 64) {
    double sc = scale;
    if (!(sc > 0.0)) {
      const double tot = wave_reduce_parts(part, nparts, 1, 0);
      sc = 1.0 / sqrt(tot / (double)nfine_pts);
    }
    if (threadIdx.x == 0) s_sh = sc;
  }
  __syncthreads();
  const double sc = s_sh;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)NQ * g.ncell) return;
  const int64_t cell = idx / NQ;
  const int q = (int)(idx - cell * NQ);
  double x[D], G[D][D];
  gauss_point<D>(g, cell, q, x);
  fourier_grad<D>(amp, M, x, G);
  double eps[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) eps[a][b] = 0.5 * sc * (G[a][b] + G[b][a]);
  const double mu0 = (mu_max - mu_min) * (1.0 - sinker_chi<D>(ctr, ns, omega, delta, x)) + mu_min;
  double wv[NS];
  mu[idx] = capped_law<D>(eps, mu0, tau_y, mu_floor, wv);
#pragma unroll
  for (int k = 0; k < NS; ++k) cw[(cell * NS + k) * NQ + q] = wv[k];
}

// mu_eff and w at the Gauss points of one level from an FE velocity u of
// that level (stored layout): eps(u) = sym grad u from the cell's 3^d nodal
// values, mu0 from the sinker field (the state of a Newton linearisation).
template <int D>
__global__ void __launch_bounds__(kCoefThreads)
k_coef_fe(LevelGeo g, const double* __restrict__ u, const double* __restrict__ ctr, int ns, double omega,
          double delta, double mu_min, double mu_max, double mu_floor, double tau_y, double* __restrict__ mu,
          double* __restrict__ cw) {
  constexpr int NQ = Dims<D>::NQ, NN = Dims<D>::NN, NS = SymIdx<D>::NS;
  constexpr const RefTab<D>& T = Ref<D>::T;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)NQ * g.ncell) return;
  const int64_t cell = idx / NQ;
  const int q = (int)(idx - cell * NQ);
  int c[3];
  cell_coords<D>(g, cell, c);
  double G[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) G[a][b] = 0.0;
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    const int a0 = 2 * c[0] + digit(n, 0), a1 = 2 * c[1] + digit(n, 1), a2 = D == 3 ? 2 * c[2] + digit(n, 2) : 0;
    bool bnd = a0 == 0 || a0 == 2 * g.N || a1 == 0 || a1 == 2 * g.N;
    if (D == 3) bnd = bnd || a2 == 0 || a2 == 2 * g.N;
    const int64_t nd = node_index<D>(g, a0, a1, a2);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double ua = bnd ? 0.0 : u[a * g.nnodes + nd];
#pragma unroll
      for (int b = 0; b < D; ++b) G[a][b] += ua * T.dphi[q][n][b];
    }
  }
  double eps[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) eps[a][b] = 0.5 * (G[a][b] + G[b][a]) / g.h;
  double x[D];
  gauss_point<D>(g, cell, q, x);
  const double mu0 = (mu_max - mu_min) * (1.0 - sinker_chi<D>(ctr, ns, omega, delta, x)) + mu_min;
  double wv[NS];
  mu[idx] = capped_law<D>(eps, mu0, tau_y, mu_floor, wv);
#pragma unroll
  for (int k = 0; k < NS; ++k) cw[(cell * NS + k) * NQ + q] = wv[k];
}

// Injection of a fine stored velocity to the next coarser level: coarse
// node i is fine node 2i (nested Q2 spaces); Dirichlet entries 0.
template <int D>
__global__ void k_inject(LevelGeo gf, LevelGeo gc, const double* __restrict__ uf, double* __restrict__ uc) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * gc.nnodes) return;
  const int comp = (int)(idx / gc.nnodes);
  const int64_t nd = idx - (int64_t)comp * gc.nnodes;
  int i[3];
  i[0] = (int)(nd % gc.n1);
  i[1] = (int)((nd / gc.n1) % gc.n1);
  i[2] = D == 3 ? (int)(nd / ((int64_t)gc.n1 * gc.n1)) : 0;
  bool bnd = false;
#pragma unroll
  for (int k = 0; k < D; ++k) bnd = bnd || i[k] == 0 || i[k] == 2 * gc.N;
  uc[idx] = bnd ? 0.0 : uf[comp * gf.nnodes + node_index<D>(gf, 2 * i[0], 2 * i[1], 2 * i[2])];
}

// ---------------------------------------------------------------------------
// Cell kernel. A wavefront handles CPW = floor(64 / 3^d) cells (7 in 2D, 2 in
// 3D) with one lane per (cell, Gauss point) in the first phase and one lane
// per (cell, node) in the second; the cell's velocity and the weighted stress
// at the Gauss points are exchanged through LDS.
//   phase 1 (lane = Gauss point q): reference gradient G of u at q by sum
//     factorisation over the tensor axes; S_q = w_q mu_q (G + G^T) plus the
//     pressure-like diagonal w_q pi_q, pi_q = sum_m c_m psi_m(q) with
//     c = gamma Mhat^{-1} Bhat u - h p (the divergence moments Bhat u are
//     summed over the cell's lanes in a fixed order).
//   phase 2 (lane = node n): y_n = h^{d-2} sum_q S_q : dphi_n(q), again
//     sum-factorised; element vectors E[cell][comp * 3^d + n].
// All table entries are exact compile-time values selected by the lane's
// digits; no atomics.
constexpr double kB1[3][3] = {{lag(0, kGaussX[0]), lag(1, kGaussX[0]), lag(2, kGaussX[0])},
                              {lag(0, kGaussX[1]), lag(1, kGaussX[1]), lag(2, kGaussX[1])},
                              {lag(0, kGaussX[2]), lag(1, kGaussX[2]), lag(2, kGaussX[2])}};
constexpr double kD1[3][3] = {{dlag(0, kGaussX[0]), dlag(1, kGaussX[0]), dlag(2, kGaussX[0])},
                              {dlag(0, kGaussX[1]), dlag(1, kGaussX[1]), dlag(2, kGaussX[1])},
                              {dlag(0, kGaussX[2]), dlag(1, kGaussX[2]), dlag(2, kGaussX[2])}};

// tab[r][c] with a runtime row r in 0..2 (selects between compile-time constants)
__device__ inline double sel3(const double (&tab)[3][3], int r, int c) {
  return r == 0 ? tab[0][c] : (r == 1 ? tab[1][c] : tab[2][c]);
}
// tab[r][c] with a runtime column c
__device__ inline double selc(const double (&tab)[3][3], int r, int c) {
  return c == 0 ? tab[r][0] : (c == 1 ? tab[r][1] : tab[r][2]);
}

//
// With ZS the input is not a node vector but the smoother's patch-output
// buffer (u = zbuf, nvert vertices): each lane forms its node's value as the
// sum of the patch outputs there, exactly as the separate gather does, and
// the one cell that owns the node (the lowest cell containing it on every
// axis) also stores that value to zout, so the smoother's search direction
// is written once without a kernel of its own.
template <int D, int MODE, bool TENSOR, class R, bool ZS = false>
__global__ void __launch_bounds__(64)
k_elem(LevelGeo g, const R* __restrict__ mu, const R* __restrict__ cw, const R* __restrict__ winv, double gamma_d,
       const R* __restrict__ u, const double* __restrict__ p, R* __restrict__ E, double* __restrict__ pout,
       int nvert = 0, R* __restrict__ zout = nullptr, double nl_tau = 0.0, double nl_floor = 0.0) {
  constexpr int NN = Dims<D>::NN, NQ = NN, NL = Dims<D>::NL, NP = Dims<D>::NP;
  constexpr int NS = SymIdx<D>::NS;
  constexpr int CPW = 64 / NQ;
  constexpr bool need_u = (MODE & (EL_VISC | EL_AUG | EL_BOUT)) != 0;
  constexpr bool need_c = (MODE & (EL_AUG | EL_BT | EL_BOUT)) != 0;
  __shared__ R us[CPW][D][NN];
  __shared__ R ss[CPW][NQ][NS];
  __shared__ R red[CPW][NQ][NP];
  __shared__ R cms[CPW][NP];
  const R gamma = (R)gamma_d;
  const int lane = threadIdx.x;
  const int lc = lane / NQ;
  const int t = lane - lc * NQ;
  const int64_t cell = (int64_t)blockIdx.x * CPW + lc;
  const bool valid = lc < CPW && cell < g.ncell;
  const int t0 = t % 3, t1 = (t / 3) % 3, t2 = D == 3 ? t / 9 : 0;
  int c[3] = {0, 0, 0};
  if (valid) {
    c[0] = (int)(cell % g.N);
    c[1] = (int)((cell / g.N) % g.N);
    c[2] = D == 3 ? (int)(cell / ((int64_t)g.N * g.N)) : 0;
  }
  const R h = (R)g.h;
  // coefficients at this lane's Gauss point, loaded ahead of the velocity
  // (they do not depend on it) so the two sets of loads overlap
  R muq = 0;
  R wv[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) wv[k] = 0;
  if ((MODE & EL_VISC) && valid) {
    muq = mu[cell * NQ + t];
    if constexpr (TENSOR) {
#pragma unroll
      for (int k = 0; k < NS; ++k) wv[k] = cw[(cell * NS + k) * NQ + t];
    }
  }
  // ---- stage u: lane t loads node t of its cell (Dirichlet nodes masked)
  if (need_u && valid) {
    const int a0 = 2 * c[0] + t0, a1 = 2 * c[1] + t1, a2 = D == 3 ? 2 * c[2] + t2 : 0;
    bool bnd = a0 == 0 || a0 == 2 * g.N || a1 == 0 || a1 == 2 * g.N;
    if (D == 3) bnd = bnd || a2 == 0 || a2 == 2 * g.N;
    const int64_t nd = node_index<D>(g, a0, a1, a2);
    if constexpr (ZS) {
      const int ai[3] = {a0, a1, a2};
      bool own = (t0 < 2 || c[0] == g.N - 1) && (t1 < 2 || c[1] == g.N - 1);
      if (D == 3) own = own && (t2 < 2 || c[2] == g.N - 1);
#pragma unroll
      for (int comp = 0; comp < D; ++comp) {
        const R v = bnd ? (R)0 : asm_node_sum<D, R>(g, u, nvert, comp, ai);
        us[lc][comp][t] = v;
        if (own) zout[comp * g.nnodes + nd] = v;
      }
    } else {
#pragma unroll
      for (int comp = 0; comp < D; ++comp) {
        const R v = u[comp * g.nnodes + nd];
        us[lc][comp][t] = bnd ? (R)0 : v;
      }
    }
  }
  __syncthreads();
  // ---- phase 1: lane = Gauss point q = (t0, t1, t2)
  constexpr const RefTab<D>& T = Ref<D>::T;
  R S[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) S[i] = (R)0;
  const R wq = (R)(kGaussW[t0] * kGaussW[t1] * (D == 3 ? kGaussW[t2] : 1.0));
  if (valid && need_u) {
    R Bx[3], Dx[3], By[3], Dy[3], Bz[3], Dz[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Bx[a] = (R)sel3(kB1, t0, a); Dx[a] = (R)sel3(kD1, t0, a);
      By[a] = (R)sel3(kB1, t1, a); Dy[a] = (R)sel3(kD1, t1, a);
      Bz[a] = (R)sel3(kB1, t2, a); Dz[a] = (R)sel3(kD1, t2, a);
    }
    R G[D][D];
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
      if constexpr (D == 3) {
        R zB[3][3], zD[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const R u0 = us[lc][comp][a + 3 * b], u1 = us[lc][comp][a + 3 * b + 9],
                    u2 = us[lc][comp][a + 3 * b + 18];
            zB[a][b] = u0 * Bz[0] + u1 * Bz[1] + u2 * Bz[2];
            zD[a][b] = u0 * Dz[0] + u1 * Dz[1] + u2 * Dz[2];
          }
        R g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const R yBB = zB[a][0] * By[0] + zB[a][1] * By[1] + zB[a][2] * By[2];
          const R yDB = zB[a][0] * Dy[0] + zB[a][1] * Dy[1] + zB[a][2] * Dy[2];
          const R yBD = zD[a][0] * By[0] + zD[a][1] * By[1] + zD[a][2] * By[2];
          g0 += yBB * Dx[a];
          g1 += yDB * Bx[a];
          g2 += yBD * Bx[a];
        }
        G[comp][0] = g0; G[comp][1] = g1; G[comp][2] = g2;
      } else {
        R g0 = 0, g1 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const R u0 = us[lc][comp][a], u1 = us[lc][comp][a + 3], u2 = us[lc][comp][a + 6];
          const R yB = u0 * By[0] + u1 * By[1] + u2 * By[2];
          const R yD = u0 * Dy[0] + u1 * Dy[1] + u2 * Dy[2];
          g0 += yB * Dx[a];
          g1 += yD * Bx[a];
        }
        G[comp][0] = g0; G[comp][1] = g1;
      }
    }
    if (MODE & EL_VISC) {
      if constexpr ((MODE & EL_NL) != 0) muq = capped_mu_ref<D, R>(G, h, (double)muq, nl_tau, nl_floor);
      const R wm = wq * muq;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) S[SymIdx<D>::at(a, b)] = wm * (G[a][b] + G[b][a]);
      if constexpr (TENSOR) {
        // C:eps = 2 mu eps - (w:eps) w, and w:eps = w:G for symmetric w
        R wg = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          wg += wv[a] * G[a][a];
#pragma unroll
          for (int b = a + 1; b < D; ++b) wg += wv[SymIdx<D>::at(a, b)] * (G[a][b] + G[b][a]);
        }
        const R f = wq * wg;
#pragma unroll
        for (int k = 0; k < NS; ++k) S[k] -= f * wv[k];
      }
    }
    if (MODE & (EL_AUG | EL_BOUT)) {
      R dv = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) dv += G[a][a];
      red[lc][t][0] = wq * dv;
#pragma unroll
      for (int m = 1; m < NP; ++m) red[lc][t][m] = wq * (R)(kGaussX[m == 1 ? t0 : (m == 2 ? t1 : t2)] - 0.5) * dv;
    }
  }
  if constexpr (need_c) {
    __syncthreads();
    if (valid && t == 0) {
      R bu[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        bu[m] = 0;
        if (MODE & (EL_AUG | EL_BOUT))
          for (int q = 0; q < NQ; ++q) bu[m] += red[lc][q][m];
      }
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        R cm = 0;
        if (MODE & EL_AUG) {
          if (winv) {   // W = M_p(1/mu): the cell's inverse weighted mass
            R t2 = 0;
#pragma unroll
            for (int k = 0; k < NP; ++k) t2 += winv[cell * NP * NP + m * NP + k] * bu[k];
            cm += gamma * t2;
          } else {
            cm += gamma * bu[m] * (R)kInvMhat[m];
          }
        }
        if (MODE & EL_BOUT) pout[cell * NP + m] = -(D == 2 ? g.h : g.h * g.h) * (double)bu[m];
        if (MODE & EL_BT) cm -= h * (R)p[cell * NP + m];
        cms[lc][m] = cm;
      }
    }
    __syncthreads();
    if (valid && (MODE & (EL_AUG | EL_BT))) {
      R pi = cms[lc][0];
      pi += cms[lc][1] * (R)(kGaussX[t0] - 0.5);
      pi += cms[lc][2] * (R)(kGaussX[t1] - 0.5);
      if (D == 3) pi += cms[lc][3] * (R)(kGaussX[t2] - 0.5);
#pragma unroll
      for (int a = 0; a < D; ++a) S[a] += wq * pi;
    }
  }
  if (valid) {
#pragma unroll
    for (int i = 0; i < NS; ++i) ss[lc][t][i] = S[i];
  }
  __syncthreads();
  // ---- phase 2: lane = node n = (t0, t1, t2); y_n = sum_q S_q : dphi_n(q)
  if (!valid) return;
  R nBx[3], nDx[3], nBy[3], nDy[3], nBz[3], nDz[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    nBx[q] = (R)selc(kB1, q, t0); nDx[q] = (R)selc(kD1, q, t0);
    nBy[q] = (R)selc(kB1, q, t1); nDy[q] = (R)selc(kD1, q, t1);
    nBz[q] = (R)selc(kB1, q, t2); nDz[q] = (R)selc(kD1, q, t2);
  }
  const R sc = D == 2 ? (R)1 : h;   // h^{d-2}
#pragma unroll
  for (int comp = 0; comp < D; ++comp) {
    R ycomp = 0;
#pragma unroll
    for (int qz = 0; qz < (D == 3 ? 3 : 1); ++qz) {
      R Y[3] = {0, 0, 0};
#pragma unroll
      for (int qy = 0; qy < 3; ++qy) {
        R X[3] = {0, 0, 0};
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
          const int q = qx + 3 * qy + 9 * qz;
          X[0] += ss[lc][q][SymIdx<D>::at(comp, 0)] * nDx[qx];
          X[1] += ss[lc][q][SymIdx<D>::at(comp, 1)] * nBx[qx];
          if (D == 3) X[2] += ss[lc][q][SymIdx<D>::at(comp, D == 3 ? 2 : 0)] * nBx[qx];
        }
        Y[0] += X[0] * nBy[qy];
        Y[1] += X[1] * nDy[qy];
        if (D == 3) Y[2] += X[2] * nBy[qy];
      }
      if (D == 3) ycomp += Y[0] * nBz[qz] + Y[1] * nBz[qz] + Y[2] * nDz[qz];
      else ycomp += Y[0] + Y[1];
    }
    E[cell * NL + comp * NN + t] = sc * ycomp;
  }
  (void)T;
}

// ---------------------------------------------------------------------------
// 3D cell kernel with the tensor-product contractions shared across lanes.
// A wavefront handles 7 cells with 9 lanes each (lane 63 idle); in every
// stage a lane owns one pencil of 3 points along the axis being contracted,
// so each 1D contraction is done once per cell instead of once per Gauss
// point. Stages exchange their pencils through LDS:
//   gradient:   x (lane = (y,z)) -> y (lane = (qx,z)) -> z (lane = (qx,qy)),
//               leaving lane (qx,qy) with G at its 3 points (qx,qy,0..2);
//   pointwise:  S_q = w_q mu_q (G + G^T) [- w_q (w:G) w] + w_q pi_q I, the
//               divergence moments summed over the cell's 9 lanes in a fixed
//               order (every lane of the cell forms the same sum);
//   transpose:  z (lane = (qx,qy)) -> y (lane = (qx,nz)) -> x (lane = (ny,nz)),
//               leaving lane (ny,nz) with y at nodes (0..2,ny,nz).
// About 1,900 FMAs per cell each way, instead of 7,300 when every Gauss point
// forms its own gradient. Same outputs as k_elem up to rounding order.
constexpr int kE3Cells = 7;

// [cell slot][27]: slot 7 belongs to the idle lane 63. The divergence
// moments share storage with the x-stage pencils (neither is live while the
// other is).
template <class R>
struct E3Smem {
  union {
    R x[kE3Cells + 1][2][27];
    R red[kE3Cells + 1][9][4];
  };
  R y[kE3Cells + 1][3][27];
};

__device__ constexpr int i3(int a, int b, int c) { return a + 3 * b + 9 * c; }

template <int MODE, bool TENSOR, class R>
__global__ void __launch_bounds__(64)
k_elem3(LevelGeo g, const R* __restrict__ mu, const R* __restrict__ cw, const R* __restrict__ winv, double gamma_d,
        const R* __restrict__ u, const double* __restrict__ p, R* __restrict__ E, double* __restrict__ pout,
        double nl_tau = 0.0, double nl_floor = 0.0) {
  constexpr int NQ = 27, NL = 81, NP = 4, NS = 6;
  constexpr bool need_u = (MODE & (EL_VISC | EL_AUG | EL_BOUT)) != 0;
  constexpr bool need_c = (MODE & (EL_AUG | EL_BT | EL_BOUT)) != 0;
  // without the viscous term the stress is diagonal (pi I): the forward
  // stages need only the divergence, d_c u_c, and the transposed stages only
  // the diagonal entries, so each component runs one contraction chain
  // (the same arithmetic as the full chains on the entries that are used)
  constexpr bool DIAG = (MODE & EL_VISC) == 0;
  __shared__ E3Smem<R> sm;
  const R gamma = (R)gamma_d;
  const int lane = threadIdx.x;
  const int lc = lane / 9;                 // cell slot 0..7 (7 = idle lane)
  const int pa = lane - 9 * lc;            // pencil: (pa % 3, pa / 3)
  const int p0 = pa % 3, p1 = pa / 3;
  const int64_t cell = (int64_t)blockIdx.x * kE3Cells + lc;
  const bool valid = lc < kE3Cells && cell < g.ncell;
  int c[3] = {0, 0, 0};
  if (valid) {
    c[0] = (int)(cell % g.N);
    c[1] = (int)((cell / g.N) % g.N);
    c[2] = (int)(cell / ((int64_t)g.N * g.N));
  }
  // ---- lane (y,z) = (p0,p1) loads the x-pencil of each component; the x
  // stage below contracts exactly this pencil, so it stays in registers
  R upen[3][3] = {};   // [comp][x]
  if (need_u) {
    const int a1 = 2 * c[1] + p0, a2 = 2 * c[2] + p1;
    const bool bnd12 = a1 == 0 || a1 == 2 * g.N || a2 == 0 || a2 == 2 * g.N;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int a0 = 2 * c[0] + a;
      const bool bnd = bnd12 || a0 == 0 || a0 == 2 * g.N;
      const int64_t nd = node_index<3>(g, a0, a1, a2);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp)
        if (valid && !bnd) upen[comp][a] = u[comp * g.nnodes + nd];
    }
  }
  // ---- gradient at the lane's Gauss points (qx,qy) = (p0,p1), qz = 0..2
  R G[3][3][3];   // [qz][comp][k]
#pragma unroll
  for (int qz = 0; qz < 3; ++qz)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[qz][a][b] = (R)0;
  if (need_u) {
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      // x: lane (y,z) = (p0,p1)
      {
        const R u0 = upen[comp][0], u1 = upen[comp][1], u2 = upen[comp][2];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (!DIAG || comp != 0)
            sm.x[lc][0][i3(q, p0, p1)] = u0 * (R)kB1[q][0] + u1 * (R)kB1[q][1] + u2 * (R)kB1[q][2];
          if (!DIAG || comp == 0)
            sm.x[lc][1][i3(q, p0, p1)] = u0 * (R)kD1[q][0] + u1 * (R)kD1[q][1] + u2 * (R)kD1[q][2];
        }
      }
      __syncthreads();
      // y: lane (qx,z) = (p0,p1); outputs B_y B_x u, D_y B_x u, B_y D_x u
      {
        R xb[3] = {}, xd[3] = {};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (!DIAG || comp != 0) xb[b] = sm.x[lc][0][i3(p0, b, p1)];
          if (!DIAG || comp == 0) xd[b] = sm.x[lc][1][i3(p0, b, p1)];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (!DIAG || comp == 2)
            sm.y[lc][0][i3(p0, q, p1)] = xb[0] * (R)kB1[q][0] + xb[1] * (R)kB1[q][1] + xb[2] * (R)kB1[q][2];
          if (!DIAG || comp == 1)
            sm.y[lc][1][i3(p0, q, p1)] = xb[0] * (R)kD1[q][0] + xb[1] * (R)kD1[q][1] + xb[2] * (R)kD1[q][2];
          if (!DIAG || comp == 0)
            sm.y[lc][2][i3(p0, q, p1)] = xd[0] * (R)kB1[q][0] + xd[1] * (R)kB1[q][1] + xd[2] * (R)kB1[q][2];
        }
      }
      __syncthreads();
      // z: lane (qx,qy) = (p0,p1)
      {
        R ybb[3] = {}, ybd[3] = {}, ydb[3] = {};
#pragma unroll
        for (int z = 0; z < 3; ++z) {
          if (!DIAG || comp == 2) ybb[z] = sm.y[lc][0][i3(p0, p1, z)];
          if (!DIAG || comp == 1) ybd[z] = sm.y[lc][1][i3(p0, p1, z)];
          if (!DIAG || comp == 0) ydb[z] = sm.y[lc][2][i3(p0, p1, z)];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (!DIAG || comp == 0)
            G[q][comp][0] = ydb[0] * (R)kB1[q][0] + ydb[1] * (R)kB1[q][1] + ydb[2] * (R)kB1[q][2];
          if (!DIAG || comp == 1)
            G[q][comp][1] = ybd[0] * (R)kB1[q][0] + ybd[1] * (R)kB1[q][1] + ybd[2] * (R)kB1[q][2];
          if (!DIAG || comp == 2)
            G[q][comp][2] = ybb[0] * (R)kD1[q][0] + ybb[1] * (R)kD1[q][1] + ybb[2] * (R)kD1[q][2];
        }
      }
      // the next component's x stage overwrites sm.x only after this
      // component's y stage has read it (barrier above); its y stage
      // overwrites sm.y after the barrier that follows its x stage
    }
  }
  // ---- pointwise stress at (p0, p1, qz)
  auto sel = [](int i, double a, double b, double c) { return (R)(i == 0 ? a : (i == 1 ? b : c)); };
  const R wxy = sel(p0, kGaussW[0], kGaussW[1], kGaussW[2]) * sel(p1, kGaussW[0], kGaussW[1], kGaussW[2]);
  const R gx = sel(p0, kGaussX[0] - 0.5, kGaussX[1] - 0.5, kGaussX[2] - 0.5);
  const R gy = sel(p1, kGaussX[0] - 0.5, kGaussX[1] - 0.5, kGaussX[2] - 0.5);
  R S[3][NS];
#pragma unroll
  for (int qz = 0; qz < 3; ++qz) {
    const R wq = wxy * (R)kGaussW[qz];
    const int q = i3(p0, p1, qz);
#pragma unroll
    for (int k = 0; k < NS; ++k) S[qz][k] = (R)0;
    if ((MODE & EL_VISC) && valid) {
      R muq = mu[cell * NQ + q];
      if constexpr ((MODE & EL_NL) != 0) muq = capped_mu_ref<3, R>(G[qz], (R)g.h, (double)muq, nl_tau, nl_floor);
      const R wm = wq * muq;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) S[qz][SymIdx<3>::at(a, b)] = wm * (G[qz][a][b] + G[qz][b][a]);
      if constexpr (TENSOR) {
        R wv[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) wv[k] = cw[(cell * NS + k) * NQ + q];
        R wg = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          wg += wv[a] * G[qz][a][a];
#pragma unroll
          for (int b = a + 1; b < 3; ++b) wg += wv[SymIdx<3>::at(a, b)] * (G[qz][a][b] + G[qz][b][a]);
        }
        const R f = wq * wg;
#pragma unroll
        for (int k = 0; k < NS; ++k) S[qz][k] -= f * wv[k];
      }
    }
  }
  if constexpr (need_c) {
    if (MODE & (EL_AUG | EL_BOUT)) {
      R part[NP] = {0, 0, 0, 0};
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) {
        const R wd = wxy * (R)kGaussW[qz] * (G[qz][0][0] + G[qz][1][1] + G[qz][2][2]);
        part[0] += wd;
        part[1] += wd * gx;
        part[2] += wd * gy;
        part[3] += wd * (R)(kGaussX[qz] - 0.5);
      }
#pragma unroll
      for (int m = 0; m < NP; ++m) sm.red[lc][pa][m] = part[m];
    }
    __syncthreads();
    R bu[NP] = {0, 0, 0, 0};
    if (MODE & (EL_AUG | EL_BOUT)) {
#pragma unroll
      for (int m = 0; m < NP; ++m)
#pragma unroll
        for (int k = 0; k < 9; ++k) bu[m] += sm.red[lc][k][m];
    }
    R cm[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      cm[m] = 0;
      if (MODE & EL_AUG) {
        if (winv) {   // W = M_p(1/mu): the cell's inverse weighted mass
          R t2 = 0;
          if (valid) {
#pragma unroll
            for (int k = 0; k < NP; ++k) t2 += winv[cell * NP * NP + m * NP + k] * bu[k];
          }
          cm[m] += gamma * t2;
        } else {
          cm[m] += gamma * bu[m] * (R)kInvMhat[m];
        }
      }
      if ((MODE & EL_BOUT) && valid && pa == 0) pout[cell * NP + m] = -(g.h * g.h) * (double)bu[m];
      if ((MODE & EL_BT) && valid) cm[m] -= (R)g.h * (R)p[cell * NP + m];
    }
    if (MODE & (EL_AUG | EL_BT)) {
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) {
        const R wq = wxy * (R)kGaussW[qz];
        const R pi = cm[0] + cm[1] * gx + cm[2] * gy + cm[3] * (R)(kGaussX[qz] - 0.5);
#pragma unroll
        for (int a = 0; a < 3; ++a) S[qz][a] += wq * pi;
      }
    }
  }
  if constexpr (!need_c) __syncthreads();   // the z stages below overwrite sm.y
  // ---- transpose contractions, one component at a time
  const R h = (R)g.h;   // h^{d-2}
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    // z: lane (qx,qy) = (p0,p1) -> (qx,qy,nz)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      R t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (!DIAG || comp == 0) t0 += S[q][SymIdx<3>::at(comp, 0)] * (R)kB1[q][n];
        if (!DIAG || comp == 1) t1 += S[q][SymIdx<3>::at(comp, 1)] * (R)kB1[q][n];
        if (!DIAG || comp == 2) t2 += S[q][SymIdx<3>::at(comp, 2)] * (R)kD1[q][n];
      }
      if (!DIAG || comp == 0) sm.y[lc][0][i3(p0, p1, n)] = t0;
      if (!DIAG || comp == 1) sm.y[lc][1][i3(p0, p1, n)] = t1;
      if (!DIAG || comp == 2) sm.y[lc][2][i3(p0, p1, n)] = t2;
    }
    __syncthreads();
    // y: lane (qx,nz) = (p0,p1) -> (qx,ny,nz); outputs D_x-bound and B_x-bound parts
    {
      R t0[3] = {}, t1[3] = {}, t2[3] = {};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (!DIAG || comp == 0) t0[q] = sm.y[lc][0][i3(p0, q, p1)];
        if (!DIAG || comp == 1) t1[q] = sm.y[lc][1][i3(p0, q, p1)];
        if (!DIAG || comp == 2) t2[q] = sm.y[lc][2][i3(p0, q, p1)];
      }
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        R w0 = 0, w12 = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (!DIAG) {
            w0 += t0[q] * (R)kB1[q][n];
            w12 += t1[q] * (R)kD1[q][n] + t2[q] * (R)kB1[q][n];
          } else if (comp == 0) {
            w0 += t0[q] * (R)kB1[q][n];
          } else if (comp == 1) {
            w12 += t1[q] * (R)kD1[q][n];
          } else {
            w12 += t2[q] * (R)kB1[q][n];
          }
        }
        if (!DIAG || comp == 0) sm.x[lc][0][i3(p0, n, p1)] = w0;
        if (!DIAG || comp != 0) sm.x[lc][1][i3(p0, n, p1)] = w12;
      }
    }
    __syncthreads();
    // x: lane (ny,nz) = (p0,p1) -> nodes (0..2, ny, nz)
    {
      R w0[3] = {}, w12[3] = {};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (!DIAG || comp == 0) w0[q] = sm.x[lc][0][i3(q, p0, p1)];
        if (!DIAG || comp != 0) w12[q] = sm.x[lc][1][i3(q, p0, p1)];
      }
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        R yv = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (!DIAG) yv += w0[q] * (R)kD1[q][n] + w12[q] * (R)kB1[q][n];
          else if (comp == 0) yv += w0[q] * (R)kD1[q][n];
          else yv += w12[q] * (R)kB1[q][n];
        }
        if (valid) E[cell * NL + comp * 27 + i3(n, p0, p1)] = h * yv;
      }
    }
    // the next component's z stage overwrites sm.y after this component's
    // y stage read it (barrier above) and sm.x after this x stage (the
    // barrier that follows the next z stage)
  }
}

// ---------------------------------------------------------------------------
// Sum of the element outputs of the <= 2^d cells containing stored entry idx
// (fixed order); 0 on Dirichlet nodes (flag set).
template <int D, class R>
__device__ inline R gather_sum(const LevelGeo& g, const R* __restrict__ E, int64_t idx, bool& dirichlet) {
  constexpr int NN = Dims<D>::NN;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  int i[3];
  i[0] = (int)(nd % g.n1);
  i[1] = (int)((nd / g.n1) % g.n1);
  i[2] = D == 3 ? (int)(nd / ((int64_t)g.n1 * g.n1)) : 0;
  bool bnd = false;
#pragma unroll
  for (int k = 0; k < D; ++k) bnd = bnd || i[k] == 0 || i[k] == 2 * g.N;
  dirichlet = bnd;
  if (bnd) return (R)0;
  // per axis up to two (cell, local) pairs; an absent second pair repeats
  // the first so that every address below is valid
  int cc[3][2], ll[3][2], cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) {
      cnt[k] = 1; cc[k][0] = cc[k][1] = 0; ll[k][0] = ll[k][1] = 0;
      continue;
    }
    if (i[k] & 1) {
      cnt[k] = 1; cc[k][0] = cc[k][1] = (i[k] - 1) >> 1; ll[k][0] = ll[k][1] = 1;
    } else {
      cnt[k] = 2; cc[k][0] = (i[k] >> 1) - 1; ll[k][0] = 2; cc[k][1] = i[k] >> 1; ll[k][1] = 0;
    }
  }
  // all (up to 2^d) loads issued together, then summed in the fixed order
  constexpr int NT = D == 3 ? 8 : 4;
  R v[NT];
  bool ok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int t0 = t & 1, t1 = (t >> 1) & 1, t2 = t >> 2;
    ok[t] = t0 < cnt[0] && t1 < cnt[1] && t2 < cnt[2];
    const int64_t cell = cell_index<D>(g, cc[0][t0], cc[1][t1], cc[2][t2]);
    const int loc = ll[0][t0] + 3 * ll[1][t1] + 9 * ll[2][t2];
    v[t] = ok[t] ? E[cell * (D * NN) + comp * NN + loc] : (R)0;
  }
  R s = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (ok[t]) s += v[t];
  return s;
}

// out[idx] = base[idx] + alpha * sum_{cells K containing node} E_K[local],
// 0 on Dirichlet nodes. One thread per stored entry.
template <int D, class R>
__global__ void k_gather(LevelGeo g, const R* __restrict__ E, const R* __restrict__ base,
                         double alpha_d, R* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * g.nnodes) return;
  bool dir;
  const R s = gather_sum<D, R>(g, E, idx, dir);
  out[idx] = dir ? (R)0 : (base ? base[idx] : (R)0) + (R)alpha_d * s;
}

// The gather of y = A u fused with the dot products V_k . y (k < nk) over the
// whole vector of length nvec >= d*nnodes (entries past the velocity block,
// e.g. a pressure block already written, are read as they are). Block
// partials part[b*nk + k] on the fixed grid-stride partition of red_parts(nvec).
template <int D, class R>
__global__ void __launch_bounds__(kRedThreads)
k_gather_dots(LevelGeo g, const R* __restrict__ E, R* __restrict__ out, int64_t nvec, const R* __restrict__ V,
              int64_t ldv, int nk, double* __restrict__ part) {
  __shared__ double sh[8 * (kRedThreads / 64)];
  const int64_t nvel = (int64_t)D * g.nnodes;
  for (int k0 = 0; k0 < nk; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvec;
         i += (int64_t)gridDim.x * blockDim.x) {
      // the V entries do not depend on the gather: their loads go first so
      // that both sets are in flight together
      double vk[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) vk[kk] = k0 + kk < nk ? (double)V[(int64_t)(k0 + kk) * ldv + i] : 0.0;
      R wi;
      if (i < nvel) {
        if (k0 == 0) {
          bool dir;
          wi = gather_sum<D, R>(g, E, i, dir);
          out[i] = wi;
        } else {
          wi = out[i];   // written by this thread in the first chunk
        }
      } else {
        wi = out[i];
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < nk) acc[kk] += vk[kk] * (double)wi;
    }
    double tot[8];
    block_sum_n<8>(acc, nk - k0, sh, tot);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < nk) part[blockIdx.x * nk + k0 + kk] = tot[kk];
    }
  }
}

// ---------------------------------------------------------------------------
// Element right-hand side (f, phi) with f = (0, .., beta (chi - 1)).
template <int D>
__global__ void k_rhs_elem(LevelGeo g, const double* __restrict__ ctr, int ns, double omega,
                           double delta, double beta, double* __restrict__ E) {
  constexpr int NN = Dims<D>::NN;
  constexpr const RefTab<D>& T = Ref<D>::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  int c[3];
  cell_coords<D>(g, cell, c);
  double be[NN];
#pragma unroll
  for (int n = 0; n < NN; ++n) be[n] = 0.0;
  for (int q = 0; q < NN; ++q) {
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = g.h * ((double)c[k] + kGaussX[digit(q, k)]);
    const double f = beta * (sinker_chi<D>(ctr, ns, omega, delta, x) - 1.0);
#pragma unroll
    for (int n = 0; n < NN; ++n) be[n] += T.w[q] * T.phi[q][n] * f;
  }
  const double vol = D == 2 ? g.h * g.h : g.h * g.h * g.h;
  for (int comp = 0; comp < D - 1; ++comp)
    for (int n = 0; n < NN; ++n) E[cell * (D * NN) + comp * NN + n] = 0.0;
#pragma unroll
  for (int n = 0; n < NN; ++n) E[cell * (D * NN) + (D - 1) * NN + n] = vol * be[n];
}

// [Q3]^2 x P2disc: the sinker viscosity at a cell's 4 x 4 Gauss points, and
// the element loads (f, phi) of the cubic basis with the same forcing.
__global__ void k3_mu_sinker(LevelGeo g, const double* __restrict__ ctr, int ns, double omega, double delta,
                             double mu_min, double mu_max, double* __restrict__ mu) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)q3::NQ * g.ncell) return;
  const int64_t cell = idx / q3::NQ;
  const int q = (int)(idx - cell * q3::NQ);
  const double x[2] = {g.h * ((double)(cell % g.N) + q3::kGx[q % q3::NA]),
                       g.h * ((double)(cell / g.N) + q3::kGx[q / q3::NA])};
  const double chi = sinker_chi<2>(ctr, ns, omega, delta, x);
  mu[idx] = (mu_max - mu_min) * (1.0 - chi) + mu_min;
}

__global__ void k3_rhs_elem(LevelGeo g, const double* __restrict__ ctr, int ns, double omega, double delta,
                            double beta, double* __restrict__ E) {
  constexpr const q3::Tab& T = q3::RefQ3::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double be[q3::NN];
#pragma unroll
  for (int n = 0; n < q3::NN; ++n) be[n] = 0.0;
  for (int q = 0; q < q3::NQ; ++q) {
    const double x[2] = {g.h * ((double)(cell % g.N) + q3::kGx[q % q3::NA]),
                         g.h * ((double)(cell / g.N) + q3::kGx[q / q3::NA])};
    const double f = beta * (sinker_chi<2>(ctr, ns, omega, delta, x) - 1.0);
#pragma unroll
    for (int n = 0; n < q3::NN; ++n) be[n] += T.w[q] * T.phi[q][n] * f;
  }
  const double vol = g.h * g.h;
#pragma unroll
  for (int n = 0; n < q3::NN; ++n) {
    E[cell * q3::NL + n] = 0.0;
    E[cell * q3::NL + q3::NN + n] = vol * be[n];
  }
}

// ---------------------------------------------------------------------------
// Per cell: Winv = (sum_q w_q / mu_q psi psi^T)^{-1} on the reference cell,
// the inverse weighted pressure mass of W = M_p(1/mu) (eq. (P1P2), P2) without
// the cell volume (M_K(1/mu) = h^d times this matrix).
template <int D>
__global__ void k_winv_setup(LevelGeo g, const double* __restrict__ mu, double* __restrict__ winv) {
  constexpr int NN = Dims<D>::NN, NP = Dims<D>::NP;
  constexpr const RefTab<D>& T = Ref<D>::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  double M[NP][NP], X[NP][NP];
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      M[a][b] = 0.0;
      X[a][b] = a == b ? 1.0 : 0.0;
    }
  for (int q = 0; q < NN; ++q) {
    const double wq = T.w[q] / mu[cell * NN + q];
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
      for (int b = 0; b < NP; ++b) M[a][b] += wq * T.psi[q][a] * T.psi[q][b];
  }
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
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) winv[cell * NP * NP + a * NP + b] = X[a][b];
}

// Schur blocks (eq. (P1P2)): P1 Shat_gamma,K^{-1} = M_K(1/mu)^{-1} + gamma M_K^{-1};
// P2 (p2 != 0) Shat_gamma,K^{-1} = (1 + gamma) M_K(1/mu)^{-1}.
template <int D>
__global__ void k_schur_setup(LevelGeo g, const double* __restrict__ mu, double gamma, int p2,
                              double* __restrict__ Sinv) {
  constexpr int NN = Dims<D>::NN, NP = Dims<D>::NP;
  constexpr const RefTab<D>& T = Ref<D>::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const double vol = D == 2 ? g.h * g.h : g.h * g.h * g.h;
  double M[NP][NP], X[NP][NP];
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      M[a][b] = 0.0;
      X[a][b] = a == b ? 1.0 : 0.0;
    }
  for (int q = 0; q < NN; ++q) {
    const double wq = T.w[q] * vol / mu[cell * NN + q];
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
      for (int b = 0; b < NP; ++b) M[a][b] += wq * T.psi[q][a] * T.psi[q][b];
  }
  // Gauss-Jordan on the SPD block (no pivoting needed)
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
#pragma unroll
  for (int a = 0; a < NP; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      double v = X[a][b];
      if (p2) v *= 1.0 + gamma;
      else if (a == b) v += gamma / (vol * T.mhat[a]);
      Sinv[cell * NP * NP + a * NP + b] = v;
    }
}

// z_p = -Sinv (v_p - B y) per cell (y == NULL: z_p = -Sinv v_p).
template <int D>
__global__ void k_schur_apply(LevelGeo g, const double* __restrict__ Sinv, const double* __restrict__ y,
                              const double* __restrict__ vp, double* __restrict__ zp) {
  constexpr int NN = Dims<D>::NN, NP = Dims<D>::NP;
  constexpr const RefTab<D>& T = Ref<D>::T;
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  int c[3];
  cell_coords<D>(g, cell, c);
  double bu[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) bu[m] = 0.0;
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    if (!y) break;
    const int a0 = 2 * c[0] + digit(n, 0), a1 = 2 * c[1] + digit(n, 1);
    const int a2 = D == 3 ? 2 * c[2] + digit(n, 2) : 0;
    bool bnd = a0 == 0 || a0 == 2 * g.N || a1 == 0 || a1 == 2 * g.N;
    if (D == 3) bnd = bnd || a2 == 0 || a2 == 2 * g.N;
    if (bnd) continue;
    const int64_t nd = node_index<D>(g, a0, a1, a2);
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
      const double v = y[comp * g.nnodes + nd];
#pragma unroll
      for (int m = 0; m < NP; ++m)
        if (T.bhat[m][comp * NN + n] != 0.0) bu[m] += T.bhat[m][comp * NN + n] * v;
    }
  }
  const double sc = -(D == 2 ? g.h : g.h * g.h);
  double t[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) t[m] = vp[cell * NP + m] - sc * bu[m];
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b) s += Sinv[cell * NP * NP + a * NP + b] * t[b];
    zp[cell * NP + a] = -s;
  }
}

// Deterministic mean of the psi_0 coefficients: red_parts(ncell) partial sums,
// then every block of the subtraction kernel reduces them the same way.
template <int NP>
__global__ void k_p0_partials(int64_t ncell, const double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x)
    s += p[c * NP];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <int NP>
__global__ void k_p0_subtract(int64_t ncell, const double* __restrict__ part, int nparts, double* __restrict__ p) {
  __shared__ double mean;
  if (threadIdx.x < 64) {
    const double s = wave_reduce_parts(part, nparts, 1, 0);
    if (threadIdx.x == 0) mean = s / (double)ncell;
  }
  __syncthreads();
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x)
    p[c * NP] -= mean;
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// [Q3]^3 x P2disc: the sinker viscosity at a cell's 4^3 Gauss points and the
// element loads of the tricubic basis.
__global__ void k3d_mu_sinker(LevelGeo g, const double* __restrict__ ctr, int ns, double omega, double delta,
                              double mu_min, double mu_max, double* __restrict__ mu) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)q3d::NQ * g.ncell) return;
  const int64_t cell = idx / q3d::NQ;
  const int q = (int)(idx - cell * q3d::NQ);
  const int64_t c0 = cell % g.N, c1 = (cell / g.N) % g.N, c2 = cell / ((int64_t)g.N * g.N);
  const double x[3] = {g.h * ((double)c0 + q3::kGx[q & 3]), g.h * ((double)c1 + q3::kGx[(q >> 2) & 3]),
                       g.h * ((double)c2 + q3::kGx[q >> 4])};
  const double chi = sinker_chi<3>(ctr, ns, omega, delta, x);
  mu[idx] = (mu_max - mu_min) * (1.0 - chi) + mu_min;
}

__global__ void k3d_rhs_elem(LevelGeo g, const double* __restrict__ ctr, int ns, double omega, double delta,
                             double beta, double* __restrict__ E) {
  const int64_t cell = blockIdx.x;
  const int n = threadIdx.x;   // 64 lanes: lane n owns basis n
  __shared__ double fq[q3d::NQ];
  const int64_t c0 = cell % g.N, c1 = (cell / g.N) % g.N, c2 = cell / ((int64_t)g.N * g.N);
  {
    const int q = n;
    const double x[3] = {g.h * ((double)c0 + q3::kGx[q & 3]), g.h * ((double)c1 + q3::kGx[(q >> 2) & 3]),
                         g.h * ((double)c2 + q3::kGx[q >> 4])};
    fq[q] = q3d::gauss_w(q) * beta * (sinker_chi<3>(ctr, ns, omega, delta, x) - 1.0);
  }
  __syncthreads();
  double be = 0.0;
  for (int q = 0; q < q3d::NQ; ++q) be += fq[q] * q3d::phi(q, n);
  const double vol = g.h * g.h * g.h;
  E[cell * q3d::NL + n] = 0.0;
  E[cell * q3d::NL + q3d::NN + n] = 0.0;
  E[cell * q3d::NL + 2 * q3d::NN + n] = vol * be;
}

void q3d_mu_sinker(const Hier& H, const Level& l, double* out, hipStream_t s) {
  const int64_t n = (int64_t)q3d::NQ * l.g.ncell;
  hipLaunchKernelGGL(k3d_mu_sinker, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers, H.omega,
                     H.delta, H.mu_min, H.mu_max, out);
}

void q3d_rhs_elem(const Hier& H, const Level& l, hipStream_t s) {
  hipLaunchKernelGGL(k3d_rhs_elem, dim3((unsigned)l.g.ncell), dim3(64), 0, s, l.g, H.centers, H.n_sinkers, H.omega,
                     H.delta, H.beta, l.E);
}

void q3_mu_sinker(const Hier& H, const Level& l, double* out, hipStream_t s) {
  if (H.dim == 3) return q3d_mu_sinker(H, l, out, s);
  const int64_t n = (int64_t)q3::NQ * l.g.ncell;
  hipLaunchKernelGGL(k3_mu_sinker, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers, H.omega, H.delta,
                     H.mu_min, H.mu_max, out);
}

void q3_rhs_elem(const Hier& H, const Level& l, hipStream_t s) {
  if (H.dim == 3) return q3d_rhs_elem(H, l, s);
  hipLaunchKernelGGL(k3_rhs_elem, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, H.centers, H.n_sinkers, H.omega,
                     H.delta, H.beta, l.E);
}

void launch_mu_sinker(const Hier& H, const Level& l, hipStream_t s) {
  if (H.deg == 3) return q3_mu_sinker(H, l, l.mu, s);
  if (H.dim == 2) {
    const int64_t n = (int64_t)Dims<2>::NQ * l.g.ncell;
    hipLaunchKernelGGL(k_mu_sinker<2>, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers,
                       H.omega, H.delta, H.mu_min, H.mu_max, l.mu);
  } else {
    const int64_t n = (int64_t)Dims<3>::NQ * l.g.ncell;
    hipLaunchKernelGGL(k_mu_sinker<3>, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers,
                       H.omega, H.delta, H.mu_min, H.mu_max, l.mu);
  }
}

template <class R>
static const R* level_mu(const Level& l);
template <>
const double* level_mu<double>(const Level& l) { return l.mu; }
template <>
const float* level_mu<float>(const Level& l) { return l.mu32; }
template <class R>
static const R* level_cw(const Level& l);
template <>
const double* level_cw<double>(const Level& l) { return l.cw; }
template <>
const float* level_cw<float>(const Level& l) { return l.cw32; }

template <class R>
static const R* level_winv(const Level& l);
template <>
const double* level_winv<double>(const Level& l) { return l.winv; }
template <>
const float* level_winv<float>(const Level& l) { return l.winv32; }

template <int D, int MODE, class R>
static void elem_launch(const Hier& H, const Level& l, const R* u, const double* p, double* pout, hipStream_t s) {
  const R* wi = level_winv<R>(l);
  if constexpr (D == 3) {
    const dim3 grid(nblk(l.g.ncell, kE3Cells));
    if ((MODE & EL_VISC) && l.cw)
      hipLaunchKernelGGL((k_elem3<MODE, true, R>), grid, dim3(64), 0, s, l.g, level_mu<R>(l), level_cw<R>(l), wi,
                         H.gamma, u, p, reinterpret_cast<R*>(l.E), pout);
    else
      hipLaunchKernelGGL((k_elem3<MODE, false, R>), grid, dim3(64), 0, s, l.g, level_mu<R>(l), (const R*)nullptr,
                         wi, H.gamma, u, p, reinterpret_cast<R*>(l.E), pout);
  } else {
    constexpr int CPW = 64 / Dims<D>::NQ;
    const dim3 grid(nblk(l.g.ncell, CPW));
    if ((MODE & EL_VISC) && l.cw)
      hipLaunchKernelGGL((k_elem<D, MODE, true, R>), grid, dim3(64), 0, s, l.g, level_mu<R>(l), level_cw<R>(l), wi,
                         H.gamma, u, p, reinterpret_cast<R*>(l.E), pout);
    else
      hipLaunchKernelGGL((k_elem<D, MODE, false, R>), grid, dim3(64), 0, s, l.g, level_mu<R>(l), (const R*)nullptr,
                         wi, H.gamma, u, p, reinterpret_cast<R*>(l.E), pout);
  }
}

template <int D, class R>
static void elem_dispatch(const Hier& H, const Level& l, int mode, const R* u, const double* p, double* pout,
                          hipStream_t s) {
  switch (mode) {
    case EL_VISC | EL_AUG: elem_launch<D, EL_VISC | EL_AUG, R>(H, l, u, p, pout, s); break;
    case EL_AUG: elem_launch<D, EL_AUG, R>(H, l, u, p, pout, s); break;
    default:
      if constexpr (std::is_same<R, double>::value) {
        if (mode == EL_BT) elem_launch<D, EL_BT, R>(H, l, u, p, pout, s);
        else if (mode == (EL_VISC | EL_AUG | EL_BT | EL_BOUT))
          elem_launch<D, EL_VISC | EL_AUG | EL_BT | EL_BOUT, R>(H, l, u, p, pout, s);
      }
      break;
  }
}

// 2D smoother: cell kernel of A_gamma on the sum of the patch outputs in the
// level's patch-output buffer, also storing that sum (the preconditioned
// direction) to z.
template <class R>
void launch_elem_asm(const Hier& H, const Level& l, R* z, hipStream_t s) {
  if (H.dim != 2) return;
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) {
      q3_asm_gather(H, l, l.zbuf, z, s);
      q3_elem(H, l, EL_VISC | EL_AUG, z, nullptr, nullptr, s);
      return;
    }
  }
  constexpr int MODE = EL_VISC | EL_AUG;
  constexpr int CPW = 64 / Dims<2>::NQ;
  const dim3 grid(nblk(l.g.ncell, CPW));
  const R* wi = level_winv<R>(l);
  const R* zb = reinterpret_cast<const R*>(l.zbuf);
  if (l.cw)
    hipLaunchKernelGGL((k_elem<2, MODE, true, R, true>), grid, dim3(64), 0, s, l.g, level_mu<R>(l), level_cw<R>(l),
                       wi, H.gamma, zb, (const double*)nullptr, reinterpret_cast<R*>(l.E), (double*)nullptr,
                       l.nvert, z);
  else
    hipLaunchKernelGGL((k_elem<2, MODE, false, R, true>), grid, dim3(64), 0, s, l.g, level_mu<R>(l),
                       (const R*)nullptr, wi, H.gamma, zb, (const double*)nullptr, reinterpret_cast<R*>(l.E),
                       (double*)nullptr, l.nvert, z);
}
template void launch_elem_asm<double>(const Hier&, const Level&, double*, hipStream_t);
template void launch_elem_asm<float>(const Hier&, const Level&, float*, hipStream_t);

void launch_eps_partials(const Hier& H, const Level& fine, hipStream_t s) {
  const int64_t n = (int64_t)(H.dim == 2 ? 9 : 27) * fine.g.ncell;
  const int np = coef_parts(n);
  if (H.dim == 2)
    hipLaunchKernelGGL(k_eps_partials<2>, dim3(np), dim3(kCoefThreads), 0, s, fine.g, H.vp_amp, H.vp_modes,
                       H.partials);
  else
    hipLaunchKernelGGL(k_eps_partials<3>, dim3(np), dim3(kCoefThreads), 0, s, fine.g, H.vp_amp, H.vp_modes,
                       H.partials);
}

void launch_mu_sinker_to(const Hier& H, const Level& l, double* out, hipStream_t s) {
  if (H.deg == 3) return q3_mu_sinker(H, l, out, s);
  const int64_t n = (int64_t)(H.dim == 2 ? 9 : 27) * l.g.ncell;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_mu_sinker<2>, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers, H.omega,
                       H.delta, H.mu_min, H.mu_max, out);
  else
    hipLaunchKernelGGL(k_mu_sinker<3>, dim3(nblk(n, 256)), dim3(256), 0, s, l.g, H.centers, H.n_sinkers, H.omega,
                       H.delta, H.mu_min, H.mu_max, out);
}

void launch_coef_fe(const Hier& H, const Level& l, const double* u, hipStream_t s) {
  const int64_t n = (int64_t)(H.dim == 2 ? 9 : 27) * l.g.ncell;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_coef_fe<2>, dim3(nblk(n, kCoefThreads)), dim3(kCoefThreads), 0, s, l.g, u, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.mu_min, H.mu_max, H.vp_floor, H.vp_tau_y, l.mu, l.cw);
  else
    hipLaunchKernelGGL(k_coef_fe<3>, dim3(nblk(n, kCoefThreads)), dim3(kCoefThreads), 0, s, l.g, u, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.mu_min, H.mu_max, H.vp_floor, H.vp_tau_y, l.mu, l.cw);
}

void launch_inject(const Hier& H, const Level& fine, const Level& coarse, const double* uf, double* uc,
                   hipStream_t s) {
  const int64_t n = (int64_t)H.dim * coarse.g.nnodes;
  if (H.dim == 2) hipLaunchKernelGGL(k_inject<2>, dim3(nblk(n, 256)), dim3(256), 0, s, fine.g, coarse.g, uf, uc);
  else hipLaunchKernelGGL(k_inject<3>, dim3(nblk(n, 256)), dim3(256), 0, s, fine.g, coarse.g, uf, uc);
}

void launch_nl_elem(const Hier& H, const Level& l, const double* u, const double* p, double* pout, hipStream_t s) {
  constexpr int MODE = EL_NL | EL_VISC | EL_AUG | EL_BT | EL_BOUT;
  const double* wi = level_winv<double>(l);
  double* E = l.E;
  if (H.dim == 3) {
    hipLaunchKernelGGL((k_elem3<MODE, false, double>), dim3(nblk(l.g.ncell, kE3Cells)), dim3(64), 0, s, l.g,
                       (const double*)H.mu0, (const double*)nullptr, wi, H.gamma, u, p, E, pout, H.vp_tau_y,
                       H.vp_floor);
  } else {
    constexpr int CPW = 64 / Dims<2>::NQ;
    hipLaunchKernelGGL((k_elem<2, MODE, false, double>), dim3(nblk(l.g.ncell, CPW)), dim3(64), 0, s, l.g,
                       (const double*)H.mu0, (const double*)nullptr, wi, H.gamma, u, p, E, pout, 0, (double*)nullptr,
                       H.vp_tau_y, H.vp_floor);
  }
}

void launch_coef_tensor(const Hier& H, const Level& l, const Level& fine, hipStream_t s) {
  const int64_t nf = (int64_t)(H.dim == 2 ? 9 : 27) * fine.g.ncell;
  const int np = coef_parts(nf);
  const int64_t n = (int64_t)(H.dim == 2 ? 9 : 27) * l.g.ncell;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_coef_tensor<2>, dim3(nblk(n, kCoefThreads)), dim3(kCoefThreads), 0, s, l.g, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.mu_min, H.mu_max, H.vp_floor, H.vp_amp, H.vp_modes, H.vp_tau_y,
                       H.vp_scale, H.partials, np, nf, l.mu, l.cw);
  else
    hipLaunchKernelGGL(k_coef_tensor<3>, dim3(nblk(n, kCoefThreads)), dim3(kCoefThreads), 0, s, l.g, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.mu_min, H.mu_max, H.vp_floor, H.vp_amp, H.vp_modes, H.vp_tau_y,
                       H.vp_scale, H.partials, np, nf, l.mu, l.cw);
}

template <class R>
void launch_elem(const Hier& H, const Level& l, int mode, const R* u, const double* p, double* pout, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_elem(H, l, mode, u, p, pout, s);
  }
  if (H.dim == 2) elem_dispatch<2, R>(H, l, mode, u, p, pout, s);
  else elem_dispatch<3, R>(H, l, mode, u, p, pout, s);
}

template <class R>
void launch_gather(const Hier& H, const Level& l, const R* base, double alpha, R* out, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_gather(H, l, base, alpha, out, s);
  }
  const int64_t n = (int64_t)H.dim * l.g.nnodes;
  const R* E = reinterpret_cast<const R*>(l.E);
  if (H.dim == 2)
    hipLaunchKernelGGL((k_gather<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, E, base, alpha, out);
  else
    hipLaunchKernelGGL((k_gather<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, E, base, alpha, out);
}

template <class R>
void launch_gather_dots(const Hier& H, const Level& l, R* out, int64_t nvec, const R* V, int64_t ldv, int nk,
                        double* part, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) {
      // the gather, then the dot products on the same partition
      q3_gather(H, l, nullptr, 1.0, out, s);
      launch_dots<R>(V, ldv, nk, out, nvec, part, s);
      return;
    }
  }
  const R* E = reinterpret_cast<const R*>(l.E);
  const int np = red_parts(nvec);
  if (H.dim == 2)
    hipLaunchKernelGGL((k_gather_dots<2, R>), dim3(np), dim3(red_threads(nvec)), 0, s, l.g, E, out, nvec, V, ldv, nk, part);
  else
    hipLaunchKernelGGL((k_gather_dots<3, R>), dim3(np), dim3(red_threads(nvec)), 0, s, l.g, E, out, nvec, V, ldv, nk, part);
}

template void launch_gather_dots<double>(const Hier&, const Level&, double*, int64_t, const double*, int64_t, int,
                                         double*, hipStream_t);
template void launch_gather_dots<float>(const Hier&, const Level&, float*, int64_t, const float*, int64_t, int,
                                        double*, hipStream_t);
template void launch_elem<double>(const Hier&, const Level&, int, const double*, const double*, double*, hipStream_t);
template void launch_elem<float>(const Hier&, const Level&, int, const float*, const double*, double*, hipStream_t);
template void launch_gather<double>(const Hier&, const Level&, const double*, double, double*, hipStream_t);
template void launch_gather<float>(const Hier&, const Level&, const float*, double, float*, hipStream_t);

void launch_rhs_elem(const Hier& H, const Level& l, hipStream_t s) {
  if (H.deg == 3) return q3_rhs_elem(H, l, s);
  if (H.dim == 2)
    hipLaunchKernelGGL(k_rhs_elem<2>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.beta, l.E);
  else
    hipLaunchKernelGGL(k_rhs_elem<3>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, H.centers,
                       H.n_sinkers, H.omega, H.delta, H.beta, l.E);
}

void launch_schur_setup(const Hier& H, const Level& l, hipStream_t s) {
  if (H.deg == 3) return q3_schur_setup(H, l, s);
  const int p2 = H.schur == 2 ? 1 : 0;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_schur_setup<2>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, l.mu, H.gamma, p2,
                       H.Sinv);
  else
    hipLaunchKernelGGL(k_schur_setup<3>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, l.mu, H.gamma, p2,
                       H.Sinv);
}

void launch_winv_setup(const Hier& H, const Level& l, hipStream_t s) {
  if (H.deg == 3) return q3_winv_setup(H, l, s);
  if (H.dim == 2)
    hipLaunchKernelGGL(k_winv_setup<2>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, l.mu, l.winv);
  else
    hipLaunchKernelGGL(k_winv_setup<3>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, l.mu, l.winv);
}

void launch_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp,
                        hipStream_t s) {
  if (H.deg == 3) return q3_schur_apply(H, l, y, vp, zp, s);
  if (H.dim == 2)
    hipLaunchKernelGGL(k_schur_apply<2>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, H.Sinv, y, vp, zp);
  else
    hipLaunchKernelGGL(k_schur_apply<3>, dim3(nblk(l.g.ncell, 128)), dim3(128), 0, s, l.g, H.Sinv, y, vp, zp);
}

void launch_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s) {
  if (H.deg == 3) return q3_project_mean(H, l, p, s);
  const int np = red_parts(l.g.ncell);
  if (H.dim == 2) {
    hipLaunchKernelGGL(k_p0_partials<3>, dim3(np), dim3(red_threads(l.g.ncell)), 0, s, l.g.ncell, p, H.partials);
    hipLaunchKernelGGL(k_p0_subtract<3>, dim3(nblk(l.g.ncell, 256)), dim3(256), 0, s, l.g.ncell, H.partials, np, p);
  } else {
    hipLaunchKernelGGL(k_p0_partials<4>, dim3(np), dim3(red_threads(l.g.ncell)), 0, s, l.g.ncell, p, H.partials);
    hipLaunchKernelGGL(k_p0_subtract<4>, dim3(nblk(l.g.ncell, 256)), dim3(256), 0, s, l.g.ncell, H.partials, np, p);
  }
}

}  // namespace stk
