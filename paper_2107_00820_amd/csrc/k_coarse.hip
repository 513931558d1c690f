// Coarsest level: A_0,gamma over the interior unknowns, its explicit inverse
// by a blocked symmetric sweep, and the solve as one symmetric tile GEMV.
// The paper solves the coarsest level with a sparse direct solver (Section
// 5.1); the coarse systems here (<= ~4*10^4 unknowns) fit HBM as dense
// symmetric matrices, and an explicit inverse turns every coarse solve into
// one fully parallel, coalesced pass instead of two sequential triangular
// sweeps.
//
// Storage: the lower triangle in 64 x 64 tiles, tile (I, J), J <= I, at
// index I(I+1)/2 + J, row-major inside the tile; diagonal tiles hold both
// triangles. Unknowns beyond n (padding of the last tile) carry an identity
// block, which the sweep keeps and the solve ignores.
//
// Sweep of pivot block K (symmetric Gauss-Jordan; after all blocks the array
// holds -A^{-1}): with P = A_KK and C_I = A_IK (old),
//   A_KK <- -P^{-1};  A_IK <- C_I P^{-1};  A_IJ <- A_IJ - C_I P^{-1} C_J^T,
// for I, J != K. P stays SPD (a Schur complement of an SPD matrix). Every
// product with P^{-1} goes through the Cholesky factor P = L L^T: with
// V_I = C_I L^{-T} the update is the symmetric A_IJ -= V_I V_J^T and the new
// off-diagonal block is V_I L^{-1}. Multiplying by an explicit P^{-1}
// instead loses accuracy in proportion to kappa(P), and the pivot blocks of
// these coarse operators are about as ill-conditioned as the whole matrix;
// the factored form keeps the inverse as accurate as one formed from the
// Cholesky factor of the whole matrix. The rank-64 updates are 64 x 64 x 64
// tile products on the FP64 matrix cores (v_mfma_f64_16x16x4f64); the pivot
// factorisation and inversion run in LDS. Pivots are taken in pairs with a
// look-ahead on the second one's block column, so that one pass over the
// matrix applies both updates (half the passes; the same products, summed
// in one accumulator per tile).
#include "stk_q3d.h"
#include "stk_spd.h"

namespace stk {

constexpr int kT = 64;           // tile width
constexpr int kTT = kT * kT;
constexpr int kLd = kT + 1;      // LDS row stride (doubles)


// Interior unknown i (component-major over the (n1-2)^d interior nodes,
// (kN-1)^d for degree k) -> (component, node coordinates).
template <int D>
__device__ inline int interior_dof(const LevelGeo& g, int64_t i, int nd[3]) {
  const int ni = g.n1 - 2;
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
__device__ inline int64_t interior_stored(const LevelGeo& g, int64_t i) {
  int nd[3];
  const int c = interior_dof<D>(g, i, nd);
  return c * g.nnodes + node_index<D>(g, nd[0], nd[1], nd[2]);
}

// Tile t of the lower triangle -> (I, J).
__device__ inline void tile_ij(int64_t t, int& I, int& J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  I = i;
  J = (int)(t - (int64_t)i * (i + 1) / 2);
}

__device__ inline const double* tile_ptr(const double* A, int I, int J) {
  return A + ((int64_t)I * (I + 1) / 2 + J) * kTT;
}
__device__ inline double* tile_ptr(double* A, int I, int J) {
  return A + ((int64_t)I * (I + 1) / 2 + J) * kTT;
}

// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_coarse_assemble(LevelGeo g, const double* __restrict__ mu,
                                                          const double* __restrict__ cw,
                                                          const double* __restrict__ winv, double gamma, int64_t n,
                                                          int64_t ntiles, double* __restrict__ A) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= ntiles * kTT) return;
  const int64_t t = idx / kTT;
  const int e = (int)(idx - t * kTT);
  int I, J;
  tile_ij(t, I, J);
  const int64_t i = (int64_t)I * kT + e / kT, j = (int64_t)J * kT + e % kT;
  double v;
  if (i < n && j < n) {
    int ni[3], nj[3];
    const int ci = interior_dof<D>(g, i, ni);
    const int cj = interior_dof<D>(g, j, nj);
    v = global_entry<D>(g, mu, cw, winv, gamma, ci, ni, cj, nj);
  } else {
    v = i == j ? 1.0 : 0.0;
  }
  A[idx] = v;
}

// [Q3]^2 x P2disc: the same tiles from the degree-3 entries of A_gamma.
__global__ void __launch_bounds__(256) k3_coarse_assemble(LevelGeo g, const double* __restrict__ mu,
                                                           const double* __restrict__ winv, double gamma,
                                                           int64_t n, int64_t ntiles, double* __restrict__ A) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= ntiles * kTT) return;
  const int64_t t = idx / kTT;
  const int e = (int)(idx - t * kTT);
  int I, J;
  tile_ij(t, I, J);
  const int64_t i = (int64_t)I * kT + e / kT, j = (int64_t)J * kT + e % kT;
  double v;
  if (i < n && j < n) {
    int ni[3], nj[3];
    const int ci = interior_dof<2>(g, i, ni);
    const int cj = interior_dof<2>(g, j, nj);
    v = q3::global_entry(g, mu, winv, gamma, ci, ni[0], ni[1], cj, nj[0], nj[1]);
  } else {
    v = i == j ? 1.0 : 0.0;
  }
  A[idx] = v;
}

// [Q3]^3 x P2disc: the same tiles from the cell matrices CM[cell][192][192]
// of the level (sum over the cells that contain both nodes, ascending z, y, x).
__global__ void __launch_bounds__(256) k3d_coarse_assemble(LevelGeo g, const double* __restrict__ CM, int64_t n,
                                                            int64_t ntiles, double* __restrict__ A) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= ntiles * kTT) return;
  const int64_t t = idx / kTT;
  const int e = (int)(idx - t * kTT);
  int I, J;
  tile_ij(t, I, J);
  const int64_t i = (int64_t)I * kT + e / kT, j = (int64_t)J * kT + e % kT;
  double v = i == j ? 1.0 : 0.0;
  if (i < n && j < n) {
    int ni[3], nj[3];
    const int ci = interior_dof<3>(g, i, ni);
    const int cj = interior_dof<3>(g, j, nj);
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
                const int64_t cell = (int64_t)ca[0][t0] + (int64_t)g.N * ((int64_t)ca[1][t1] + (int64_t)g.N * ca[2][t2]);
                const int a = la[0][t0] + 4 * la[1][t1] + 16 * la[2][t2];
                const int b = lb[0][u0] + 4 * lb[1][u1] + 16 * lb[2][u2];
                v += CM[cell * (192 * 192) + (int64_t)(ci * 64 + a) * 192 + cj * 64 + b];
              }
          }
      }
  }
  A[idx] = v;
}

// Pivot: with A_KK = L L^T, Linv = L^{-1} (64 x 64 row-major, zeros above
// the diagonal) and Pinv = A_KK^{-1} = L^{-T} L^{-1} (full symmetric), by the
// blocked Cholesky inversion in 16 x 16 tiles on the FP64 matrix cores.
// Batched use (degree-3 3D star patches): blockIdx.y selects a matrix at
// A + y * as with its work at + y * ws; the coarse level runs one matrix.
__global__ void __launch_bounds__(256) k_sweep_pivot(const double* __restrict__ A, int K,
                                                      double* __restrict__ Pinv, double* __restrict__ Linv,
                                                      int* __restrict__ flag, int64_t as = 0, int64_t ws = 0) {
  A += blockIdx.y * as;
  Pinv += blockIdx.y * ws;
  Linv += blockIdx.y * ws;
  constexpr int NB = kT / 16, NT = NB * (NB + 1) / 2;
  __shared__ double L[NT * kTile17];
  __shared__ double W[NB * kTile17];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  const double* T = tile_ptr(A, K, K);
  for (int e = threadIdx.x; e < NT * 256; e += blockDim.x) {
    const int t = e / 256, r = (e % 256) / 16, c = e % 16;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    L[t * kTile17 + r * 17 + c] = T[(16 * I + r) * kT + 16 * J + c];
  }
  __syncthreads();
  spd_cholinv_lower16(L, NB, W, &bad);
  for (int e = threadIdx.x; e < kTT; e += blockDim.x) {
    const int r = e / kT, c = e % kT;
    Linv[e] = c > r ? 0.0 : L[ltile(r / 16, c / 16) * kTile17 + (r % 16) * 17 + c % 16];
  }
  __syncthreads();   // L is read above before the product below replaces it
  spd_xtx_lower16(L, NB, W);
  for (int e = threadIdx.x; e < kTT; e += blockDim.x) {
    int r = e / kT, c = e % kT;
    if (c > r) { const int t = r; r = c; c = t; }
    Pinv[e] = L[ltile(r / 16, c / 16) * kTile17 + (r % 16) * 17 + c % 16];
  }
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// Stage block C_I = A_IK (I != K) into LDS as X[r][k] (row stride kLd).
__device__ inline void stage_panel(const double* __restrict__ A, int I, int K, double* X) {
  if (I > K) {
    const double* T = tile_ptr(A, I, K);
    for (int e = threadIdx.x; e < kTT; e += blockDim.x) X[(e / kT) * kLd + e % kT] = T[e];
  } else {
    const double* T = tile_ptr(A, K, I);   // A_IK = (A_KI)^T
    for (int e = threadIdx.x; e < kTT; e += blockDim.x) X[(e % kT) * kLd + e / kT] = T[e];
  }
}

__device__ inline void stage_full(const double* __restrict__ T, double* X) {
  for (int e = threadIdx.x; e < kTT; e += blockDim.x) X[(e / kT) * kLd + e % kT] = T[e];
}

// acc = X Y^T over 64 x 64 x 64 with four wavefronts; wavefront w owns the
// 32 x 32 quadrant (rows 32(w/2).., cols 32(w%2)..) as 2 x 2 MFMA 16 x 16
// blocks. Operands (v_mfma_f64_16x16x4f64): lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l is D[l/16 + 4r][l%16].
__device__ inline void tile_gemm_xyt(const double* X, const double* Y, d4 acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = 32 * (w >> 1), cb = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < kT; k0 += 4) {
    const int k = k0 + lk;
    const double a0 = X[(rb + li) * kLd + k], a1 = X[(rb + 16 + li) * kLd + k];
    const double b0 = Y[(cb + li) * kLd + k], b1 = Y[(cb + 16 + li) * kLd + k];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// Output element of register r in block (a, b) for this lane: (row, col).
__device__ inline void acc_rc(int a, int b, int r, int& row, int& col) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  row = 32 * (w >> 1) + 16 * a + (lane >> 4) + 4 * r;
  col = 32 * (w & 1) + 16 * b + (lane & 15);
}

// V_I = C_I L^{-T} for every I != K (grid: one workgroup per block row).
__global__ void __launch_bounds__(256) k_sweep_panel(const double* __restrict__ A, int K,
                                                      const double* __restrict__ Linv, double* __restrict__ W,
                                                      int64_t as = 0, int64_t ws = 0) {
  A += blockIdx.y * as;
  Linv += blockIdx.y * ws;
  W += blockIdx.y * ws;
  __shared__ double X[kT * kLd];
  __shared__ double Y[kT * kLd];
  const int I = blockIdx.x;
  if (I == K) return;
  stage_panel(A, I, K, X);
  stage_full(Linv, Y);       // X Y^T = C_I L^{-T}
  __syncthreads();
  d4 acc[2][2];
  tile_gemm_xyt(X, Y, acc);
  // stored transposed, V_I[r][k] at k*64 + r: the consumers' MFMA operand
  // loads (16 rows at a fixed k per lane group) then read 128 contiguous bytes
  double* out = W + (int64_t)I * kTT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_rc(a, b, r, row, col);
        out[col * kT + row] = acc[a][b][r];
      }
}

// acc += X Y^T over k = 0..63 for panel blocks stored transposed (X[r][k]
// at k*64 + r). The MFMA operands are read straight from global memory (the
// panel blocks are shared by a whole block row / column and stay in L2), so
// there is no LDS staging or barrier.
__device__ inline void panel_gemm_acc(const double* __restrict__ X, const double* __restrict__ Y, d4 acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = 32 * (w >> 1), cb = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < kT; k0 += 4) {
    const int k = k0 + lk;
    const double a0 = X[k * kT + rb + li], a1 = X[k * kT + rb + 16 + li];
    const double b0 = Y[k * kT + cb + li], b1 = Y[k * kT + cb + 16 + li];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ inline void tile_sub(double* __restrict__ T, const d4 acc[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_rc(a, b, r, row, col);
        T[row * kT + col] -= acc[a][b][r];
      }
}

// A_IJ -= V_I V_J^T for every lower tile with I, J != K.
__global__ void __launch_bounds__(256) k_sweep_update(double* __restrict__ A, int K, const double* __restrict__ W,
                                                       int64_t as = 0, int64_t ws = 0) {
  A += blockIdx.y * as;
  W += blockIdx.y * ws;
  int I, J;
  tile_ij(blockIdx.x, I, J);
  if (I == K || J == K) return;
  d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  panel_gemm_acc(W + (int64_t)I * kTT, W + (int64_t)J * kTT, acc);
  tile_sub(tile_ptr(A, I, J), acc);
}

// Two pivot blocks per pass over the matrix (look-ahead): after the panel of
// pivot K, only block column K+1 is brought up to date (this kernel: tile of
// (I, K+1) for every I != K, including the pivot tile (K+1, K+1)), so that
// pivot K+1 can be factored and its panel formed before the one pass that
// applies both rank-64 updates (k_sweep_update2).
__global__ void __launch_bounds__(256) k_sweep_colupdate(double* __restrict__ A, int K, const double* __restrict__ W) {
  const int I = blockIdx.x;
  if (I == K) return;
  const int Kn = K + 1;
  const int a = I > Kn ? I : Kn, b = I > Kn ? Kn : I;   // lower tile (a, b), a >= b
  d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  panel_gemm_acc(W + (int64_t)a * kTT, W + (int64_t)b * kTT, acc);
  tile_sub(tile_ptr(A, a, b), acc);
}

// The combined update of pivots K (panel V) and K+1 (panel V2): every lower
// tile outside block row and column K+1 loses V2_I V2_J^T, and those outside
// block row and column K as well V_I V_J^T (block row and column K already
// hold their step-K values, written by k_sweep_write).
__global__ void __launch_bounds__(256) k_sweep_update2(double* __restrict__ A, int K, const double* __restrict__ V,
                                                        const double* __restrict__ V2) {
  int I, J;
  tile_ij(blockIdx.x, I, J);
  if (I == K + 1 || J == K + 1) return;
  d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  if (I != K && J != K) panel_gemm_acc(V + (int64_t)I * kTT, V + (int64_t)J * kTT, acc);
  panel_gemm_acc(V2 + (int64_t)I * kTT, V2 + (int64_t)J * kTT, acc);
  tile_sub(tile_ptr(A, I, J), acc);
}

// A_IK <- V_I L^{-1} (tile (I,K) for I > K, its transpose in tile (K,I) for
// I < K); A_KK <- -P^{-1}. Operands straight from global memory as in the
// update.
__global__ void __launch_bounds__(256) k_sweep_write(double* __restrict__ A, int K, const double* __restrict__ Pinv,
                                                      const double* __restrict__ Linv, const double* __restrict__ W,
                                                      int64_t as = 0, int64_t ws = 0) {
  A += blockIdx.y * as;
  Pinv += blockIdx.y * ws;
  Linv += blockIdx.y * ws;
  W += blockIdx.y * ws;
  const int I = blockIdx.x;
  if (I == K) {
    double* T = tile_ptr(A, K, K);
    for (int e = threadIdx.x; e < kTT; e += blockDim.x) T[e] = -Pinv[e];
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = 32 * (w >> 1), cb = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
  const double* X = W + (int64_t)I * kTT;                  // V_I[r][k] at k*64 + r
  d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < kT; k0 += 4) {
    const int k = k0 + lk;
    const double a0 = X[k * kT + rb + li], a1 = X[k * kT + rb + 16 + li];
    const double b0 = Linv[k * kT + cb + li], b1 = Linv[k * kT + cb + 16 + li];   // B[k][c] = L^{-1}[k][c]
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  double* T = I > K ? tile_ptr(A, I, K) : tile_ptr(A, K, I);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_rc(a, b, r, row, col);
        if (I > K) T[row * kT + col] = acc[a][b][r];
        else T[col * kT + row] = acc[a][b][r];
      }
}

// ---------------------------------------------------------------------------
// Solve x = A^{-1} b = -(stored) b.
// bc[i] = b at interior unknown i (0 in the padding).
template <int D, class R>
__global__ void k_coarse_gather(LevelGeo g, int64_t n, int64_t npad, const R* __restrict__ b,
                                double* __restrict__ bc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npad) return;
  bc[i] = i < n ? (double)b[interior_stored<D>(g, i)] : 0.0;
}

// One workgroup per stored tile (I, J): part[I][J] = T x_J and, below the
// diagonal, part[J][I] = T^T x_I (each slot written exactly once). Thread
// (tr, tc) = (t / 16, t % 16) holds the 4 x 4 block rows 4tr.., columns
// 4tc.. in registers (a wavefront reads 16 full rows, 512 contiguous bytes
// each); row sums are reduced across the 16 threads of a row band, column
// sums across the 4 bands of a wavefront and then the 4 wavefronts, all in a
// fixed order.
__global__ void __launch_bounds__(256) k_coarse_tile_gemv(const double* __restrict__ A, int nb,
                                                           const double* __restrict__ bc,
                                                           double* __restrict__ part) {
  __shared__ double vs[4][kT];
  int I, J;
  tile_ij(blockIdx.x, I, J);
  const double* T = tile_ptr(A, I, J);
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15, wave = t >> 6;
  const double* xj = bc + (int64_t)J * kT;
  const double* xi = bc + (int64_t)I * kT;
  double m[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) m[a][b] = T[(4 * tr + a) * kT + 4 * tc + b];
  double xc[4], xr[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) xc[b] = xj[4 * tc + b];
#pragma unroll
  for (int a = 0; a < 4; ++a) xr[a] = xi[4 * tr + a];
  double u[4], v[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    u[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) u[a] += m[a][b] * xc[b];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    v[b] = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) v[b] += m[a][b] * xr[a];
  }
  // rows: sum over the 16 lanes tc of this row band (lanes 16*band .. +15)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) u[a] += __shfl_xor(u[a], off, 64);
  if (tc == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a) part[((int64_t)I * nb + J) * kT + 4 * tr + a] = u[a];
  }
  if (I != J) {
    // columns: the 4 row bands of this wavefront (lane bits 4, 5), then the 4 wavefronts
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      v[b] += __shfl_xor(v[b], 16, 64);
      v[b] += __shfl_xor(v[b], 32, 64);
    }
    if ((t & 48) == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) vs[wave][4 * tc + b] = v[b];
    }
    __syncthreads();
    if (t < kT) part[((int64_t)J * nb + I) * kT + t] = (vs[0][t] + vs[1][t]) + (vs[2][t] + vs[3][t]);
  }
}

// x at interior unknown i = -sum_J part[I][J][r]: one workgroup per row
// tile I; wavefront w sums the partials J = w, w + 16, .. in order, and the
// 16 wavefront sums are added in order w = 0..15 (a fixed order independent
// of timing). Dirichlet entries are zeroed beforehand.
constexpr int kReduceWaves = 16;

template <int D, class R>
__global__ void __launch_bounds__(kReduceWaves * kT) k_coarse_reduce(LevelGeo g, int64_t n, int nb,
                                                                     const double* __restrict__ part,
                                                                     R* __restrict__ x) {
  __shared__ double sh[kReduceWaves][kT];
  const int I = blockIdx.x;
  const int r = threadIdx.x % kT, w = threadIdx.x / kT;
  double s = 0.0;
  for (int J = w; J < nb; J += kReduceWaves) s += part[((int64_t)I * nb + J) * kT + r];
  sh[w][r] = s;
  __syncthreads();
  const int64_t i = (int64_t)I * kT + r;
  if (w == 0 && i < n) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kReduceWaves; ++k) t += sh[k][r];
    x[interior_stored<D>(g, i)] = (R)(-t);
  }
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int coarse_tiles(int64_t n) { return (int)((n + kT - 1) / kT); }

void launch_coarse_assemble(const Hier& H, const Level& l, double* A, hipStream_t s) {
  const int64_t nb = coarse_tiles(H.n0);
  const int64_t ntiles = nb * (nb + 1) / 2;
  const dim3 grid(nblk(ntiles * kTT, 256));
  if (H.deg == 3 && H.dim == 3) {
    q3d_cell_matrices(H, l, H.q3cm, s);
    hipLaunchKernelGGL(k3d_coarse_assemble, grid, dim3(256), 0, s, l.g, (const double*)H.q3cm, H.n0, ntiles, A);
  } else if (H.deg == 3)
    hipLaunchKernelGGL(k3_coarse_assemble, grid, dim3(256), 0, s, l.g, (const double*)l.mu, (const double*)l.winv,
                       H.gamma, H.n0, ntiles, A);
  else if (H.dim == 2)
    hipLaunchKernelGGL(k_coarse_assemble<2>, grid, dim3(256), 0, s, l.g, l.mu, l.cw, l.winv, H.gamma, H.n0, ntiles, A);
  else
    hipLaunchKernelGGL(k_coarse_assemble<3>, grid, dim3(256), 0, s, l.g, l.mu, l.cw, l.winv, H.gamma, H.n0, ntiles, A);
}

// work: P^{-1} (kTT) + two panels V, V2 (nb * kTT each) doubles; a pivot's
// L^{-1} sits in the block-row slot of its own panel, which the panel leaves
// unused. Pivots go in pairs (one pass over the matrix per pair; the pivot
// of a pair's second block is factored after the first block's panel has
// updated its block column), the last one alone if nb is odd.
int launch_coarse_invert(const Hier& H, double* A, int64_t n, double* work, hipStream_t s) {
  const int nb = coarse_tiles(n);
  const int64_t ntiles = (int64_t)nb * (nb + 1) / 2;
  double* Pinv = work;
  double* V = work + kTT;
  double* V2 = V + (int64_t)nb * kTT;
  int K = 0;
  for (; K + 1 < nb; K += 2) {
    double* Linv = V + (int64_t)K * kTT;
    double* Linv2 = V2 + (int64_t)(K + 1) * kTT;
    hipLaunchKernelGGL(k_sweep_pivot, dim3(1), dim3(256), 0, s, A, K, Pinv, Linv, H.flag);
    hipLaunchKernelGGL(k_sweep_panel, dim3(nb), dim3(256), 0, s, A, K, (const double*)Linv, V);
    hipLaunchKernelGGL(k_sweep_colupdate, dim3(nb), dim3(256), 0, s, A, K, (const double*)V);
    hipLaunchKernelGGL(k_sweep_write, dim3(nb), dim3(256), 0, s, A, K, (const double*)Pinv, (const double*)Linv,
                       (const double*)V);
    hipLaunchKernelGGL(k_sweep_pivot, dim3(1), dim3(256), 0, s, A, K + 1, Pinv, Linv2, H.flag);
    hipLaunchKernelGGL(k_sweep_panel, dim3(nb), dim3(256), 0, s, A, K + 1, (const double*)Linv2, V2);
    hipLaunchKernelGGL(k_sweep_update2, dim3((unsigned)ntiles), dim3(256), 0, s, A, K, (const double*)V,
                       (const double*)V2);
    hipLaunchKernelGGL(k_sweep_write, dim3(nb), dim3(256), 0, s, A, K + 1, (const double*)Pinv,
                       (const double*)Linv2, (const double*)V2);
  }
  if (K < nb) {
    double* Linv = V + (int64_t)K * kTT;
    hipLaunchKernelGGL(k_sweep_pivot, dim3(1), dim3(256), 0, s, A, K, Pinv, Linv, H.flag);
    hipLaunchKernelGGL(k_sweep_panel, dim3(nb), dim3(256), 0, s, A, K, (const double*)Linv, V);
    hipLaunchKernelGGL(k_sweep_update, dim3((unsigned)ntiles), dim3(256), 0, s, A, K, (const double*)V);
    hipLaunchKernelGGL(k_sweep_write, dim3(nb), dim3(256), 0, s, A, K, (const double*)Pinv, (const double*)Linv,
                       (const double*)V);
  }
  return 0;
}

// The coarse solve is FP64 in both forms; R only selects the vector storage.
// H.cvec holds bc (nb*64 doubles), H.cpart the tile partials (nb*nb*64).
// In-place -A^{-1} of `count` SPD matrices of nb x nb tiles (coarse-matrix
// tile layout; matrix k at A + k * as, its work of (nb + 1) * 4096 doubles at
// work + k * ws): the single-pivot sweep, every launch over the whole batch.
void launch_tile_invert_batched(const Hier& H, double* A, int nb, int64_t count, int64_t as, double* work,
                                int64_t ws, hipStream_t s) {
  const int64_t ntiles = (int64_t)nb * (nb + 1) / 2;
  const unsigned cy = (unsigned)count;
  double* Pinv = work;
  double* V = work + kTT;
  for (int K = 0; K < nb; ++K) {
    double* Linv = V + (int64_t)K * kTT;
    hipLaunchKernelGGL(k_sweep_pivot, dim3(1, cy), dim3(256), 0, s, (const double*)A, K, Pinv, Linv, H.flag, as, ws);
    hipLaunchKernelGGL(k_sweep_panel, dim3(nb, cy), dim3(256), 0, s, (const double*)A, K, (const double*)Linv, V, as,
                       ws);
    hipLaunchKernelGGL(k_sweep_update, dim3((unsigned)ntiles, cy), dim3(256), 0, s, A, K, (const double*)V, as, ws);
    hipLaunchKernelGGL(k_sweep_write, dim3(nb, cy), dim3(256), 0, s, A, K, (const double*)Pinv, (const double*)Linv,
                       (const double*)V, as, ws);
  }
}

template <class R>
void launch_coarse_apply(const Hier& H, const Level& l, const R* b, R* x, hipStream_t s) {
  const int nb = coarse_tiles(H.n0);
  const int64_t npad = (int64_t)nb * kT, ntiles = (int64_t)nb * (nb + 1) / 2;
  launch_fill<R>(x, 0.0, (int64_t)H.dim * l.g.nnodes, s);
  if (H.dim == 2)
    hipLaunchKernelGGL((k_coarse_gather<2, R>), dim3(nblk(npad, 256)), dim3(256), 0, s, l.g, H.n0, npad, b, H.cvec);
  else
    hipLaunchKernelGGL((k_coarse_gather<3, R>), dim3(nblk(npad, 256)), dim3(256), 0, s, l.g, H.n0, npad, b, H.cvec);
  hipLaunchKernelGGL(k_coarse_tile_gemv, dim3((unsigned)ntiles), dim3(256), 0, s, H.Ainv0, nb, H.cvec, H.cpart);
  const dim3 rgrid((unsigned)nb), rblk(kReduceWaves * kT);
  if (H.dim == 2)
    hipLaunchKernelGGL((k_coarse_reduce<2, R>), rgrid, rblk, 0, s, l.g, H.n0, nb, H.cpart, x);
  else
    hipLaunchKernelGGL((k_coarse_reduce<3, R>), rgrid, rblk, 0, s, l.g, H.n0, nb, H.cpart, x);
}

template void launch_coarse_apply<double>(const Hier&, const Level&, const double*, double*, hipStream_t);
template void launch_coarse_apply<float>(const Hier&, const Level&, const float*, float*, hipStream_t);

}  // namespace stk
