// Setup of the vertex-star patch inverses (Section 4.1, eq. (viim)): one
// workgroup per patch assembles the patch matrix from Gauss-point integrals of
// the cells of the star (equal to the rows and columns of the assembled
// A_gamma) and inverts it through its Cholesky factor; the inverse is stored
// as a packed lower triangle in the interleaved layout the patch solve reads
// (element k of patch s at ((s/64)*P + k)*64 + s%64, P = n(n+1)/2).
#include "stk_spd.h"

namespace stk {

template <int D>
__global__ void k_patch_setup(LevelGeo g, const double* __restrict__ mu, const double* __restrict__ cw,
                              const double* __restrict__ winv, double gamma, int n,
                              const int* __restrict__ verts, int count, double* __restrict__ inv,
                              int* __restrict__ flag) {
  extern __shared__ double sm[];
  const int s = blockIdx.x;
  if (s >= count) return;
  const int ld = n + 1;
  double* a = sm;
  double* tmp = sm + n * ld;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  int lo[3], ext[3], vc[3];
  patch_box<D>(g, verts[s], lo, ext, vc);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    if (j > i) continue;
    int ni[3], nj[3];
    const int ci = patch_dof<D>(i, lo, ext, ni);
    const int cj = patch_dof<D>(j, lo, ext, nj);
    const double v = global_entry<D>(g, mu, cw, winv, gamma, ci, ni, cj, nj);
    a[i * ld + j] = v;
    a[j * ld + i] = v;
  }
  __syncthreads();
  spd_invert_lds(a, n, ld, tmp, &bad);
  const int64_t P = (int64_t)n * (n + 1) / 2;
  double* dst = inv + ((int64_t)(s / 64) * P) * 64 + (s % 64);
  for (int i = 0; i < n; ++i)
    for (int j = threadIdx.x; j <= i; j += blockDim.x)
      dst[((int64_t)i * (i + 1) / 2 + j) * 64] = a[i * ld + j];
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// 3D interior patches (81 unknowns): the same entries as k_patch_setup,
// assembled cell by cell into the lower 16 x 16 tiles of the matrix padded
// to 96 x 96 with the identity, then inverted through its Cholesky factor by
// spd_invert_lower16 (tile products on the FP64 matrix cores). Per star cell
// the Gauss-point weights, coefficients and the reference gradients of its 8
// patch nodes are staged in LDS, and each thread forms entries of the cell's
// 24 x 24 block (same arithmetic, and same cell order, as global_entry). LDS:
// 21 matrix tiles and 6 scratch tiles, within the 64 KB a workgroup can use.
constexpr int kP81 = 81, kP81Blocks = 6;

__global__ void __launch_bounds__(256) k_patch_setup81(LevelGeo g, const double* __restrict__ mu,
                                                        const double* __restrict__ cw,
                                                        const double* __restrict__ winv, double gamma,
                                                        const int* __restrict__ verts, int count,
                                                        double* __restrict__ inv, int* __restrict__ flag) {
  constexpr int NT = kP81Blocks * (kP81Blocks + 1) / 2, NN = 27, NP = 4, NS = 6;
  // scratch (W): staging of one cell during assembly, tiles during inversion
  constexpr int kWmu = 0, kWv = kWmu + NN, kWinv = kWv + NN * NS, kGrad = kWinv + NP * NP,
                kBh = kGrad + 8 * NN * 3, kStage = kBh + NP * 24;
  constexpr int kW = kStage > kP81Blocks * kTile17 ? kStage : kP81Blocks * kTile17;
  __shared__ double L[NT * kTile17];
  __shared__ double W[kW];
  __shared__ int bad;
  const int s = blockIdx.x;
  if (s >= count) return;
  constexpr int n = kP81;
  const RefTab<3>& T = ctab<3>();
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  int lo[3], ext[3], vc[3];
  patch_box<3>(g, verts[s], lo, ext, vc);
  for (int e = tid; e < NT * kTile17; e += blockDim.x) L[e] = 0.0;
  __syncthreads();
  const double sc = g.h;   // h^{d-2}
  for (int cd = 0; cd < 8; ++cd) {
    const int dx = cd & 1, dy = (cd >> 1) & 1, dz = cd >> 2;
    const int64_t cell = cell_index<3>(g, vc[0] - 1 + dx, vc[1] - 1 + dy, vc[2] - 1 + dz);
    for (int t = tid; t < kStage; t += blockDim.x) {
      double v = 0.0;
      if (t < kWv) {
        v = T.w[t] * mu[cell * NN + t];
      } else if (t < kWinv) {
        const int q = (t - kWv) / NS, k = (t - kWv) % NS;   // [q][sym k]
        v = cw ? cw[(cell * NS + k) * NN + q] : 0.0;
      } else if (t < kGrad) {
        v = winv ? winv[cell * NP * NP + (t - kWinv)] : 0.0;
      } else if (t < kBh) {
        const int u = t - kGrad, e = u / (NN * 3), q = (u / 3) % NN, k = u % 3;   // [e][q][k]
        const int nl = ((e & 1) - dx + 1) + 3 * (((e >> 1) & 1) - dy + 1) + 9 * ((e >> 2) - dz + 1);
        v = T.dphi[q][nl][k];
      } else {
        const int u = t - kBh, m = u / 24, c = (u % 24) / 8, e = u % 8;   // [m][c*8+e]
        const int nl = ((e & 1) - dx + 1) + 3 * (((e >> 1) & 1) - dy + 1) + 9 * ((e >> 2) - dz + 1);
        v = T.bhat[m][c * NN + nl];
      }
      W[t] = v;
    }
    __syncthreads();
    for (int pr = tid; pr < 24 * 25 / 2; pr += blockDim.x) {
      int r = 0;
      while ((r + 1) * (r + 2) / 2 <= pr) ++r;
      const int c2 = pr - r * (r + 1) / 2;
      const int ci = r / 8, ei = r % 8, cj = c2 / 8, ej = c2 % 8;
      const double* ga = W + kGrad + ei * NN * 3;
      const double* gb = W + kGrad + ej * NN * 3;
      double acc = 0.0;
      for (int q = 0; q < NN; ++q) {
        double gg = ga[q * 3 + cj] * gb[q * 3 + ci];
        if (ci == cj) {
#pragma unroll
          for (int k = 0; k < 3; ++k) gg += ga[q * 3 + k] * gb[q * 3 + k];
        }
        acc += W[kWmu + q] * gg;
        if (cw) {
          double wi = 0.0, wj = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            wi += W[kWv + q * NS + SymIdx<3>::at(ci, k)] * ga[q * 3 + k];
            wj += W[kWv + q * NS + SymIdx<3>::at(cj, k)] * gb[q * 3 + k];
          }
          acc -= T.w[q] * wi * wj;
        }
      }
      double al = 0.0;
      const double* bh = W + kBh;
      if (winv) {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          double t2 = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) t2 += W[kWinv + m * NP + k] * bh[k * 24 + c2];
          al += bh[m * 24 + r] * t2;
        }
      } else {
#pragma unroll
        for (int m = 0; m < NP; ++m) al += bh[m * 24 + r] * bh[m * 24 + c2] * kInvMhat[m];
      }
      const double v = sc * (acc + gamma * al);
      // patch unknowns: component-major, node offset (d + e) per axis from 2v - 1
      const int li = (dx + (ei & 1)) + 3 * (dy + ((ei >> 1) & 1)) + 9 * (dz + (ei >> 2));
      const int lj = (dx + (ej & 1)) + 3 * (dy + ((ej >> 1) & 1)) + 9 * (dz + (ej >> 2));
      const int i = ci * NN + li, j = cj * NN + lj;   // i >= j
      const int I = i / 16, J = j / 16;
      L[ltile(I, J) * kTile17 + (i % 16) * 17 + j % 16] += v;
      if (I == J && i != j) L[ltile(I, J) * kTile17 + (j % 16) * 17 + i % 16] += v;
    }
    __syncthreads();
  }
  for (int i = n + tid; i < 16 * kP81Blocks; i += blockDim.x) L[ltile(i / 16, i / 16) * kTile17 + (i % 16) * 18] = 1.0;
  __syncthreads();
  spd_invert_lower16(L, kP81Blocks, W, &bad);
  const int64_t P = (int64_t)n * (n + 1) / 2;
  double* dst = inv + ((int64_t)(s / 64) * P) * 64 + (s % 64);
  for (int i = 0; i < n; ++i)
    for (int j = threadIdx.x; j <= i; j += blockDim.x)
      dst[((int64_t)i * (i + 1) / 2 + j) * 64] = L[ltile(i / 16, j / 16) * kTile17 + (i % 16) * 17 + j % 16];
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// ---------------------------------------------------------------------------
void launch_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s) {
  if (pc.count == 0) return;
  if (H.deg == 3) return q3_patch_setup(H, l, pc, s);
  if (H.dim == 3 && pc.n == kP81) {
    hipLaunchKernelGGL(k_patch_setup81, dim3(pc.count), dim3(256), 0, s, l.g, l.mu, l.cw, l.winv, H.gamma,
                       pc.verts, pc.count, pc.inv, H.flag);
    return;
  }
  const size_t shm = (size_t)(pc.n * (pc.n + 1) + pc.n) * sizeof(double);
  const int nt = pc.n > 32 ? 256 : 64;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_patch_setup<2>, dim3(pc.count), dim3(nt), shm, s, l.g, l.mu, l.cw, l.winv, H.gamma, pc.n, pc.verts,
                       pc.count, pc.inv, H.flag);
  else
    hipLaunchKernelGGL(k_patch_setup<3>, dim3(pc.count), dim3(nt), shm, s, l.g, l.mu, l.cw, l.winv, H.gamma, pc.n, pc.verts,
                       pc.count, pc.inv, H.flag);
}

}  // namespace stk
