// Standard Q2 prolongation P_H between nested levels and its transpose
// (Section 4.2: V_H is contained in V_h, so P_H evaluates the coarse field at
// the fine nodes). Per axis a fine node i lies in coarse cell floor(i/4) at
// offset r = i mod 4 quarters; the 1D weights l_a(r/4) are exact binary
// fractions (1, 3/8, 3/4, -1/8, ...), so P_H itself introduces no rounding
// beyond the sums. Both kernels are node-parallel gathers (no atomics).
#include "stk_internal.h"

namespace stk {

template <int D, class R>
__global__ void k_prolong_std(LevelGeo gc, LevelGeo gf, const R* __restrict__ xc, R* __restrict__ xf) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * gf.nnodes) return;
  const int comp = (int)(idx / gf.nnodes);
  const int64_t nd = idx - (int64_t)comp * gf.nnodes;
  int i[3];
  i[0] = (int)(nd % gf.n1);
  i[1] = (int)((nd / gf.n1) % gf.n1);
  i[2] = D == 3 ? (int)(nd / ((int64_t)gf.n1 * gf.n1)) : 0;
  bool bnd = false;
#pragma unroll
  for (int k = 0; k < D; ++k) bnd = bnd || i[k] == 0 || i[k] == 2 * gf.N;
  if (bnd) {
    xf[idx] = (R)0;
    return;
  }
  int cell[3], r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { cell[k] = 0; r[k] = 0; continue; }
    cell[k] = i[k] >> 2;
    r[k] = i[k] & 3;
    if (cell[k] == gc.N) { cell[k] = gc.N - 1; r[k] = 4; }
  }
  R s = 0;
  for (int a2 = 0; a2 < (D == 3 ? 3 : 1); ++a2) {
    const double w2 = D == 3 ? kProlW[r[2]][a2] : 1.0;
    if (w2 == 0.0) continue;
    const int j2 = 2 * cell[2] + a2;
    if (D == 3 && (j2 == 0 || j2 == 2 * gc.N)) continue;
    for (int a1 = 0; a1 < 3; ++a1) {
      const double w1 = kProlW[r[1]][a1];
      if (w1 == 0.0) continue;
      const int j1 = 2 * cell[1] + a1;
      if (j1 == 0 || j1 == 2 * gc.N) continue;
      for (int a0 = 0; a0 < 3; ++a0) {
        const double w0 = kProlW[r[0]][a0];
        if (w0 == 0.0) continue;
        const int j0 = 2 * cell[0] + a0;
        if (j0 == 0 || j0 == 2 * gc.N) continue;
        s += (R)(w0 * w1 * w2) * xc[comp * gc.nnodes + node_index<D>(gc, j0, j1, j2)];
      }
    }
  }
  xf[idx] = s;
}

// Transpose: coarse node j gathers from the fine nodes where its basis
// function is nonzero. Per axis: j even (= 2C) -> fine 4C + t, t = -3..3 with
// weights l2((4+t)/4) for t < 0 and l0(t/4) for t >= 0; j odd (= 2C+1) ->
// fine 4C + t, t = 1..3 with weights l1(t/4).
__device__ inline int fine_support(int j, int Nc, int nodes[7], double w[7]) {
  int n = 0;
  if ((j & 1) == 0) {
    const int C = j >> 1;
    for (int t = -3; t <= 3; ++t) {
      const double wt = t < 0 ? kProlW[4 + t][2] : kProlW[t][0];
      if (wt == 0.0) continue;
      if (t < 0 && C == 0) continue;
      if (t > 0 && C == Nc) continue;
      nodes[n] = 4 * C + t;
      w[n] = wt;
      ++n;
    }
  } else {
    const int C = j >> 1;
    for (int t = 1; t <= 3; ++t) {
      nodes[n] = 4 * C + t;
      w[n] = kProlW[t][1];
      ++n;
    }
  }
  return n;
}

template <int D, class R>
__global__ void k_restrict_std(LevelGeo gf, LevelGeo gc, const R* __restrict__ rf, R* __restrict__ rc) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * gc.nnodes) return;
  const int comp = (int)(idx / gc.nnodes);
  const int64_t nd = idx - (int64_t)comp * gc.nnodes;
  int j[3];
  j[0] = (int)(nd % gc.n1);
  j[1] = (int)((nd / gc.n1) % gc.n1);
  j[2] = D == 3 ? (int)(nd / ((int64_t)gc.n1 * gc.n1)) : 0;
  bool bnd = false;
#pragma unroll
  for (int k = 0; k < D; ++k) bnd = bnd || j[k] == 0 || j[k] == 2 * gc.N;
  if (bnd) {
    rc[idx] = (R)0;
    return;
  }
  int fn[3][7], cnt[3];
  double fw[3][7];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { cnt[k] = 1; fn[k][0] = 0; fw[k][0] = 1.0; continue; }
    cnt[k] = fine_support(j[k], gc.N, fn[k], fw[k]);
  }
  R s = 0;
  for (int t2 = 0; t2 < cnt[2]; ++t2) {
    const int i2 = fn[2][t2];
    if (D == 3 && (i2 == 0 || i2 == 2 * gf.N)) continue;
    for (int t1 = 0; t1 < cnt[1]; ++t1) {
      const int i1 = fn[1][t1];
      if (i1 == 0 || i1 == 2 * gf.N) continue;
      for (int t0 = 0; t0 < cnt[0]; ++t0) {
        const int i0 = fn[0][t0];
        if (i0 == 0 || i0 == 2 * gf.N) continue;
        s += (R)(fw[0][t0] * fw[1][t1] * fw[2][t2]) * rf[comp * gf.nnodes + node_index<D>(gf, i0, i1, i2)];
      }
    }
  }
  rc[idx] = s;
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class R>
void launch_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const R* xc, R* xf, hipStream_t s) {
  const int64_t n = (int64_t)H.dim * fine.g.nnodes;
  if (H.dim == 2)
    hipLaunchKernelGGL((k_prolong_std<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
  else
    hipLaunchKernelGGL((k_prolong_std<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
}

template <class R>
void launch_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const R* rf, R* rc, hipStream_t s) {
  const int64_t n = (int64_t)H.dim * coarse.g.nnodes;
  if (H.dim == 2)
    hipLaunchKernelGGL((k_restrict_std<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, fine.g, coarse.g, rf, rc);
  else
    hipLaunchKernelGGL((k_restrict_std<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, fine.g, coarse.g, rf, rc);
}

template void launch_prolong_std<double>(const Hier&, const Level&, const Level&, const double*, double*, hipStream_t);
template void launch_prolong_std<float>(const Hier&, const Level&, const Level&, const float*, float*, hipStream_t);
template void launch_restrict_std<double>(const Hier&, const Level&, const Level&, const double*, double*,
                                          hipStream_t);
template void launch_restrict_std<float>(const Hier&, const Level&, const Level&, const float*, float*, hipStream_t);

}  // namespace stk
