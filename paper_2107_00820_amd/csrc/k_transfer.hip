// Standard Q2 prolongation P_H between nested levels and its transpose
// (Section 4.2: V_H is contained in V_h, so P_H evaluates the coarse field at
// the fine nodes). Per axis a fine node i lies in coarse cell floor(i/4) at
// offset r = i mod 4 quarters; the 1D weights l_a(r/4) are exact binary
// fractions (1, 3/8, 3/4, -1/8, ...), so P_H itself introduces no rounding
// beyond the sums. Both are node-parallel gathers (no atomics); the transpose
// runs one axis at a time.
#include <type_traits>

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
  // all (up to 3^d) loads issued together, then summed in the fixed order
  // (a2, a1, a0 ascending, zero weights and coarse Dirichlet nodes skipped)
  constexpr int NA2 = D == 3 ? 3 : 1, NT = NA2 * 9;
  R v[NT];
  double wt[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int a0 = t % 3, a1 = (t / 3) % 3, a2 = t / 9;
    const double w2 = D == 3 ? kProlW[r[2]][a2] : 1.0;
    const double w1 = kProlW[r[1]][a1], w0 = kProlW[r[0]][a0];
    const int j0 = 2 * cell[0] + a0, j1 = 2 * cell[1] + a1, j2 = D == 3 ? 2 * cell[2] + a2 : 0;
    bool ok = w0 != 0.0 && w1 != 0.0 && w2 != 0.0 && j0 != 0 && j0 != 2 * gc.N && j1 != 0 && j1 != 2 * gc.N;
    if (D == 3) ok = ok && j2 != 0 && j2 != 2 * gc.N;
    wt[t] = ok ? w0 * w1 * w2 : 0.0;
    v[t] = ok ? xc[comp * gc.nnodes + node_index<D>(gc, j0, j1, j2)] : (R)0;
  }
  R s = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (wt[t] != 0.0) s += (R)wt[t] * v[t];
  xf[idx] = s;
}

// Transpose: coarse node j collects from the fine nodes where its basis
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

// P_H^T as d one-dimensional passes (the weights are a tensor product): pass
// AX maps extents (.., n1f along AX, ..) to (.., n1c along AX, ..) with the
// axes before AX already coarse. Each output gathers the <= 5 nonzero fine
// weights of its coarse node along AX; fine nodes on the Dirichlet boundary of
// that axis are skipped, so that over all passes a fine node contributes only
// if it is interior (the same set as the direct d-dimensional sum). The last
// pass writes 0 on coarse Dirichlet nodes. Layout: component-major, x fastest.
template <int D, int AX, class R>
__global__ void k_restrict_pass(LevelGeo gf, LevelGeo gc, const R* __restrict__ in, R* __restrict__ out) {
  const int nf = gf.n1, nc = gc.n1;
  int eo[3], ei[3];   // output and input extents per axis
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    eo[k] = k >= D ? 1 : (k <= AX ? nc : nf);
    ei[k] = k >= D ? 1 : (k < AX ? nc : nf);
  }
  const int64_t per = (int64_t)eo[0] * eo[1] * eo[2];
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * per) return;
  const int comp = (int)(idx / per);
  const int64_t r = idx - (int64_t)comp * per;
  int o[3];
  o[0] = (int)(r % eo[0]);
  o[1] = (int)((r / eo[0]) % eo[1]);
  o[2] = (int)(r / ((int64_t)eo[0] * eo[1]));
  if (AX == D - 1) {
    bool bnd = false;
#pragma unroll
    for (int k = 0; k < D; ++k) bnd = bnd || o[k] == 0 || o[k] == 2 * gc.N;
    if (bnd) {
      out[idx] = (R)0;
      return;
    }
  }
  int fn[7] = {};
  double fw[7] = {};
  const int cnt = fine_support(o[AX], gc.N, fn, fw);
  const int64_t stride = AX == 0 ? 1 : (AX == 1 ? (int64_t)ei[0] : (int64_t)ei[0] * ei[1]);
  int base3[3] = {o[0], o[1], o[2]};
  base3[AX] = 0;
  const int64_t base = (int64_t)comp * ei[0] * ei[1] * ei[2] + base3[0] +
                       (int64_t)ei[0] * (base3[1] + (int64_t)ei[1] * base3[2]);
  // all (up to 7) loads issued together, then summed in support order
  R v[7];
  bool ok[7];
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int i = t < cnt ? fn[t] : 0;
    ok[t] = t < cnt && i != 0 && i != 2 * gf.N;
    v[t] = ok[t] ? in[base + stride * i] : (R)0;
  }
  R s = 0;
#pragma unroll
  for (int t = 0; t < 7; ++t)
    if (ok[t]) s += (R)fw[t] * v[t];
  out[idx] = s;
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class R>
void launch_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const R* xc, R* xf, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_prolong_std(H, coarse, fine, xc, xf, s);
  }
  const int64_t n = (int64_t)H.dim * fine.g.nnodes;
  if (H.dim == 2)
    hipLaunchKernelGGL((k_prolong_std<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
  else
    hipLaunchKernelGGL((k_prolong_std<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
}

// The intermediate passes go through the fine level's T buffer (nvel
// entries; the pass outputs need at most 3/4 of it), which is free while a
// restriction runs: the V-cycle writes it only for the prolongation after the
// coarse correction.
template <class R>
void launch_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const R* rf, R* rc, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_restrict_std(H, fine, coarse, rf, rc, s);
  }
  const int64_t nf = fine.g.n1, nc = coarse.g.n1;
  R* t1 = reinterpret_cast<R*>(fine.T);
  if (H.dim == 2) {
    const int64_t n1 = 2 * nf * nc, n2 = 2 * nc * nc;
    hipLaunchKernelGGL((k_restrict_pass<2, 0, R>), dim3(nblk(n1, 256)), dim3(256), 0, s, fine.g, coarse.g, rf, t1);
    hipLaunchKernelGGL((k_restrict_pass<2, 1, R>), dim3(nblk(n2, 256)), dim3(256), 0, s, fine.g, coarse.g,
                       (const R*)t1, rc);
  } else {
    const int64_t n1 = 3 * nf * nf * nc, n2 = 3 * nf * nc * nc, n3 = 3 * nc * nc * nc;
    R* t2 = t1 + n1;
    hipLaunchKernelGGL((k_restrict_pass<3, 0, R>), dim3(nblk(n1, 256)), dim3(256), 0, s, fine.g, coarse.g, rf, t1);
    hipLaunchKernelGGL((k_restrict_pass<3, 1, R>), dim3(nblk(n2, 256)), dim3(256), 0, s, fine.g, coarse.g,
                       (const R*)t1, t2);
    hipLaunchKernelGGL((k_restrict_pass<3, 2, R>), dim3(nblk(n3, 256)), dim3(256), 0, s, fine.g, coarse.g,
                       (const R*)t2, rc);
  }
}

template void launch_prolong_std<double>(const Hier&, const Level&, const Level&, const double*, double*, hipStream_t);
template void launch_prolong_std<float>(const Hier&, const Level&, const Level&, const float*, float*, hipStream_t);
template void launch_restrict_std<double>(const Hier&, const Level&, const Level&, const double*, double*,
                                          hipStream_t);
template void launch_restrict_std<float>(const Hier&, const Level&, const Level&, const float*, float*, hipStream_t);

}  // namespace stk
