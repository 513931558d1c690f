// Standard Q2 prolongation P_H between nested levels and its transpose
// (Section 4.2: V_H is contained in V_h, so P_H evaluates the coarse field at
// the fine nodes). Per axis a fine node i lies in coarse cell floor(i/4) at
// offset r = i mod 4 quarters; the 1D weights l_a(r/4) are exact binary
// fractions (1, 3/8, 3/4, -1/8, ...), so P_H itself introduces no rounding
// beyond the sums. Both are gathers (no atomics): the prolongation writes
// four fine nodes of a row per thread, the transpose runs one axis at a time.
#include <type_traits>

#include "stk_internal.h"

namespace stk {

// 1D weight l_a(r/4) for a lane-dependent quarter offset r and a compile-time
// a, chosen among constants (no table read with a lane-dependent index).
template <int A>
__device__ inline double prol_w(int r) {
  return r == 0 ? kProlW[0][A] : (r == 1 ? kProlW[1][A] : (r == 2 ? kProlW[2][A] : (r == 3 ? kProlW[3][A] : kProlW[4][A])));
}

// P_H x_c, four fine nodes per thread: the nodes 4c .. 4c+3 of one fine row
// (i1, i2) along x, which lie in coarse cell c at the quarter offsets 0..3
// (thread c = N_c owns the last node 4 N_c, a Dirichlet node). The coarse
// values of the row's (y, z) stencil (at most 3 x 3 entries, the same for all
// four nodes) are summed per coarse x-node first, then each output takes its
// x weights, compile-time constants. Coarse Dirichlet nodes contribute
// nothing; fine Dirichlet nodes are written as 0.
template <int D, class R>
__global__ void k_prolong_std(LevelGeo gc, LevelGeo gf, const R* __restrict__ xc, R* __restrict__ xf) {
  const int Nc = gc.N, nf1 = gf.n1;
  const int64_t nc1 = gc.n1;
  const int64_t nrow = D == 3 ? (int64_t)nf1 * nf1 : (int64_t)nf1;
  const int64_t per = nrow * (Nc + 1);
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * per) return;
  const int comp = (int)(idx / per);
  const int64_t rem = idx - (int64_t)comp * per;
  const int c = (int)(rem % (Nc + 1));
  const int64_t row = rem / (Nc + 1);
  const int i1 = (int)(row % nf1), i2 = D == 3 ? (int)(row / nf1) : 0;
  R* out = xf + (int64_t)comp * gf.nnodes + (int64_t)nf1 * (i1 + (int64_t)nf1 * i2) + 4 * c;
  const bool bndrow = i1 == 0 || i1 == 2 * gf.N || (D == 3 && (i2 == 0 || i2 == 2 * gf.N));
  if (c == Nc || bndrow) {
    const int nout = c == Nc ? 1 : 4;
    for (int k = 0; k < nout; ++k) out[k] = (R)0;
    return;
  }
  int cl1 = i1 >> 2, r1 = i1 & 3;
  if (cl1 == Nc) { cl1 = Nc - 1; r1 = 4; }
  int cl2 = D == 3 ? i2 >> 2 : 0, r2 = D == 3 ? i2 & 3 : 0;
  if (D == 3 && cl2 == Nc) { cl2 = Nc - 1; r2 = 4; }
  const double w1[3] = {prol_w<0>(r1), prol_w<1>(r1), prol_w<2>(r1)};
  const double w2[3] = {D == 3 ? prol_w<0>(r2) : 1.0, prol_w<1>(r2), prol_w<2>(r2)};
  // (y, z)-weighted coarse values at the cell's x-nodes 2c, 2c+1, 2c+2
  R t[3] = {(R)0, (R)0, (R)0};
  const R* src0 = xc + (int64_t)comp * gc.nnodes + 2 * c;
#pragma unroll
  for (int a2 = 0; a2 < (D == 3 ? 3 : 1); ++a2) {
    const int j2 = 2 * cl2 + a2;
    if (D == 3 && (w2[a2] == 0.0 || j2 == 0 || j2 == 2 * Nc)) continue;
#pragma unroll
    for (int a1 = 0; a1 < 3; ++a1) {
      const int j1 = 2 * cl1 + a1;
      if (w1[a1] == 0.0 || j1 == 0 || j1 == 2 * Nc) continue;
      const R w = (R)(w1[a1] * w2[a2]);
      const R* src = src0 + nc1 * (j1 + nc1 * j2);
      const R v0 = c > 0 ? src[0] : (R)0;             // x-node 2c is Dirichlet for c = 0
      const R v1 = src[1];
      const R v2 = c < Nc - 1 ? src[2] : (R)0;        // x-node 2c+2 is Dirichlet for c = Nc - 1
      t[0] += w * v0;
      t[1] += w * v1;
      t[2] += w * v2;
    }
  }
#pragma unroll
  for (int r0 = 0; r0 < 4; ++r0) {
    R y = (R)0;
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0)
      if (kProlW[r0][a0] != 0.0) y += (R)kProlW[r0][a0] * t[a0];
    out[r0] = (c == 0 && r0 == 0) ? (R)0 : y;          // fine node 0 is Dirichlet
  }
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
  // threads: components x fine rows x (coarse cells along x + 1)
  const int64_t nf1 = fine.g.n1, per_row = coarse.g.N + 1;
  if (H.dim == 2) {
    const int64_t n = 2 * nf1 * per_row;
    hipLaunchKernelGGL((k_prolong_std<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
  } else {
    const int64_t n = 3 * nf1 * nf1 * per_row;
    hipLaunchKernelGGL((k_prolong_std<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, coarse.g, fine.g, xc, xf);
  }
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
