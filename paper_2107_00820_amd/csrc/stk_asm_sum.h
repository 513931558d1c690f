// Device helper shared by the patch-output gather and the 2D cell kernel
// that consumes the patch outputs directly (vertex-star additive Schwarz
// smoother, Section 4.1: the preconditioned vector is the sum over patches
// of the prolongated local solutions).
#pragma once
#include "stk_internal.h"

namespace stk {

// Sum of the patch-solve outputs at an interior node i[] (component comp):
// the <= 2^d star patches containing the node, in a fixed order (vertex
// offsets x fastest), all loads issued before the first add. zbuf is the
// vertex-indexed output buffer [comp * 3^d + local node][vertex].
template <int D, class R>
__device__ inline R asm_node_sum(const LevelGeo& g, const R* __restrict__ zbuf, int nvert, int comp,
                                 const int i[3]) {
  constexpr int NN = Dims<D>::NN;
  // per axis up to two (vertex, local) pairs; an absent second pair repeats
  // the first so that every address below is valid
  int vv[3][2], ll[3][2], cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { cnt[k] = 1; vv[k][0] = vv[k][1] = 0; ll[k][0] = ll[k][1] = 0; continue; }
    if (i[k] & 1) {
      cnt[k] = 2; vv[k][0] = (i[k] - 1) >> 1; ll[k][0] = 2; vv[k][1] = (i[k] + 1) >> 1; ll[k][1] = 0;
    } else {
      cnt[k] = 1; vv[k][0] = vv[k][1] = i[k] >> 1; ll[k][0] = ll[k][1] = 1;
    }
  }
  const int nv = g.N + 1;
  constexpr int NT = D == 3 ? 8 : 4;
  R v[NT];
  bool ok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int t0 = t & 1, t1 = (t >> 1) & 1, t2 = t >> 2;
    ok[t] = t0 < cnt[0] && t1 < cnt[1] && t2 < cnt[2];
    const int vert = vv[0][t0] + nv * (vv[1][t1] + nv * vv[2][t2]);
    const int loc = ll[0][t0] + 3 * ll[1][t1] + 9 * ll[2][t2];
    v[t] = ok[t] ? zbuf[(int64_t)(comp * NN + loc) * nvert + vert] : (R)0;
  }
  R s = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (ok[t]) s += v[t];
  return s;
}

}  // namespace stk
