// Vertex-star additive Schwarz (Section 4.1, eq. (viim)): patch setup,
// the batched patch solve and the deterministic overlap sum; plus the local
// solves of the robust prolongation (Section 4.2, eq. (Ptilde)), which reuse
// the factors of the star patches centred in the coarse cells.
//
// Patch of vertex v: the unknowns at the nodes strictly inside the cells
// around v, i.e. per axis the nodes 2v-1, 2v, 2v+1 that are interior to the
// domain (one node for a vertex on the boundary), all components.
// Unknown order inside a patch: component-major, then nodes x-fastest.
//
// Setup (one workgroup per patch): the patch matrix is assembled from
// Gauss-point integrals of the cells of the star (equal to the rows and
// columns of the assembled A_gamma), factored A = L L^T in LDS, inverted
// (L^{-1}, then L^{-T} L^{-1}) and stored as a packed lower triangle. Patches
// of one class are interleaved in blocks of 64: element k of patch s sits at
// ((s/64)*P + k)*64 + s%64 (P = n(n+1)/2), so a wavefront processing 64
// patches reads 512 contiguous bytes per element.
//
// Apply (one lane per patch): gather the patch residual, symmetric GEMV from
// the packed inverse, write the result into a vertex-indexed buffer; a node
// kernel then sums the <= 2^d overlapping patch results in a fixed order.
#include <utility>

#include "stk_dev.h"

namespace stk {

template <class F, int... I>
__device__ __attribute__((always_inline)) inline void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, i>) for i = 0..N-1, expanded at compile time.
template <int N, class F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

// ---------------------------------------------------------------------------
// y = A^{-1} x with A^{-1} packed lower, element stride 64.
// Packed symmetric GEMV y = A x over one patch, A's element k at A[k*64]
// (lower triangle, row major). The element order is expanded at compile time
// so that every index into x and y is a constant and both stay in registers.
// Row index of packed lower-triangle element e (largest i with i(i+1)/2 <= e).
constexpr int tri_row(int e) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  return i;
}

// x staged in LDS (column `lane` of xs[NPT][64]); used for the 81-unknown 3D
// patches, where x and y together would not fit the register file. Each lane
// reads only its own column, so no barrier is needed. The 3321 packed
// elements stream in chunks of CH with the next chunk's loads issued before
// the current chunk's arithmetic (scheduling barriers keep the compiler from
// hoisting all loads at once, which would spill).
template <int NPT, int CH, int C, class X, class R>
__device__ __attribute__((always_inline)) inline void symv_chunk_load(const R* __restrict__ A, R (&buf)[CH]) {
  constexpr int NE = NPT * (NPT + 1) / 2;
  static_for<CH>([&](auto T) {
    constexpr int e = C * CH + T;
    if constexpr (e < NE) buf[T] = A[(int64_t)e * 64];
  });
}

template <int NPT, int CH, int C, class X, class R>
__device__ __attribute__((always_inline)) inline void symv_chunk_fma(const X& x, const R (&buf)[CH], R (&y)[NPT]) {
  constexpr int NE = NPT * (NPT + 1) / 2;
  static_for<CH>([&](auto T) {
    constexpr int e = C * CH + T;
    if constexpr (e < NE) {
      constexpr int i = tri_row(e);
      constexpr int j = e - i * (i + 1) / 2;
      if constexpr (j != i) {
        y[i] += buf[T] * x(j);
        y[j] += buf[T] * x(i);
      } else {
        y[i] += buf[T] * x(i);
      }
    }
  });
}

template <int NPT, int CH, class X, class R>
__device__ __attribute__((always_inline)) inline void packed_symv_chunked(const R* __restrict__ A, const X& xr,
                                                                          R (&y)[NPT]) {
  constexpr int NE = NPT * (NPT + 1) / 2;
  constexpr int NC = (NE + CH - 1) / CH;
#pragma unroll
  for (int i = 0; i < NPT; ++i) y[i] = (R)0;
  R b0[CH], b1[CH];
  symv_chunk_load<NPT, CH, 0, X>(A, b0);
  static_for<NC>([&](auto C) {
    constexpr int c = C;
    if constexpr (c + 1 < NC) {
      if constexpr ((c & 1) == 0) symv_chunk_load<NPT, CH, c + 1, X>(A, b1);
      else symv_chunk_load<NPT, CH, c + 1, X>(A, b0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr ((c & 1) == 0) symv_chunk_fma<NPT, CH, c>(xr, b0, y);
    else symv_chunk_fma<NPT, CH, c>(xr, b1, y);
    __builtin_amdgcn_sched_barrier(0);
  });
}

#ifndef STK_CH_LDS64
#define STK_CH_LDS64 16
#endif
#ifndef STK_CH_LDS32
#define STK_CH_LDS32 32
#endif
template <int NPT, class R>
__device__ __attribute__((always_inline)) inline void packed_symv_lds(const R* __restrict__ A, const R* xs, int lane,
                                                                      R (&y)[NPT]) {
  auto xr = [&](int j) { return xs[j * 64 + lane]; };
  packed_symv_chunked<NPT, sizeof(R) == 8 ? STK_CH_LDS64 : STK_CH_LDS32>(A, xr, y);
}

// x from registers (patches of up to 27 unknowns): four double-buffered chunks
template <int NPT, class R>
__device__ __attribute__((always_inline)) inline void packed_symv(const R* __restrict__ A, const R (&x)[NPT],
                                                                  R (&y)[NPT]) {
  auto xr = [&](int j) { return x[j]; };
  constexpr int NE = NPT * (NPT + 1) / 2;
  constexpr int CH = NPT <= 18 ? (NE + 3) / 4 : 24;
  packed_symv_chunked<NPT, CH>(A, xr, y);
}

// One lane per patch: gather the patch residual, packed symmetric GEMV,
// write the result into the vertex-indexed buffer.
template <int D, int NPT, class R>
__device__ __attribute__((always_inline)) inline void asm_patch(const LevelGeo& g, const int* __restrict__ verts, int count,
                                 const R* __restrict__ inv, const R* __restrict__ r,
                                 R* __restrict__ zbuf, int nvert, int s) {
  constexpr int NN = Dims<D>::NN;
  constexpr int NBOX = NPT / D;
  constexpr bool FULL = NBOX == NN;
  if (s >= count) return;
  const int vert = verts[s];
  int lo[3], ext[3], vc[3];
  patch_box<D>(g, vert, lo, ext, vc);
  if (FULL) { ext[0] = 3; ext[1] = 3; ext[2] = D == 3 ? 3 : 1; }
  R x[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    int nd[3];
    const int comp = patch_dof<D>(i, lo, ext, nd);
    x[i] = r[comp * g.nnodes + node_index<D>(g, nd[0], nd[1], nd[2])];
  }
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)(s / 64) * P) * 64 + (s % 64);
  R y[NPT];
  packed_symv<NPT>(A, x, y);
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    int nd[3];
    const int comp = patch_dof<D>(i, lo, ext, nd);
    int loc = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      loc += (nd[k] - (2 * vc[k] - 1)) * mul;
      mul *= 3;
    }
    zbuf[(int64_t)(comp * NN + loc) * nvert + vert] = y[i];
  }
}

// Interior (full) patch with x staged in LDS; all unknown indices are
// compile-time: unknown i = comp*3^d + a + 3b + 9c sits at node 2v-1 + (a,b,c).
template <int D, int NPT, class R>
__device__ __attribute__((always_inline)) inline void asm_patch_lds(const LevelGeo& g, const int* __restrict__ verts, int count,
                                     const R* __restrict__ inv, const R* __restrict__ r,
                                     R* __restrict__ zbuf, int nvert, int s, R* xs, int lane) {
  constexpr int NN = Dims<D>::NN;
  if (s >= count) return;
  const int vert = verts[s];
  int lo[3], ext[3], vc[3];
  patch_box<D>(g, vert, lo, ext, vc);
  const int64_t base = node_index<D>(g, lo[0], lo[1], lo[2]);
  const int64_t n1 = g.n1;
  static_for<NPT>([&](auto I) {
    constexpr int i = I;
    constexpr int comp = i / NN, loc = i % NN;
    xs[i * 64 + lane] = r[comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * digit(loc, 2))];
  });
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)(s / 64) * P) * 64 + (s % 64);
  R y[NPT];
  packed_symv_lds<NPT>(A, xs, lane, y);
  static_for<NPT>([&](auto I) {
    constexpr int i = I;
    zbuf[(int64_t)i * nvert + vert] = y[i];
  });
}

// All patch classes of a level in one launch: block ranges select the class
// (sizes d*3^d, d*3^(d-1), .., d; interior patches first).
template <class R>
struct AsmClasses {
  const int* verts[4];
  const R* inv[4];
  int count[4];
  int first_block[5];
};

template <int D, class R>
__global__ void __launch_bounds__(64) k_asm_gemv(LevelGeo g, AsmClasses<R> c, const R* __restrict__ r,
                                                  R* __restrict__ zbuf, int nvert) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  if (b < c.first_block[1]) {
    if (D == 2) {
      asm_patch<D, 18>(g, c.verts[0], c.count[0], c.inv[0], r, zbuf, nvert, b * 64 + lane);
    } else {
      __shared__ R xs[81 * 64];
      asm_patch_lds<D, 81>(g, c.verts[0], c.count[0], c.inv[0], r, zbuf, nvert, b * 64 + lane, xs, lane);
    }
  } else if (b < c.first_block[2]) {
    const int s = (b - c.first_block[1]) * 64 + lane;
    asm_patch<D, D == 2 ? 6 : 27>(g, c.verts[1], c.count[1], c.inv[1], r, zbuf, nvert, s);
  } else if (b < c.first_block[3]) {
    const int s = (b - c.first_block[2]) * 64 + lane;
    asm_patch<D, D == 2 ? 2 : 9>(g, c.verts[2], c.count[2], c.inv[2], r, zbuf, nvert, s);
  } else if (D == 3 && b < c.first_block[4]) {
    const int s = (b - c.first_block[3]) * 64 + lane;
    asm_patch<D, 3>(g, c.verts[3], c.count[3], c.inv[3], r, zbuf, nvert, s);
  }
}

// y[idx] = sum over the patches containing the node of their results; 0 on Dirichlet nodes.
template <int D, class R>
__global__ void k_asm_gather(LevelGeo g, const R* __restrict__ zbuf, int nvert, R* __restrict__ y) {
  constexpr int NN = Dims<D>::NN;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)D * g.nnodes) return;
  const int comp = (int)(idx / g.nnodes);
  const int64_t nd = idx - (int64_t)comp * g.nnodes;
  int i[3];
  i[0] = (int)(nd % g.n1);
  i[1] = (int)((nd / g.n1) % g.n1);
  i[2] = D == 3 ? (int)(nd / ((int64_t)g.n1 * g.n1)) : 0;
  bool bnd = false;
#pragma unroll
  for (int k = 0; k < D; ++k) bnd = bnd || i[k] == 0 || i[k] == 2 * g.N;
  if (bnd) {
    y[idx] = (R)0;
    return;
  }
  int vv[3][2], ll[3][2], cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= D) { cnt[k] = 1; vv[k][0] = 0; ll[k][0] = 0; continue; }
    if (i[k] & 1) {
      cnt[k] = 2; vv[k][0] = (i[k] - 1) >> 1; ll[k][0] = 2; vv[k][1] = (i[k] + 1) >> 1; ll[k][1] = 0;
    } else {
      cnt[k] = 1; vv[k][0] = i[k] >> 1; ll[k][0] = 1;
    }
  }
  const int nv = g.N + 1;
  R s = 0;
  for (int t2 = 0; t2 < cnt[2]; ++t2)
    for (int t1 = 0; t1 < cnt[1]; ++t1)
      for (int t0 = 0; t0 < cnt[0]; ++t0) {
        const int vert = vv[0][t0] + nv * (vv[1][t1] + nv * vv[2][t2]);
        const int loc = ll[0][t0] + 3 * ll[1][t1] + 9 * ll[2][t2];
        s += zbuf[(int64_t)(comp * NN + loc) * nvert + vert];
      }
  y[idx] = s;
}

// Local solves of the robust transfer: for every coarse cell K (one lane),
// z = A_K^{-1} in|_K where A_K is the star patch of the fine vertex 2K+1
// (interior-patch slot lex(K)); out|_K = (accumulate ? out|_K : 0) + alpha z.
template <int D, bool ACC, class R>
__global__ void __launch_bounds__(64) k_center_solve(LevelGeo g, const R* __restrict__ inv,
                                                      const R* __restrict__ in, R* __restrict__ out,
                                                      double alpha_d) {
  const R alpha = (R)alpha_d;
  constexpr int NN = Dims<D>::NN, NPT = Dims<D>::NL;
  const int nc = g.N / 2;
  const int ncc = D == 2 ? nc * nc : nc * nc * nc;
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= ncc) return;
  const int K0 = s % nc, K1 = (s / nc) % nc, K2 = D == 3 ? s / (nc * nc) : 0;
  const int64_t base = node_index<D>(g, 4 * K0 + 1, 4 * K1 + 1, D == 3 ? 4 * K2 + 1 : 0);
  const int64_t n1 = g.n1;
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)(s / 64) * P) * 64 + (s % 64);
  R y[NPT];
  if constexpr (D == 2) {
    R x[NPT];
    static_for<NPT>([&](auto I) {
      constexpr int i = I;
      constexpr int comp = i / NN, loc = i % NN;
      x[i] = in[comp * g.nnodes + base + digit(loc, 0) + n1 * digit(loc, 1)];
    });
    packed_symv<NPT>(A, x, y);
  } else {
    __shared__ R xs[NPT * 64];
    const int lane = threadIdx.x;
    static_for<NPT>([&](auto I) {
      constexpr int i = I;
      constexpr int comp = i / NN, loc = i % NN;
      xs[i * 64 + lane] = in[comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * digit(loc, 2))];
    });
    packed_symv_lds<NPT>(A, xs, lane, y);
  }
  static_for<NPT>([&](auto I) {
    constexpr int i = I;
    constexpr int comp = i / NN, loc = i % NN;
    const int64_t o = comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * (D == 3 ? digit(loc, 2) : 0));
    if constexpr (ACC) out[o] += alpha * y[i];
    else out[o] = alpha * y[i];
  });
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s) {
  if (pc.count == 0) return;
  const size_t shm = (size_t)(pc.n * (pc.n + 1) + pc.n) * sizeof(double);
  const int nt = pc.n > 32 ? 256 : 64;
  if (H.dim == 2)
    hipLaunchKernelGGL(k_patch_setup<2>, dim3(pc.count), dim3(nt), shm, s, l.g, l.mu, l.cw, l.winv, H.gamma, pc.n, pc.verts,
                       pc.count, pc.inv, H.flag);
  else
    hipLaunchKernelGGL(k_patch_setup<3>, dim3(pc.count), dim3(nt), shm, s, l.g, l.mu, l.cw, l.winv, H.gamma, pc.n, pc.verts,
                       pc.count, pc.inv, H.flag);
}

template <class R>
static const R* class_inv(const PatchClass& pc);
template <>
const double* class_inv<double>(const PatchClass& pc) { return pc.inv; }
template <>
const float* class_inv<float>(const PatchClass& pc) { return pc.inv32; }

template <class R>
void launch_asm(Hier& H, const Level& l, const R* r, R* y, hipStream_t s) {
  AsmClasses<R> c{};
  int blocks = 0;
  double bytes = (double)sizeof(R) * (double)l.nvel;   // one read of the residual
  const int ncls = H.dim == 2 ? 3 : 4;
  for (int ci = 0; ci < 4; ++ci) {
    c.first_block[ci] = blocks;
    if (ci < ncls && ci < (int)l.cls.size()) {
      const PatchClass& pc = l.cls[ci];
      c.verts[ci] = pc.verts;
      c.inv[ci] = class_inv<R>(pc);
      c.count[ci] = pc.count;
      blocks += (pc.count + 63) / 64;
      // algorithmic bytes: packed inverse and patch output of every patch
      bytes += (double)sizeof(R) * (double)pc.count * (pc.n * (pc.n + 1) / 2 + pc.n);
    }
  }
  c.first_block[4] = blocks;
  R* zbuf = reinterpret_cast<R*>(l.zbuf);
  hipEvent_t ev = nullptr;
  const int reps = prof_begin(H, s, &ev);
  // the kernel is a pure function of (r, inverses) -> zbuf, so a profiled
  // call may repeat it back to back to time it without launch gaps
  for (int k = 0; k < reps; ++k) {
    if (H.dim == 2)
      hipLaunchKernelGGL((k_asm_gemv<2, R>), dim3(blocks), dim3(64), 0, s, l.g, c, r, zbuf, l.nvert);
    else
      hipLaunchKernelGGL((k_asm_gemv<3, R>), dim3(blocks), dim3(64), 0, s, l.g, c, r, zbuf, l.nvert);
  }
  prof_end(H, s, PROF_ASM_GEMV, ev, bytes, reps);
  const int64_t n = (int64_t)H.dim * l.g.nnodes;
  if (H.dim == 2)
    hipLaunchKernelGGL((k_asm_gather<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
  else
    hipLaunchKernelGGL((k_asm_gather<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
}

template <class R>
void launch_center_solve(const Hier& H, const Level& fine, const R* in, R* out, double alpha, bool accumulate,
                         hipStream_t s) {
  const int nc = fine.g.N / 2;
  const int ncc = H.dim == 2 ? nc * nc : nc * nc * nc;
  const dim3 grid(nblk(ncc, 64)), blk(64);
  const R* inv = class_inv<R>(fine.cls[0]);
  if (H.dim == 2) {
    if (accumulate) hipLaunchKernelGGL((k_center_solve<2, true, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
    else hipLaunchKernelGGL((k_center_solve<2, false, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
  } else {
    if (accumulate) hipLaunchKernelGGL((k_center_solve<3, true, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
    else hipLaunchKernelGGL((k_center_solve<3, false, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
  }
}

template void launch_asm<double>(Hier&, const Level&, const double*, double*, hipStream_t);
template void launch_asm<float>(Hier&, const Level&, const float*, float*, hipStream_t);
template void launch_center_solve<double>(const Hier&, const Level&, const double*, double*, double, bool,
                                          hipStream_t);
template void launch_center_solve<float>(const Hier&, const Level&, const float*, float*, double, bool,
                                         hipStream_t);

}  // namespace stk
