// Vertex-star additive Schwarz (Section 4.1, eq. (viim)): the batched patch
// solve and the deterministic overlap sum; plus the local solves of the
// robust prolongation (Section 4.2, eq. (Ptilde)), which reuse the inverses
// of the star patches centred in the coarse cells. The inverses themselves
// are formed in k_setup.hip.
//
// Patch of vertex v: the unknowns at the nodes strictly inside the cells
// around v, i.e. per axis the nodes 2v-1, 2v, 2v+1 that are interior to the
// domain (one node for a vertex on the boundary), all components.
// Unknown order inside a patch: component-major, then nodes x-fastest.
// Patch inverses are stored as packed lower triangles; patches of one class
// are interleaved in blocks of 64: element k of patch s sits at
// ((s/64)*P + k)*64 + s%64 (P = n(n+1)/2), so a wavefront processing 64
// patches reads 512 contiguous bytes per element.
//
// Apply: gather the patch residual, symmetric GEMV from the packed inverse,
// write the result into a vertex-indexed buffer; a node kernel then sums the
// <= 2^d overlapping patch results in a fixed order. One lane per patch,
// except the 81-unknown 3D interior patches, whose GEMV four wavefronts
// share (split_symv81).
#include <algorithm>
#include <type_traits>
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

// A piece of the packed lower triangle: the elements (i, j), j <= i, with
// row_lo <= i < row_hi and col_lo <= j < col_hi, enumerated row by row. A
// piece is either a triangle (col range = row range) or a block left of the
// diagonal (col_hi <= row_lo). The result rows it touches are kept in ny
// slots: slot(i) = i - row_lo for a triangle; for a block the column rows
// first (i - col_lo), then the rows (col_hi - col_lo + i - row_lo).
template <int RL, int RH, int CL, int CH>
struct TriPiece {
  static_assert((CL == RL && CH == RH) || CH <= RL, "triangle or block below the diagonal");
  static constexpr bool tri = CL == RL && CH == RH;
  static constexpr int ny = tri ? RH - RL : (CH - CL) + (RH - RL);
  static constexpr int slot(int i) { return tri ? i - RL : (i < CH ? i - CL : (CH - CL) + (i - RL)); }
  static constexpr int row_len(int i) {
    const int b = i + 1 < CH ? i + 1 : CH;
    return b > CL ? b - CL : 0;
  }
  static constexpr int count() {
    int n = 0;
    for (int i = RL; i < RH; ++i) n += row_len(i);
    return n;
  }
  // packed index i(i+1)/2 + j of the t-th element
  static constexpr int elem(int t) {
    int i = RL;
    while (t >= row_len(i)) t -= row_len(i++);
    return i * (i + 1) / 2 + CL + t;
  }
};
template <int NPT>
using FullTri = TriPiece<0, NPT, 0, NPT>;

// The elements of the piece stream in chunks of CH with the next chunk's
// loads issued before the current chunk's arithmetic (scheduling barriers
// keep the compiler from hoisting all loads at once, which would spill).
// NT: non-temporal loads (the packed inverses are streamed once per
// application and never reused within it).
template <class PC, int CH, int C, bool NT, class R>
__device__ __attribute__((always_inline)) inline void symv_chunk_load(const R* __restrict__ A, R (&buf)[CH]) {
  static_for<CH>([&](auto T) {
    constexpr int t = C * CH + T;
    if constexpr (t < PC::count()) {
      constexpr int e = PC::elem(t);   // folded at compile time
      if constexpr (NT) buf[T] = __builtin_nontemporal_load(A + (int64_t)e * 64);
      else buf[T] = A[(int64_t)e * 64];
    }
  });
}

template <class PC, int CH, int C, class X, class R>
__device__ __attribute__((always_inline)) inline void symv_chunk_fma(const X& x, const R (&buf)[CH],
                                                                     R (&y)[PC::ny]) {
  static_for<CH>([&](auto T) {
    constexpr int t = C * CH + T;
    if constexpr (t < PC::count()) {
      constexpr int e = PC::elem(t);
      constexpr int i = tri_row(e);
      constexpr int j = e - i * (i + 1) / 2;
      if constexpr (j != i) {
        y[PC::slot(i)] += buf[T] * x(j);
        y[PC::slot(j)] += buf[T] * x(i);
      } else {
        y[PC::slot(i)] += buf[T] * x(i);
      }
    }
  });
}

// y = (piece PC of A) x over the piece's result slots, counting each
// off-diagonal element for both (i, j) and (j, i).
template <int CH, class PC, bool NT = false, class X, class R>
__device__ __attribute__((always_inline)) inline void piece_symv(const R* __restrict__ A, const X& xr,
                                                                 R (&y)[PC::ny]) {
  constexpr int NC = (PC::count() + CH - 1) / CH;
#pragma unroll
  for (int i = 0; i < PC::ny; ++i) y[i] = (R)0;
  R b0[CH], b1[CH];
  symv_chunk_load<PC, CH, 0, NT>(A, b0);
  static_for<NC>([&](auto C) {
    constexpr int c = C;
    if constexpr (c + 1 < NC) {
      if constexpr ((c & 1) == 0) symv_chunk_load<PC, CH, c + 1, NT>(A, b1);
      else symv_chunk_load<PC, CH, c + 1, NT>(A, b0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr ((c & 1) == 0) symv_chunk_fma<PC, CH, c>(xr, b0, y);
    else symv_chunk_fma<PC, CH, c>(xr, b1, y);
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Whole packed triangle: y = A x.
template <int NPT, int CH, bool NT = false, class X, class R>
__device__ __attribute__((always_inline)) inline void packed_symv_chunked(const R* __restrict__ A, const X& xr,
                                                                          R (&y)[NPT]) {
  piece_symv<CH, FullTri<NPT>, NT>(A, xr, y);
}

#ifndef STK_CH_LDS64
#define STK_CH_LDS64 16
#endif
#ifndef STK_CH_LDS32
#define STK_CH_LDS32 32
#endif

// 81-unknown (3D interior) patch solve by the four wavefronts of a 256-thread
// workgroup that share one 64-patch x tile in LDS (xs[81][64], column = lane).
// The 3321 packed elements split into four pieces of 820..861: the leading
// 40x40 triangle (touches y[0,40)), the 41x40 block below it in two column
// halves (y[0,20) + y[40,81), y[20,40) + y[40,81)) and the trailing 41x41
// triangle (y[40,81)). Each wavefront keeps only the rows its piece touches
// (at most 61) and the partial results meet in the x tile once every
// wavefront is done with it, summed in a fixed order:
//   y[0,20) = y0 + y1,  y[20,40) = y0 + y2,  y[40,81) = (y1 + y2) + y3.
// store(integral_constant i, value) receives each final y[i] once.
// Every thread of the workgroup must call this (it holds barriers).
using Q81_0 = TriPiece<0, 40, 0, 40>;    // slots: rows 0..39
using Q81_1 = TriPiece<40, 81, 0, 20>;   // slots: rows 0..19, then 40..80
using Q81_2 = TriPiece<40, 81, 20, 40>;  // slots: rows 20..39, then 40..80
using Q81_3 = TriPiece<40, 81, 40, 81>;  // slots: rows 40..80
static_assert(Q81_0::count() + Q81_1::count() + Q81_2::count() + Q81_3::count() == 81 * 82 / 2, "pieces");
static_assert(Q81_1::ny == 61 && Q81_2::ny == 61, "slots");

template <class PC, int CH, bool NT = false, class X, class R>
__device__ __attribute__((always_inline)) inline void piece_into(const R* __restrict__ A, const X& xr, R (&yc)[61]) {
  R y[PC::ny];
  piece_symv<CH, PC, NT>(A, xr, y);
  static_for<PC::ny>([&](auto I) { yc[I] = y[I]; });
}

template <int CHK, class R, class Store>
__device__ __attribute__((always_inline)) inline void split_symv81(const R* __restrict__ A, R* xs, int lane, int w,
                                                                   Store&& store) {
  auto xr = [&](int j) { return xs[j * 64 + lane]; };
  R yc[61];
  if (w == 0) piece_into<Q81_0, CHK>(A, xr, yc);
  else if (w == 1) piece_into<Q81_1, CHK>(A, xr, yc);
  else if (w == 2) piece_into<Q81_2, CHK>(A, xr, yc);
  else piece_into<Q81_3, CHK>(A, xr, yc);
  __syncthreads();   // every wavefront is done reading x
  if (w == 1) {
    static_for<20>([&](auto I) { xs[I * 64 + lane] = yc[I]; });
    static_for<41>([&](auto I) { xs[(40 + I) * 64 + lane] = yc[20 + I]; });
  } else if (w == 2) {
    static_for<20>([&](auto I) { xs[(20 + I) * 64 + lane] = yc[I]; });
  }
  __syncthreads();
  if (w == 0) {
    static_for<40>([&](auto I) { store(I, yc[I] + xs[I * 64 + lane]); });
  } else if (w == 2) {
    static_for<41>([&](auto I) { xs[(40 + I) * 64 + lane] += yc[20 + I]; });
  }
  __syncthreads();
  if (w == 3) {
    static_for<41>([&](auto I) {
      store(std::integral_constant<int, 40 + I>{}, xs[(40 + I) * 64 + lane] + yc[I]);
    });
  }
}

// split_symv81 with x[0..80) in the LDS tile (80 x 64, exactly a quarter of
// the 160 KB LDS, so four workgroups fit on a compute unit) and x[80] in a
// register of every lane. The partial results meet in the tile as in
// split_symv81, row 80's two partials through tile rows 0 and 1 once the
// first 40 rows are final, with the same additions in the same order:
//   y[0,20) = y0 + y1,  y[20,40) = y0 + y2,  y[40,81) = (y1 + y2) + y3.
template <int CHK, bool NT, class R, class Store>
__device__ __attribute__((always_inline)) inline void split_symv81_t80(const R* __restrict__ A, R* xs, R x80,
                                                                       int lane, int w, Store&& store) {
  auto xr = [&](int j) { return j == 80 ? x80 : xs[j * 64 + lane]; };
  R yc[61];
  if (w == 0) piece_into<Q81_0, CHK, NT>(A, xr, yc);
  else if (w == 1) piece_into<Q81_1, CHK, NT>(A, xr, yc);
  else if (w == 2) piece_into<Q81_2, CHK, NT>(A, xr, yc);
  else piece_into<Q81_3, CHK, NT>(A, xr, yc);
  __syncthreads();   // every wavefront is done reading x
  if (w == 1) {
    static_for<20>([&](auto I) { xs[I * 64 + lane] = yc[I]; });
    static_for<40>([&](auto I) { xs[(40 + I) * 64 + lane] = yc[20 + I]; });
  } else if (w == 2) {
    static_for<20>([&](auto I) { xs[(20 + I) * 64 + lane] = yc[I]; });
  }
  __syncthreads();
  if (w == 0) {
    static_for<40>([&](auto I) { store(I, yc[I] + xs[I * 64 + lane]); });
  } else if (w == 2) {
    static_for<40>([&](auto I) { xs[(40 + I) * 64 + lane] += yc[20 + I]; });
  }
  __syncthreads();   // rows 0..39 are free again
  if (w == 1) xs[lane] = yc[60];
  else if (w == 2) xs[64 + lane] = yc[60];
  __syncthreads();
  if (w == 3) {
    static_for<40>([&](auto I) {
      store(std::integral_constant<int, 40 + I>{}, xs[(40 + I) * 64 + lane] + yc[I]);
    });
    store(std::integral_constant<int, 80>{}, (xs[lane] + xs[64 + lane]) + yc[40]);
  }
}

// x from registers (patches of up to 27 unknowns): double-buffered chunks,
// NCH of them (0: four for up to 18 unknowns, chunks of 12 above)
template <int NPT, int NCH = 0, class R>
__device__ __attribute__((always_inline)) inline void packed_symv(const R* __restrict__ A, const R (&x)[NPT],
                                                                  R (&y)[NPT]) {
  auto xr = [&](int j) { return x[j]; };
  constexpr int NE = NPT * (NPT + 1) / 2;
  constexpr int CH = NCH > 0 ? (NE + NCH - 1) / NCH : (NPT <= 18 ? (NE + 3) / 4 : 12);
  packed_symv_chunked<NPT, CH>(A, xr, y);
}

// Tuning variants of the batched patch solve. They differ only in how many
// packed elements a lane loads ahead (the chunk), which sets the registers a
// lane holds and with them the occupancy, and in the cache policy of those
// loads (variant 3: variant 2's chunks with non-temporal loads); every
// variant performs the same multiply-adds in the same order, so their results
// are bit-identical and a tuner may choose any (kAsmVariants of them).
template <int D, class R, int V>
struct AsmTune {
  // 3D interior patches (81 unknowns, LDS-staged residual): elements per chunk
  static constexpr int ch81 = sizeof(R) == 8 ? (V == 0 ? 16 : (V == 1 ? 24 : 12)) : (V == 0 ? 32 : (V == 1 ? 48 : 24));
  // 2D interior patches (18 unknowns from registers): number of chunks
  static constexpr int nch18 = V == 0 ? 4 : (V == 1 ? 6 : 8);   // variant 3: as variant 2
  // non-temporal loads of the packed inverses (variant 3: otherwise variant 2)
  static constexpr bool nt = V == 3;
  // minimum wavefronts per SIMD requested from the compiler
  static constexpr int min_waves = 2;
};

// One lane per patch: gather the patch residual, packed symmetric GEMV,
// write the result into the vertex-indexed buffer.
template <int D, int NPT, int NCH = 0, class R>
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
  packed_symv<NPT, NCH>(A, x, y);
  // 27-unknown patches: the scatter recomputes its indices rather than
  // keeping the gather's, which would hold 27 index triples in registers
  // across the GEMV and spill (smaller patches keep them)
  if constexpr (NPT == 27) {
#pragma unroll
    for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(lo[k]), "+v"(ext[k]), "+v"(vc[k]));
  }
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

// 3D interior (full) patches, 64 per 256-thread workgroup: the residual
// restricted to each patch is staged in LDS by all four wavefronts, then
// split_symv81 solves. All unknown indices are compile-time: unknown
// i = comp*27 + a + 3b + 9c sits at node 2v-1 + (a,b,c). Lanes past the
// class count take part in the barriers with a clamped vertex and store
// nothing (the inverse storage is padded to whole blocks of 64 patches).
template <int CHK, bool NT, class R>
__device__ __attribute__((always_inline)) inline void asm_patch81(const LevelGeo& g, const int* __restrict__ verts,
                                                                  int count, const R* __restrict__ inv,
                                                                  const R* __restrict__ r, R* __restrict__ zbuf,
                                                                  int nvert, int blk, R* xs, int tid) {
  constexpr int NN = 27, NPT = 81;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int s = blk * 64 + lane;
  const bool valid = s < count;
  const int vert = verts[valid ? s : count - 1];
  int lo[3], ext[3], vc[3];
  patch_box<3>(g, vert, lo, ext, vc);
  const int64_t base = node_index<3>(g, lo[0], lo[1], lo[2]);
  const int64_t n1 = g.n1;
  // rows 0..79 into the tile (round robin over the wavefronts), row 80
  // (component 2, local node 26) into a register of every lane
  static_for<NPT - 1>([&](auto I) {
    constexpr int i = I;
    constexpr int comp = i / NN, loc = i % NN;
    if (w == (i & 3))
      xs[i * 64 + lane] = r[comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * digit(loc, 2))];
  });
  const R x80 = r[2 * g.nnodes + base + 2 + n1 * (2 + n1 * 2)];
  __syncthreads();
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)blk * P) * 64 + lane;
  split_symv81_t80<CHK, NT>(A, xs, x80, lane, w, [&](auto I, R v) {
    if (valid) zbuf[(int64_t)I * nvert + vert] = v;
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

// One launch covers the patch solves of up to kAsmBatchMax entries (a level
// of one hierarchy with its residual and output buffer; the entries may
// belong to different hierarchies, e.g. concurrent requests of a server).
// Workgroups [first[k], first[k+1]) belong to entry k and run exactly the
// code a launch for that entry alone runs, so results do not depend on the
// batch.
template <class R>
struct AsmBatch {
  int n;
  int first[kAsmBatchMax + 1];
  LevelGeo g[kAsmBatchMax];
  AsmClasses<R> c[kAsmBatchMax];
  const R* r[kAsmBatchMax];
  R* zbuf[kAsmBatchMax];
  int nvert[kAsmBatchMax];
};

// Workgroups of 64 threads in 2D (one lane per patch); of 256 in 3D, where
// an interior workgroup covers 64 patches (split_symv81) and a boundary one
// 256 patches (one lane each).
template <int D>
constexpr int asm_threads() { return D == 2 ? 64 : 256; }

template <int D, class R, int V>
__global__ void __launch_bounds__(asm_threads<D>(), (AsmTune<D, R, V>::min_waves))
k_asm_gemv(AsmBatch<R> B) {
  constexpr int NT = asm_threads<D>();
  // the entry of this workgroup (uniform); the fields are picked by
  // compile-time indices so the kernel arguments are never indexed at run time
  const int bid = blockIdx.x;
  int k = 0;
#pragma unroll
  for (int i = 1; i < kAsmBatchMax; ++i)
    if (i < B.n && bid >= B.first[i]) k = i;
  LevelGeo g = B.g[0];
  AsmClasses<R> c = B.c[0];
  const R* r = B.r[0];
  R* zbuf = B.zbuf[0];
  int nvert = B.nvert[0], b0 = 0;
#pragma unroll
  for (int i = 1; i < kAsmBatchMax; ++i)
    if (i == k) {
      g = B.g[i];
      c = B.c[i];
      r = B.r[i];
      zbuf = B.zbuf[i];
      nvert = B.nvert[i];
      b0 = B.first[i];
    }
  const int b = bid - b0;
  const int t = threadIdx.x;
  if (b < c.first_block[1]) {
    if constexpr (D == 2) {
      asm_patch<D, 18, AsmTune<D, R, V>::nch18>(g, c.verts[0], c.count[0], c.inv[0], r, zbuf, nvert, b * 64 + t);
    } else {
      __shared__ R xs[80 * 64];
      asm_patch81<AsmTune<D, R, V>::ch81, AsmTune<D, R, V>::nt>(g, c.verts[0], c.count[0], c.inv[0], r, zbuf,
                                                               nvert, b, xs, t);
    }
  } else if (b < c.first_block[2]) {
    const int s = (b - c.first_block[1]) * NT + t;
    asm_patch<D, D == 2 ? 6 : 27>(g, c.verts[1], c.count[1], c.inv[1], r, zbuf, nvert, s);
  } else if (b < c.first_block[3]) {
    const int s = (b - c.first_block[2]) * NT + t;
    asm_patch<D, D == 2 ? 2 : 9>(g, c.verts[2], c.count[2], c.inv[2], r, zbuf, nvert, s);
  } else if (D == 3 && b < c.first_block[4]) {
    const int s = (b - c.first_block[3]) * NT + t;
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
  y[idx] = asm_node_sum<D, R>(g, zbuf, nvert, comp, i);
}

// Local solves of the robust transfer: for every coarse cell K, z =
// A_K^{-1} in|_K where A_K is the star patch of the fine vertex 2K+1
// (interior-patch slot lex(K)); out|_K = (accumulate ? out|_K : 0) + alpha z.
// 2D: one lane per cell, 64-thread workgroups. 3D: 64 cells per 256-thread
// workgroup through split_symv81; lanes past the cell count take part in
// the barriers with a clamped cell and store nothing.
template <int D>
constexpr int center_threads() { return D == 2 ? 64 : 256; }

template <int D, bool ACC, class R>
__global__ void __launch_bounds__(center_threads<D>()) k_center_solve(LevelGeo g, const R* __restrict__ inv,
                                                                      const R* __restrict__ in, R* __restrict__ out,
                                                                      double alpha_d) {
  const R alpha = (R)alpha_d;
  constexpr int NN = Dims<D>::NN, NPT = Dims<D>::NL;
  const int nc = g.N / 2;
  const int ncc = D == 2 ? nc * nc : nc * nc * nc;
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 64 + lane;
  const bool valid = s < ncc;
  if (D == 2 && !valid) return;
  const int sc = valid ? s : ncc - 1;
  const int K0 = sc % nc, K1 = (sc / nc) % nc, K2 = D == 3 ? sc / (nc * nc) : 0;
  const int64_t base = node_index<D>(g, 4 * K0 + 1, 4 * K1 + 1, D == 3 ? 4 * K2 + 1 : 0);
  const int64_t n1 = g.n1;
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)blockIdx.x * P) * 64 + lane;
  auto offset = [&](auto I) {
    constexpr int i = I;
    constexpr int comp = i / NN, loc = i % NN;
    return comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * (D == 3 ? digit(loc, 2) : 0));
  };
  auto store = [&](auto I, R v) {
    if (!valid) return;
    const int64_t o = offset(I);
    if constexpr (ACC) out[o] += alpha * v;
    else out[o] = alpha * v;
  };
  if constexpr (D == 2) {
    R x[NPT], y[NPT];
    static_for<NPT>([&](auto I) { x[I] = in[offset(I)]; });
    if constexpr (ACC) {
      // the accumulated output is read before the patch product, which it
      // does not depend on, so its loads overlap the inverse stream
      R xo[NPT];
      static_for<NPT>([&](auto I) { xo[I] = out[offset(I)]; });
      packed_symv<NPT>(A, x, y);
      static_for<NPT>([&](auto I) { out[offset(I)] = xo[I] + alpha * y[I]; });
    } else {
      packed_symv<NPT>(A, x, y);
      static_for<NPT>([&](auto I) { store(I, y[I]); });
    }
  } else {
    __shared__ R xs[NPT * 64];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    static_for<NPT>([&](auto I) {
      if (w == (I & 3)) xs[I * 64 + lane] = in[offset(I)];
    });
    __syncthreads();
    // few workgroups (one per 64 coarse cells): long chunks keep more bytes
    // in flight per wavefront, occupancy does not matter here
    split_symv81<sizeof(R) == 8 ? 32 : 64>(A, xs, lane, w, store);
  }
}

// 3D centre solves with the four pieces of split_symv81 on four separate
// single-wavefront workgroups (grid: tiles of 64 coarse cells x 4 pieces), so
// that a level with few coarse cells spreads its inverse stream over four
// times as many compute units; piece w of tile t writes its partial rows to
// part[(t*4 + w)*61 + slot][64]. k_center_combine then sums them in the
// order split_symv81 uses (y0 + y1, y0 + y2, (y1 + y2) + y3), so the result
// is bit-identical to k_center_solve.
template <class PC, int CH, class R, class XR>
__device__ __attribute__((always_inline)) inline void piece_to_global(const R* __restrict__ A, const XR& xr,
                                                                      R* __restrict__ dst, int lane) {
  R y[PC::ny];
  piece_symv<CH, PC>(A, xr, y);
  static_for<PC::ny>([&](auto I) { dst[(int64_t)I * 64 + lane] = y[I]; });
}

constexpr int kCenterCH64 = 32, kCenterCH32 = 64;

template <class R>
__global__ void __launch_bounds__(64) k_center_piece(LevelGeo g, const R* __restrict__ inv,
                                                      const R* __restrict__ in, R* __restrict__ part) {
  constexpr int NN = 27, NPT = 81;
  const int nc = g.N / 2;
  const int ncc = nc * nc * nc;
  const int lane = threadIdx.x;
  const int tile = blockIdx.x, w = blockIdx.y;
  const int s = tile * 64 + lane;
  const int sc = s < ncc ? s : ncc - 1;
  const int K0 = sc % nc, K1 = (sc / nc) % nc, K2 = sc / (nc * nc);
  const int64_t base = node_index<3>(g, 4 * K0 + 1, 4 * K1 + 1, 4 * K2 + 1);
  const int64_t n1 = g.n1;
  // each lane stages and reads only its own column: no barrier needed
  __shared__ R xs[NPT * 64];
  static_for<NPT>([&](auto I) {
    constexpr int i = I;
    constexpr int comp = i / NN, loc = i % NN;
    xs[i * 64 + lane] = in[comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * digit(loc, 2))];
  });
  const int64_t P = (int64_t)NPT * (NPT + 1) / 2;
  const R* A = inv + ((int64_t)tile * P) * 64 + lane;
  auto xr = [&](int j) { return xs[j * 64 + lane]; };
  R* dst = part + ((int64_t)(tile * 4 + w) * 61) * 64;
  constexpr int CH = sizeof(R) == 8 ? kCenterCH64 : kCenterCH32;
  if (w == 0) piece_to_global<Q81_0, CH>(A, xr, dst, lane);
  else if (w == 1) piece_to_global<Q81_1, CH>(A, xr, dst, lane);
  else if (w == 2) piece_to_global<Q81_2, CH>(A, xr, dst, lane);
  else piece_to_global<Q81_3, CH>(A, xr, dst, lane);
}

template <bool ACC, class R>
__global__ void __launch_bounds__(64) k_center_combine(LevelGeo g, const R* __restrict__ part, R* __restrict__ out,
                                                        double alpha_d) {
  constexpr int NN = 27, NPT = 81;
  const R alpha = (R)alpha_d;
  const int nc = g.N / 2;
  const int ncc = nc * nc * nc;
  const int lane = threadIdx.x;
  const int tile = blockIdx.x;
  const int s = tile * 64 + lane;
  if (s >= ncc) return;
  const int K0 = s % nc, K1 = (s / nc) % nc, K2 = s / (nc * nc);
  const int64_t base = node_index<3>(g, 4 * K0 + 1, 4 * K1 + 1, 4 * K2 + 1);
  const int64_t n1 = g.n1;
  const R* p0 = part + ((int64_t)(tile * 4 + 0) * 61) * 64 + lane;
  const R* p1 = part + ((int64_t)(tile * 4 + 1) * 61) * 64 + lane;
  const R* p2 = part + ((int64_t)(tile * 4 + 2) * 61) * 64 + lane;
  const R* p3 = part + ((int64_t)(tile * 4 + 3) * 61) * 64 + lane;
  static_for<NPT>([&](auto I) {
    constexpr int i = I;
    R y;
    if constexpr (i < 20) y = p0[Q81_0::slot(i) * 64] + p1[Q81_1::slot(i) * 64];
    else if constexpr (i < 40) y = p0[Q81_0::slot(i) * 64] + p2[Q81_2::slot(i) * 64];
    else y = (p1[Q81_1::slot(i) * 64] + p2[Q81_2::slot(i) * 64]) + p3[Q81_3::slot(i) * 64];
    constexpr int comp = i / NN, loc = i % NN;
    const int64_t o = comp * g.nnodes + base + digit(loc, 0) + n1 * (digit(loc, 1) + n1 * digit(loc, 2));
    if constexpr (ACC) out[o] += alpha * y;
    else out[o] = alpha * y;
  });
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }


template <class R>
static const R* class_inv(const PatchClass& pc);
template <>
const double* class_inv<double>(const PatchClass& pc) { return pc.inv; }
template <>
const float* class_inv<float>(const PatchClass& pc) { return pc.inv32; }

template <int D, class R>
static void asm_gemv_variant(int v, hipStream_t s, const AsmBatch<R>& B) {
  const dim3 grid((unsigned)B.first[B.n]), blk(asm_threads<D>());
  if (grid.x == 0) return;
  if (v == 1) hipLaunchKernelGGL((k_asm_gemv<D, R, 1>), grid, blk, 0, s, B);
  else if (v == 2) hipLaunchKernelGGL((k_asm_gemv<D, R, 2>), grid, blk, 0, s, B);
  else if (v == 3) hipLaunchKernelGGL((k_asm_gemv<D, R, 3>), grid, blk, 0, s, B);
  else hipLaunchKernelGGL((k_asm_gemv<D, R, 0>), grid, blk, 0, s, B);
}

// Appends the patch solves of level l (residual r, output zbuf) to a batch;
// returns their algorithmic bytes (packed inverses, patch outputs, one read
// of the residual).
template <class R>
static double asm_add_entry(const Hier& H, const Level& l, const R* r, R* zbuf, AsmBatch<R>& B) {
  const int k = B.n++;
  AsmClasses<R>& c = B.c[k];
  c = AsmClasses<R>{};
  int blocks = 0;
  double bytes = (double)sizeof(R) * (double)l.nvel;
  const int ncls = H.dim == 2 ? 3 : 4;
  for (int ci = 0; ci < 4; ++ci) {
    c.first_block[ci] = blocks;
    if (ci < ncls && ci < (int)l.cls.size()) {
      const PatchClass& pc = l.cls[ci];
      c.verts[ci] = pc.verts;
      c.inv[ci] = class_inv<R>(pc);
      c.count[ci] = pc.count;
      const int per = (H.dim == 2 || ci == 0) ? 64 : 256;   // patches per workgroup
      blocks += (pc.count + per - 1) / per;
      bytes += (double)sizeof(R) * (double)pc.count * (pc.n * (pc.n + 1) / 2 + pc.n);
    }
  }
  c.first_block[4] = blocks;
  B.g[k] = l.g;
  B.r[k] = r;
  B.zbuf[k] = zbuf;
  B.nvert[k] = l.nvert;
  B.first[k + 1] = B.first[k] + blocks;
  return bytes;
}

// The batched patch solves of one ASM application into the level's patch
// output buffer (or `zbuf` if not NULL), with the level's chosen variant
// (reps launches back to back).
template <class R>
void launch_asm_gemv(const Hier& H, const Level& l, const R* r, int reps, hipStream_t s, double* bytes_out,
                     R* zbuf) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) {
      // [Q3]^2 x P2disc: one class of 50-unknown patches
      const PatchClass& pc = l.cls[0];
      for (int k = 0; k < reps; ++k) q3_asm_solves(H, l, r, zbuf ? zbuf : l.zbuf, s);
      if (bytes_out) *bytes_out = 8.0 * ((double)l.nvel + (double)pc.count * (pc.n * (pc.n + 1) / 2 + pc.n));
      return;
    }
  }
  AsmBatch<R> B{};
  const double bytes = asm_add_entry<R>(H, l, r, zbuf ? zbuf : reinterpret_cast<R*>(l.zbuf), B);
  const int v = l.asm_variant[sizeof(R) == 8 ? 0 : 1];
  for (int k = 0; k < reps; ++k) {
    if (H.dim == 2) asm_gemv_variant<2, R>(v, s, B);
    else asm_gemv_variant<3, R>(v, s, B);
  }
  if (bytes_out) *bytes_out = bytes;
}

template <class R>
void launch_asm_gemv_batch(const Hier* const* hs, const Level* const* ls, const R* const* rs, int n,
                           hipStream_t s) {
  if (n > 0 && hs[0]->deg == 3) {
    for (int k = 0; k < n; ++k) launch_asm_gemv<R>(*hs[k], *ls[k], rs[k], 1, s, nullptr, nullptr);
    return;
  }
  for (int k0 = 0; k0 < n; k0 += kAsmBatchMax) {
    AsmBatch<R> B{};
    const int kn = std::min(kAsmBatchMax, n - k0);
    for (int k = 0; k < kn; ++k)
      asm_add_entry<R>(*hs[k0 + k], *ls[k0 + k], rs[k0 + k], reinterpret_cast<R*>(ls[k0 + k]->zbuf), B);
    const int v = ls[k0]->asm_variant[sizeof(R) == 8 ? 0 : 1];
    if (hs[k0]->dim == 2) asm_gemv_variant<2, R>(v, s, B);
    else asm_gemv_variant<3, R>(v, s, B);
  }
}

template <class R>
void launch_asm_solves(Hier& H, const Level& l, const R* r, hipStream_t s) {
  hipEvent_t ev = nullptr;
  const int reps = prof_begin(H, s, &ev);
  // the kernel is a pure function of (r, inverses) -> zbuf, so a profiled
  // call may repeat it back to back to time it without launch gaps
  double bytes = 0.0;
  launch_asm_gemv<R>(H, l, r, reps, s, &bytes, nullptr);
  prof_end(H, s, PROF_ASM_GEMV, ev, bytes, reps);
}

template <class R>
void launch_asm_gather(const Hier& H, const Level& l, const R* zbuf, R* y, hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_asm_gather(H, l, zbuf, y, s);
  }
  const int64_t n = (int64_t)H.dim * l.g.nnodes;
  if (H.dim == 2)
    hipLaunchKernelGGL((k_asm_gather<2, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
  else
    hipLaunchKernelGGL((k_asm_gather<3, R>), dim3(nblk(n, 256)), dim3(256), 0, s, l.g, zbuf, l.nvert, y);
}

template <class R>
void launch_asm(Hier& H, const Level& l, const R* r, R* y, hipStream_t s, R* zbuf) {
  if (zbuf) {
    // caller-provided patch output buffer (no tracing)
    launch_asm_gemv<R>(H, l, r, 1, s, nullptr, zbuf);
    launch_asm_gather<R>(H, l, zbuf, y, s);
    return;
  }
  launch_asm_solves<R>(H, l, r, s);
  launch_asm_gather<R>(H, l, reinterpret_cast<const R*>(l.zbuf), y, s);
}

// Below this many 64-cell tiles (about two per compute unit) the 3D centre
// solves run as four single-wavefront pieces per tile plus a combine kernel.
constexpr int kSplitCenterTiles = 512;

template <class R>
void launch_center_solve(const Hier& H, const Level& fine, const R* in, R* out, double alpha, bool accumulate,
                         hipStream_t s) {
  if constexpr (std::is_same<R, double>::value) {
    if (H.deg == 3) return q3_center_solve(H, fine, in, out, alpha, accumulate, s);
  }
  const int nc = fine.g.N / 2;
  const int ncc = H.dim == 2 ? nc * nc : nc * nc * nc;
  const dim3 grid(nblk(ncc, 64)), blk(H.dim == 2 ? center_threads<2>() : center_threads<3>());
  const R* inv = class_inv<R>(fine.cls[0]);
  if (H.dim == 2) {
    if (accumulate) hipLaunchKernelGGL((k_center_solve<2, true, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
    else hipLaunchKernelGGL((k_center_solve<2, false, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
  } else if (grid.x < (unsigned)kSplitCenterTiles &&
             (int64_t)grid.x * 4 * 61 * 64 * (int64_t)sizeof(R) <= (int64_t)Dims<3>::NL * fine.g.ncell * 8) {
    // few tiles: pieces on separate workgroups, partial rows through the
    // fine level's element buffer (unused while a transfer runs its local
    // solves; it holds 81 doubles per fine cell, enough for the partials
    // from 6^3 fine cells up)
    R* part = reinterpret_cast<R*>(fine.E);
    hipLaunchKernelGGL((k_center_piece<R>), dim3(grid.x, 4), dim3(64), 0, s, fine.g, inv, in, part);
    if (accumulate) hipLaunchKernelGGL((k_center_combine<true, R>), grid, dim3(64), 0, s, fine.g, (const R*)part, out, alpha);
    else hipLaunchKernelGGL((k_center_combine<false, R>), grid, dim3(64), 0, s, fine.g, (const R*)part, out, alpha);
  } else {
    if (accumulate) hipLaunchKernelGGL((k_center_solve<3, true, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
    else hipLaunchKernelGGL((k_center_solve<3, false, R>), grid, blk, 0, s, fine.g, inv, in, out, alpha);
  }
}

template void launch_asm_gemv<double>(const Hier&, const Level&, const double*, int, hipStream_t, double*, double*);
template void launch_asm_gemv<float>(const Hier&, const Level&, const float*, int, hipStream_t, double*, float*);
template void launch_asm_gemv_batch<double>(const Hier* const*, const Level* const*, const double* const*, int,
                                            hipStream_t);
template void launch_asm_gemv_batch<float>(const Hier* const*, const Level* const*, const float* const*, int,
                                           hipStream_t);
template void launch_asm_gather<double>(const Hier&, const Level&, const double*, double*, hipStream_t);
template void launch_asm_gather<float>(const Hier&, const Level&, const float*, float*, hipStream_t);
template void launch_asm<double>(Hier&, const Level&, const double*, double*, hipStream_t, double*);
template void launch_asm<float>(Hier&, const Level&, const float*, float*, hipStream_t, float*);
template void launch_asm_solves<double>(Hier&, const Level&, const double*, hipStream_t);
template void launch_asm_solves<float>(Hier&, const Level&, const float*, hipStream_t);
template void launch_center_solve<double>(const Hier&, const Level&, const double*, double*, double, bool,
                                          hipStream_t);
template void launch_center_solve<float>(const Hier&, const Level&, const float*, float*, double, bool,
                                         hipStream_t);

}  // namespace stk
