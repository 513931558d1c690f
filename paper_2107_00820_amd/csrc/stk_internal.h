// Internal declarations shared by the host orchestration and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <string>
#include <vector>

#include "stk_ref.h"

namespace stk {

constexpr int kMaxNu = 8;          // relaxation steps per smoothing call
// 1 / Mhat: inverse of the reference pressure mass diag(1, 1/12, ..)
constexpr double kInvMhat[4] = {1.0, 12.0, 12.0, 12.0};
constexpr int kRedBlocks = 512;    // fixed grid of the deterministic reductions
constexpr int kRedThreads = 1024;   // largest workgroup of the reductions (see red_threads)
constexpr int64_t kRedLongVector = 2000000;

// Modes of the element kernel (bit set).
enum : int {
  EL_VISC = 1,   // viscous term (2 mu eps(u), eps(v))
  EL_AUG = 2,    // augmented term gamma (Pi div u, div v)
  EL_BT = 4,     // B^T p from the pressure input
  EL_BOUT = 8,   // write (B u) to the pressure output
  EL_NL = 16     // viscous term of the capped viscoplastic law at the input's own strain rate
                 // (mu_eff from the base viscosity table; nonlinear residual)
};

// One class of vertex-star patches with the same number of unknowns.
struct PatchClass {
  int n = 0;              // unknowns per patch
  int count = 0;          // patches in the class
  int* verts = nullptr;   // [count] vertex index (lexicographic over (N+1)^d)
  double* inv = nullptr;  // packed inverses, interleaved in blocks of 64 patches
  float* inv32 = nullptr; // FP32 copy (mixed form)
};

// Variants of the batched patch solve a tuner may choose between per level
// and precision (bit-identical results; they differ in load chunking and
// occupancy only).
constexpr int kAsmVariants = 4;
// Entries (level solves of possibly different hierarchies) per batched
// patch-solve launch.
constexpr int kAsmBatchMax = 8;

struct Level {
  LevelGeo g{};
  int asm_variant[2] = {0, 0};   // chosen patch-solve variant: [0] FP64, [1] FP32
  int nvert = 0;               // (N+1)^d
  int64_t nvel = 0;            // d * nnodes
  int64_t npres = 0;           // (d+1) * ncell
  double* mu = nullptr;        // [ncell][NQ] viscosity (mu_eff for the tensor law) at Gauss points
  float* mu32 = nullptr;       // FP32 copy (mixed form)
  // tensor law only: w at the Gauss points, C:eps = 2 mu eps - (w:eps) w,
  // [ncell][d(d+1)/2][NQ] (symmetric storage order of SymIdx)
  double* cw = nullptr;
  float* cw32 = nullptr;
  // W = M_p(1/mu) (preconditioner P2 of eq. (P1P2)): per cell the inverse of
  // the reference weighted pressure mass sum_q w_q / mu_q psi psi^T,
  // [ncell][(d+1)^2]; NULL for W = M_p
  double* winv = nullptr;
  float* winv32 = nullptr;
  double* E = nullptr;         // [NL][ncell] element outputs
  // relaxation and transfer work vectors (stored layout)
  double *b = nullptr, *x = nullptr, *r = nullptr, *T = nullptr, *U = nullptr, *S = nullptr;
  // S holds A_K^{-1} r on the coarse-cell interiors and must stay zero on the
  // coarse-cell boundaries; the FP32 path keeps its own zero-initialised copy
  // because FP64 writes into S would leave non-zero bytes under FP32 views.
  float* S32 = nullptr;
  double* V = nullptr;         // (kMaxNu+1) * nvel
  double* Z = nullptr;         // kMaxNu * nvel
  double* small = nullptr;     // device scalars: H, beta, y
  std::vector<PatchClass> cls; // [0] = interior patches (all-odd parity class first)
  double* zbuf = nullptr;      // [d*3^d][nvert] patch outputs
};

// Optional per-kernel timing with HIP events on the launch stream (used by
// the benchmark to measure the average launch duration of a kernel family
// live, over the timed region).
enum ProfId : int { PROF_ASM_GEMV = 0, PROF_ELEM = 1, PROF_NIDS = 2 };
struct Prof {
  bool on = false;
  int reps = 1;            // back-to-back repetitions of a profiled launch
  struct Rec {
    int id;
    hipEvent_t a, b;
    double bytes;          // algorithmic bytes of all repetitions
    int n;                 // launches between a and b
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};

struct Hier {
  int dim = 2, L = 0, nu_pre = 2, nu_post = 2, schur = 1;
  int deg = 2;                       // velocity degree k: 2, or 3 ([Q3]^2 x P2disc, 2D, FP64)
  double gamma = 0.0;
  int n_sinkers = 0;
  double omega = 0.1, delta = 200.0, mu_min = 1.0, mu_max = 1.0, beta = 10.0;
  double* centers = nullptr;         // device [n][d]
  // viscoplastic Newton tensor (coef_kind 1)
  int coef_kind = 0;
  int vp_modes = 0;
  double* vp_amp = nullptr;          // device [d][modes^d]
  double vp_tau_y = 0.0, vp_scale = 0.0;   // vp_scale <= 0: RMS of eps_II over fine Gauss points = 1
  double vp_floor = 0.0;                   // mu_floor of the capped law
  std::vector<Level> lv;
  // coarse level
  int64_t n0 = 0;
  double* Ainv0 = nullptr;           // -A_0^{-1}, lower triangle in 64 x 64 tiles
  double* cwork = nullptr;           // sweep work: pivot inverse + two panels
  double* cvec = nullptr;            // gathered coarse right-hand side (64 * tiles)
  double* cpart = nullptr;           // tile GEMV partials (tiles^2 * 64)
  // finest-level Schur blocks and pressure work
  double* Sinv = nullptr;            // [ncell][(d+1)^2]
  double* partials = nullptr;        // kRedBlocks * 64
  int* flag = nullptr;               // device error flag
  // FGMRES storage (allocated on first solve)
  int restart_alloc = 0;
  double *fV = nullptr, *fZ = nullptr, *fw = nullptr, *fr = nullptr, *fH = nullptr, *fy = nullptr;
  double *pw_u = nullptr, *pw_y = nullptr;  // preconditioner work (fine velocity)
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::vector<void*> allocs;
  Prof prof;
  // FGMRES Arnoldi steps captured as HIP graphs (one per step index j) and
  // replayed on the library's own stream
  hipStream_t own = nullptr;
  std::vector<hipGraphExec_t> steps;
  int steps_m = 0;
  int steps_key = 0;      // preconditioner variant the graphs were captured for
  // mixed form: FP32 copies exist; fine-level FP32 V-cycle input/output
  int mixed = 0;
  double *mb = nullptr, *mx = nullptr;
  // Resumable FGMRES: the solve advances in phases (Arnoldi step, residual
  // check after a cycle, final copy-out); each phase's device work is
  // enqueued on `own`, ends in a copy of the few numbers the host needs into
  // pinned memory and an event, so several solves can have work in flight.
  enum Phase : int { SV_IDLE = 0, SV_ARNOLDI = 1, SV_RESIDUAL = 2, SV_FINISH = 3, SV_DONE = 4 };
  struct Solve {
    int phase = SV_IDLE;
    int status = 0;
    int m = 30, maxit = 300, j = 0, k = 0, it = 0;
    bool mixed = false, upper = false, graphs = true, converged = false, fcycle = false;
    bool inflight = false;   // the current phase's device work is enqueued and not yet advanced
    double rtol = 1e-8, bnorm = 0.0, beta = 0.0, t_solve = 0.0;
    double *x_u = nullptr, *x_p = nullptr;
    std::vector<double> Hh, cs, sn, g, hist;
    std::chrono::steady_clock::time_point t0;
  } sv;
  double* hpin = nullptr;          // pinned host: Hessenberg copy, norm partials, y
  hipEvent_t sev = nullptr;        // end of the last enqueued phase
  // lockstep batching of patch solves across hierarchies: this stream has
  // reached a patch-solve call (bev); the batched launch is done (cev, used
  // when this hierarchy leads a batch)
  hipEvent_t bev = nullptr, cev = nullptr;
  // viscoplastic Newton (coef_kind 2): base viscosity mu0 at the finest
  // level's Gauss points, and the Newton work vectors [u | p] (right-hand
  // side, residual, step, trial iterate)
  double* mu0 = nullptr;
  double *nl_b = nullptr, *nl_F = nullptr, *nl_d = nullptr, *nl_x = nullptr, *nl_t = nullptr;
  // degree 3 in 3D: setup workspace (cell matrices of one level, then the
  // batched sweep's work)
  double* q3cm = nullptr;
};

// Sets the thread-local message returned by stk_last_error().
void set_last_error(const std::string& msg);

// Event bracketing of one launch (no-ops unless H.prof.on).
// prof_begin returns how many times the caller issues the launch (1 unless profiling).
int prof_begin(Hier& H, hipStream_t s, hipEvent_t* ev);
void prof_end(Hier& H, hipStream_t s, int id, hipEvent_t a, double bytes, int reps);

// ---- kernel launchers (templated on dimension inside the .hip files) ----
void launch_mu_sinker(const Hier& H, const Level& l, hipStream_t s);
// the sinker viscosity at the level's Gauss points into out ([ncell][3^d])
void launch_mu_sinker_to(const Hier& H, const Level& l, double* out, hipStream_t s);
// Viscoplastic state of a Newton linearisation: mu_eff and w on a level from
// an FE velocity u of that level (stored layout).
void launch_coef_fe(const Hier& H, const Level& l, const double* u, hipStream_t s);
// uc = fine velocity at the coarse nodes (coarse node i = fine node 2i)
void launch_inject(const Hier& H, const Level& fine, const Level& coarse, const double* uf, double* uc,
                   hipStream_t s);
// Cell kernel of the nonlinear residual on the finest level: element vectors
// of a(u; v) + gamma (W^{-1} B u, B v) + (p, B v) into l.E and B u into pout.
void launch_nl_elem(const Hier& H, const Level& l, const double* u, const double* p, double* pout, hipStream_t s);
// Viscoplastic Newton tensor: partial sums of the unscaled eps_II^2 over the
// finest level's Gauss points (into H.partials), then mu_eff and w per level.
void launch_eps_partials(const Hier& H, const Level& fine, hipStream_t s);
void launch_coef_tensor(const Hier& H, const Level& l, const Level& fine, hipStream_t s);
template <class R>
void launch_elem(const Hier& H, const Level& l, int mode, const R* u, const double* p, double* pout,
                 hipStream_t s);
template <class R>
void launch_gather(const Hier& H, const Level& l, const R* base, double alpha, R* out, hipStream_t s);
// 2D only: cell kernel on the sum of the patch outputs held in l.zbuf, which
// it also stores to z (replaces the patch-output gather plus launch_elem)
template <class R>
void launch_elem_asm(const Hier& H, const Level& l, R* z, hipStream_t s);
// gather of the element outputs into out[0, d*nnodes) fused with the partial
// dot products V_k . out over out[0, nvec) (same partition as launch_dots)
template <class R>
void launch_gather_dots(const Hier& H, const Level& l, R* out, int64_t nvec, const R* V, int64_t ldv, int nk,
                        double* part, hipStream_t s);
void launch_rhs_elem(const Hier& H, const Level& l, hipStream_t s);
void launch_schur_setup(const Hier& H, const Level& l, hipStream_t s);
void launch_winv_setup(const Hier& H, const Level& l, hipStream_t s);
void launch_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp,
                        hipStream_t s);
void launch_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s);

void launch_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s);
// zbuf: patch output buffer to use instead of l.zbuf (NULL: l.zbuf; a
// caller-provided buffer is not traced).
template <class R>
void launch_asm(Hier& H, const Level& l, const R* r, R* y, hipStream_t s, R* zbuf = nullptr);
template <class R>
void launch_asm_gather(const Hier& H, const Level& l, const R* zbuf, R* y, hipStream_t s);
// The patch solves of one ASM application into l.zbuf (traced like
// launch_asm), without the gather to a node vector.
template <class R>
void launch_asm_solves(Hier& H, const Level& l, const R* r, hipStream_t s);
// The patch-solve kernel alone (reps launches), no gather and no tracing;
// *bytes_out receives its algorithmic bytes per launch if non-NULL.
template <class R>
void launch_asm_gemv(const Hier& H, const Level& l, const R* r, int reps, hipStream_t s, double* bytes_out,
                     R* zbuf = nullptr);
// One launch (per kAsmBatchMax entries) of the patch solves of n levels
// (ls[k] of hierarchy hs[k], residual rs[k], output ls[k]->zbuf); all of one
// dimension; the variant of the first entry is used (variants give
// bit-identical results).
template <class R>
void launch_asm_gemv_batch(const Hier* const* hs, const Level* const* ls, const R* const* rs, int n,
                           hipStream_t s);
template <class R>
void launch_center_solve(const Hier& H, const Level& fine, const R* in, R* out, double alpha, bool accumulate,
                         hipStream_t s);

template <class R>
void launch_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const R* xc, R* xf, hipStream_t s);
template <class R>
void launch_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const R* rf, R* rc, hipStream_t s);

int coarse_tiles(int64_t n);       // 64-wide tiles per row of the coarse matrix
void launch_coarse_assemble(const Hier& H, const Level& l, double* A, hipStream_t s);
int launch_coarse_invert(const Hier& H, double* A, int64_t n, double* work, hipStream_t s);
template <class R>
void launch_coarse_apply(const Hier& H, const Level& l, const R* b, R* x, hipStream_t s);

// Krylov helpers (vectors of length n, storage type R; reductions in double)
template <class R>
void launch_dots(const R* V, int64_t ldv, int nk, const R* w, int64_t n, double* partials, hipStream_t s);
template <class R>
void launch_orth_update(const R* V, int64_t ldv, int nk, R* w, int64_t n, const double* part_in, double* Hcol,
                        int hstride, bool accumulate, double* part_out, bool next_dots, hipStream_t s);
template <class R>
void launch_normalize(const double* norm_partials, R* w, int64_t n, R* dst, double* hout, hipStream_t s);
template <class R>
void launch_relax_update(const R* Z, int64_t ldz, int nu, const double* small, const double* norm_part, R* x,
                         int64_t n, bool x_zero, hipStream_t s);
void launch_combine(const double* Z, int64_t ldz, int nk, const double* y, double* x, int64_t n,
                    bool x_zero, hipStream_t s);
template <class R>
void launch_axpby(double a, const R* x, double b, const R* y, R* out, int64_t n, hipStream_t s);
template <class R>
void launch_fill(R* x, double v, int64_t n, hipStream_t s);
template <class A, class B>
void launch_convert(const A* x, B* y, int64_t n, hipStream_t s);
void launch_copy(const double* x, double* y, int64_t n, hipStream_t s);
void launch_fill_int(int* x, int v, int64_t n, hipStream_t s);

// ---- [Q3]^2 x P2disc levels (Hier::deg == 3; 2D, FP64, scalar viscosity):
// the same operations as the launchers above, which route to these ----
void q3_mu_sinker(const Hier& H, const Level& l, double* out, hipStream_t s);
void q3_rhs_elem(const Hier& H, const Level& l, hipStream_t s);
void q3_elem(const Hier& H, const Level& l, int mode, const double* u, const double* p, double* pout,
             hipStream_t s);
void q3_gather(const Hier& H, const Level& l, const double* base, double alpha, double* out, hipStream_t s);
void q3_winv_setup(const Hier& H, const Level& l, hipStream_t s);
void q3_schur_setup(const Hier& H, const Level& l, hipStream_t s);
void q3_schur_apply(const Hier& H, const Level& l, const double* y, const double* vp, double* zp, hipStream_t s);
void q3_project_mean(const Hier& H, const Level& l, double* p, hipStream_t s);
void q3_patch_setup(const Hier& H, const Level& l, const PatchClass& pc, hipStream_t s);
void q3_asm_solves(const Hier& H, const Level& l, const double* r, double* zbuf, hipStream_t s);
void q3_asm_gather(const Hier& H, const Level& l, const double* zbuf, double* y, hipStream_t s);
void q3_center_solve(const Hier& H, const Level& fine, const double* in, double* out, double alpha,
                     bool accumulate, hipStream_t s);
void q3_prolong_std(const Hier& H, const Level& coarse, const Level& fine, const double* xc, double* xf,
                    hipStream_t s);
void q3_restrict_std(const Hier& H, const Level& fine, const Level& coarse, const double* rf, double* rc,
                     hipStream_t s);

// layout of Level::small
constexpr int kSmallH = 0;                               // H[(kMaxNu+1) x kMaxNu], row i col j at i*kMaxNu+j
constexpr int kSmallBeta = (kMaxNu + 1) * kMaxNu;        // beta
constexpr int kSmallY = kSmallBeta + 1;                  // y[kMaxNu]
constexpr int kSmallLen = kSmallY + kMaxNu + 8;

}  // namespace stk
