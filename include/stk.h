/*
 * stk -- augmented-Lagrangian Stokes multigrid on AMD MI355X (gfx950).
 *
 * C ABI of libstk.so. Problem (Section 2, eq. (stokessys); Section 3,
 * eq. (augstokessys)): find (u, p) in [Q2]^d x P1disc on the unit square/cube,
 * u = 0 on the boundary, int p = 0, with
 *     [A_gamma  B^T] [u]   [b_u]
 *     [B        0  ] [p] = [ 0 ],   A_gamma = A + gamma B^T W^{-1} B,
 * A the viscous form (2 mu eps(u), eps(v)) (or (C:eps(u), eps(v)) for a
 * fourth-order tensor C), B the divergence -(psi, div u), W the pressure mass
 * matrix M_p (preconditioner P1) or M_p(1/mu) (P2).
 *
 * Conventions for every buffer argument:
 *  - All vectors are caller-owned contiguous DEVICE buffers unless stated.
 *  - Velocity "stored" layout on a level with N cells per axis: the full node
 *    grid of (2N+1)^d nodes per component, component-major, x fastest:
 *    index = comp*(2N+1)^d + (iz*(2N+1) + iy)*(2N+1) + ix. Entries on the
 *    boundary (Dirichlet nodes) are ignored on input and written as 0.
 *    For degree 3 (stk_desc.degree) the grid has 3N+1 nodes per axis.
 *  - Pressure layout: p[cell*(d+1) + m], cell lexicographic with x fastest,
 *    basis psi_0 = 1, psi_j = (x_j - c_j)/h on each cell (c the cell centre).
 *    For degree 3: p[cell*6 + m] with the monomials 1, x, y, x^2, xy, y^2 of
 *    (x - c)/h (total degree <= 2); in 3D p[cell*10 + m] with 1, x, y, z, x^2,
 *    xy, xz, y^2, yz, z^2.
 *  - Level 0 is the coarsest level, level n_levels-1 the finest.
 *  - Every call is asynchronous on the HIP stream passed (hipStream_t as
 *    void*, NULL = default stream) except stk_setup_hierarchy and stk_solve,
 *    which return after their work has completed.
 *  - Errors: no exception crosses the ABI; every call returns a stk_status
 *    and stk_last_error() returns a thread-local message for the last failure.
 *  - A hierarchy is used by one stream at a time; calls that overlap on one
 *    hierarchy race on its work buffers. While a resumable solve
 *    (stk_solve_begin .. the stk_poll that reports its end) is in progress,
 *    every other call on that hierarchy that would touch its device buffers
 *    returns STK_EBUSY without doing anything.
 */
#ifndef STK_H
#define STK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stk_hier stk_hier;   /* opaque, library-owned device state */

typedef enum {
  STK_OK = 0,
  STK_EINVAL = -1,      /* bad argument (size, level, null pointer, dtype) */
  STK_ENOMEM = -2,      /* device allocation failed or footprint over budget */
  STK_EDEVICE = -3,     /* a HIP call failed */
  STK_ENOTCONV = -4,    /* FGMRES hit maxit; the best iterate is returned */
  STK_ENOTSPD = -5,     /* non-positive pivot in a patch or coarse factorisation */
  STK_ENAN = -6,        /* NaN/Inf in the right-hand side or the residual */
  STK_EBUSY = -7        /* a solve is still running (serving interface) */
} stk_status;

typedef enum { STK_F64 = 0, STK_F32 = 1 } stk_dtype;

/* Multi-sinker viscosity of Section 5.2 (reading: floor mu_min and squared
 * Gaussian):  chi(x) = prod_i [1 - exp(-delta max(0,|x-c_i| - omega/2)^2)],
 * mu = (mu_max - mu_min)(1 - chi) + mu_min, forcing f = (0,..,beta(chi-1)).
 * `centers` is a HOST array [n][d] copied during setup. */
typedef struct {
  int n;
  const double* centers;
  double omega, delta, mu_min, mu_max, beta;
} stk_sinker;

/* Viscoplastic Newton tensor (Section 5.3.1; coef_kind = 1). Reading for the
 * synthetic workload: the base field mu0 is the multi-sinker field of
 * `sinker`, capped by the yield stress tau_y at the strain rate eps of a
 * smooth Fourier velocity
 *   u_c(x) = s sum_{m in {1..modes}^d} amp[c][m_1]..[m_d] / (1 + |m|^2)
 *            prod_j sin(pi m_j x_j)
 * (amp is a HOST array [d][modes]^d, C order, copied during setup):
 *   eps_II = (eps:eps / 2)^(1/2),
 *   mu_eff = mu_floor + min(mu0 - mu_floor, tau_y / (2 eps_II)),
 *   C = 2 mu_eff I - 2 (mu_eff - mu_floor) [yielded] n (x) n,  n = eps/|eps|_F,
 * the exact derivative of tau(eps) = 2 mu_eff(eps_II) eps; yielded means
 * tau_y / (2 eps_II) < mu0 - mu_floor. C is symmetric positive definite with
 * smallest eigenvalue 2 mu_floor (along n where yielded). C is stored per
 * Gauss point as mu_eff and w = (2 (mu_eff - mu_floor) [yielded])^(1/2) n, so
 * C:e = 2 mu_eff e - (w:e) w. The Schur blocks use the scalar mu_eff. */
typedef struct {
  int modes;           /* 1..8 */
  const double* amp;
  double tau_y;        /* > 0 */
  double mu_floor;     /* > 0; <= 0 selects sinker.mu_min */
  double eps_scale;    /* s above; <= 0 asks the library to choose s so that
                          the root mean square of eps_II over the finest
                          level's Gauss points is 1 */
} stk_viscoplastic;

typedef struct {
  int dim;            /* 2 or 3 */
  int n_fine;         /* cells per axis on the finest level, divisible by 2^(n_levels-1) */
  int n_levels;       /* >= 2 */
  int qpts_1d;        /* Gauss-Legendre points per axis for every integral
                         (A, B, M_p, M_p(1/mu), the right-hand side); 0 selects
                         the default 3 (exact for the constant-coefficient Q2
                         stiffness on affine cells), the only rule built */
  double gamma;       /* augmented-Lagrangian parameter, >= 0 */
  int schur;          /* W in A_gamma and the Schur blocks (eq. (P1P2)):
                         1 = P1: W = M_p, Shat^{-1} = M_p(1/mu)^{-1} + gamma M_p^{-1};
                         2 = P2: W = M_p(1/mu), Shat^{-1} = (1 + gamma) M_p(1/mu)^{-1}.
                         The augmented system has the Stokes solution for either W. */
  int coef_kind;      /* 0 = scalar sinker viscosity; 1 = viscoplastic Newton
                         tensor at the Fourier velocity of `vp`; 2 = the same law
                         at an FE velocity state (the Newton loop below; state
                         u = 0 after setup, vp.amp unused, schur must be 1) */
  stk_sinker sinker;  /* the viscosity (coef_kind 0) or the base field mu0 (1); forcing in both */
  stk_viscoplastic vp;  /* read for coef_kind 1 only */
  int nu_pre, nu_post;   /* right-preconditioned GMRES relaxation steps, 1..8 */
  int mixed;          /* 0 = FP64 form only; 1 = also keep FP32 copies of the
                         viscosity tables and packed patch inverses so that
                         the mixed form (FP32 V-cycles inside FP64 FGMRES) and
                         the STK_F32 level operations are available */
  size_t hbm_budget;  /* bytes; 0 = unlimited. Setup fails with STK_ENOMEM above it */
  int degree;         /* velocity degree k of [Q_k]^d x P_{k-1}^disc (Section 4,
                         definition of V_h^k and Q_h^{k-1}): 0 or 2 = Q2 x P1disc;
                         3 = [Q3]^d x P2disc (coef_kind 0, mixed 0; cubic Lagrange
                         basis on equispaced nodes, 4-point Gauss rule: qpts_1d 0
                         or 4; in 3D up to n_fine = 32, its 375-unknown star
                         patches held as explicit inverses in 64 x 64 tiles, the
                         diagonal tiles as their lower 4 x 4 blocks), with
                         every operation below */
} stk_desc;

/* Device bytes that stk_setup_hierarchy will allocate for `desc` (host-only
 * arithmetic, no device work). Returns STK_EINVAL for an invalid desc. */
stk_status stk_footprint(const stk_desc* desc, size_t* bytes);

/* Builds the hierarchy on the current HIP device: coefficients at the Gauss
 * points of every level (rediscretisation, Section 5.1), the inverses of all
 * vertex-star patch matrices of levels >= 1 (Section 4.1, eq. (viim);
 * factored by Cholesky in FP64 and stored as explicit packed inverses), the
 * explicit inverse of the coarsest A_gamma (the paper uses a sparse direct
 * solver; at most 80,000 coarse unknowns, whose packed inverse takes
 * 4 n0^2 bytes), and the cellwise Schur blocks Shat_gamma^{-1} = M_K(1/mu)^{-1} +
 * gamma M_K^{-1} (eq. (P1P2), Section 5.1). Synchronises `stream` before
 * returning. On failure *out is NULL and nothing is leaked. */
stk_status stk_setup_hierarchy(const stk_desc* desc, void* stream, stk_hier** out);

/* Frees everything the hierarchy owns. NULL is accepted. */
stk_status stk_destroy(stk_hier* h);

/* Stored velocity length and pressure length on `level`. */
stk_status stk_sizes(const stk_hier* h, int level, int64_t* n_vel_stored, int64_t* n_pres);

/* Right-hand side of the finest level: b_u = (f, phi_i) with the forcing
 * f = (0, .., beta (chi - 1)) of the multi-sinker benchmark (Section 5.2;
 * also for coef_kind 1, whose base field is the sinker field), in the stored
 * layout, FP64; b_p = 0 (may be NULL): the augmented system keeps the
 * original right-hand side because the divergence data is zero (Section 3,
 * eq. (augstokessys)). */
stk_status stk_rhs(stk_hier* h, double* b_u, double* b_p, void* stream);

/* y = A_gamma x on `level` (matrix-free, Section 2 entries plus the
 * augmented term of Section 3). x and y are stored-layout vectors that must
 * not alias. dtype STK_F64: FP64 vectors and arithmetic. dtype STK_F32 (needs
 * a hierarchy set up with mixed=1): FP32 vectors, FP32 viscosity table and
 * FP32 arithmetic. The same dtype rule holds for stk_asm, stk_smooth,
 * stk_prolong, stk_restrict and stk_vcycle; in FP32 the patch solves use the
 * FP32 copy of the FP64 Cholesky-based inverses. */
stk_status stk_apply_Agamma(stk_hier* h, int level, int dtype, const void* x, void* y, void* stream);

/* (y_u, y_p) = K (x_u, x_p), K = [[A_gamma, B^T], [B, 0]] on the finest level. */
stk_status stk_apply_stokes(stk_hier* h, const double* x_u, const double* x_p,
                            double* y_u, double* y_p, void* stream);

/* y = D^{-1} r = sum_i I_i A_i^{-1} I_i^T r: one application of the
 * vertex-star additive Schwarz operator on `level` >= 1 (Section 4.1). */
stk_status stk_asm(stk_hier* h, int level, int dtype, const void* r, void* y, void* stream);

/* stk_asm for callers that cannot allocate device memory around the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, same kernels and bit-identical results, but
 * the patch outputs between the batched patch solves and the node sums go
 * to a fixed 64 MiB device array of the library instead of the hierarchy's
 * own buffer, and the call allocates nothing. Each GPU holds its own array
 * until the process ends; calls on one GPU share it, so calls that overlap
 * on one GPU (any hierarchies, any streams) race. A level whose patch outputs
 * (d 3^d values of the dtype per vertex) exceed 64 MiB is rejected with
 * STK_EINVAL before anything is launched; STK_EBUSY during a resumable solve. */
stk_status stk_asm_noalloc(stk_hier* h, int level, int dtype, const void* r, void* y, void* stream);

/* x <- nsteps of GMRES relaxation on A_gamma x = b on `level` >= 1, right-
 * preconditioned by D^{-1}, starting from the x passed in (zero allowed). */
stk_status stk_smooth(stk_hier* h, int level, int dtype, const void* b, void* x, int nsteps,
                      void* stream);

/* xf = P~ xc: robust prolongation from `coarse_level` to coarse_level+1
 * (Section 4.2, eq. (Ptilde)): the standard Q2 prolongation minus the
 * solution of the local problems on the fine unknowns strictly inside each
 * coarse cell with right-hand side gamma B^T W^{-1} B P_H xc. */
stk_status stk_prolong(stk_hier* h, int coarse_level, int dtype, const void* xc, void* xf,
                       void* stream);

/* rc = P~^T rf: restriction from `fine_level` to fine_level-1 (transpose of
 * the robust prolongation). */
stk_status stk_restrict(stk_hier* h, int fine_level, int dtype, const void* rf, void* rc,
                        void* stream);

/* x = A_0,gamma^{-1} b on the coarsest level: the direct coarse solve of
 * the multigrid cycle (Section 5.1; the paper uses a sparse direct solver),
 * here one product with the explicit symmetric inverse built at setup.
 * b, x: distinct FP64 vectors in the stored layout of level 0. */
stk_status stk_coarse_solve(stk_hier* h, const double* b, double* x, void* stream);

/* x = one multigrid cycle applied to b on the finest level: the
 * approximation Ahat_gamma^{-1} of Section 5.1 and the algorithm outline
 * (pre-relaxation from 0, residual, restriction with P~^T, recursion,
 * prolongation with P~, post-relaxation). The paper uses an F-cycle; this
 * call runs the V-cycle, stk_fcycle the F-cycle. The coarsest solve always
 * uses the FP64 inverse; with STK_F32 its input and output are rounded to
 * FP32. */
stk_status stk_vcycle(stk_hier* h, int dtype, const void* b, void* x, void* stream);

/* x = one F-cycle applied to b on the finest level, the "full" multigrid
 * cycle of Section 5.1 and the algorithm outline, read as PETSc's full
 * multigrid: b is restricted with P~^T to every coarser level, the coarsest
 * level is solved directly, and on each finer level the prolongated (P~)
 * coarser result is improved by one V-cycle started from it (relaxation
 * from that iterate, coarse correction from zero). dtype as for stk_vcycle. */
stk_status stk_fcycle(stk_hier* h, int dtype, const void* b, void* x, void* stream);

/* (z_u, z_p) = P (v_u, v_p): the block preconditioner of eq. (precond) with
 * two V-cycles and the cellwise Schur blocks; z_p has zero mean. Flags:
 * STK_PC_MIXED (hierarchy set up with mixed=1) runs the V-cycles in FP32 on
 * FP32 copies of their FP64 inputs, the Schur blocks, the B and B^T applies
 * and the mean projection staying FP64; STK_PC_UPPER applies the block
 * upper-triangular part instead, z_p = -Shat^{-1} v_p (mean removed),
 * z_u = Ahat^{-1}(v_u - B^T z_p), one V-cycle (a block-triangular variant of
 * the kind the paper's introduction cites); STK_PC_FCYCLE uses F-cycles
 * (stk_fcycle) for Ahat^{-1} instead of V-cycles. */
enum { STK_PC_MIXED = 1, STK_PC_UPPER = 2, STK_PC_FCYCLE = 4 };
stk_status stk_precond(stk_hier* h, int flags, const double* v_u, const double* v_p,
                       double* z_u, double* z_p, void* stream);

typedef struct {
  double rtol;   /* stop when ||b - Kx||_2 <= rtol ||b||_2 (default 1e-8) */
  int restart;   /* FGMRES restart length (default 30, max 64) */
  int maxit;     /* maximum iterations (default 300, max 1000) */
  int eager;     /* 0 (default): each Arnoldi step (two V-cycles, Schur blocks,
                    Stokes apply, Gram-Schmidt) is captured once as a HIP graph
                    on the library's own stream and replayed; 1: plain launches.
                    Both give bit-identical results. */
  int mixed;     /* 0 (default): FP64 throughout. 1: the mixed form, where the
                    preconditioner's V-cycles run in FP32 (see stk_precond)
                    while the outer FGMRES basis, Hessenberg, orthogonalisation,
                    Stokes residual and Schur scaling stay FP64; needs a
                    hierarchy set up with mixed=1. FGMRES tolerates the
                    inexact, varying preconditioner, so the stopping test on
                    the FP64 true residual is unchanged. */
  int pc;        /* 0 (default): the preconditioner of eq. (precond); 1: its
                    block upper-triangular part (see stk_precond) */
  int cycle;     /* multigrid cycle for Ahat^{-1}: 0 (default) V-cycle
                    (stk_vcycle), 1 F-cycle (stk_fcycle, the paper's cycle) */
} stk_solve_opts;

typedef struct {
  int iters;            /* FGMRES iterations done */
  int converged;        /* 1 if the true residual met rtol */
  double rel_res;       /* true ||b - Kx|| / ||b|| at exit */
  double t_solve_s;     /* wall time of the solve */
  double hist[1001];    /* Arnoldi residual estimate / ||b|| after i iterations */
} stk_solve_info;

/* Solves the augmented Stokes system with right-preconditioned FGMRES
 * (Section 5.1) from x = 0. The work runs on a stream owned by the hierarchy
 * after `stream` has drained. b_p may be NULL (zero). The pressure of the
 * result has zero mean. Host-synchronous. Returns STK_ENOTCONV if maxit was
 * reached (x then holds the last iterate) and STK_ENAN for a non-finite
 * right-hand side or residual. */
stk_status stk_solve(stk_hier* h, const double* b_u, const double* b_p, double* x_u, double* x_p,
                     const stk_solve_opts* opts, stk_solve_info* info, void* stream);

/* ---- Serving: resumable solves (continuous batching across requests) ----
 * A solve is split into phases: one FGMRES Arnoldi step (two V-cycles, Schur
 * blocks, Stokes apply, Gram-Schmidt), the true-residual check at the end of
 * a cycle, and the final copy-out. Each phase's device work runs on the
 * hierarchy's own stream and ends with a copy of the few numbers the host
 * needs (Hessenberg column, norm partials) into pinned memory, so the phases
 * of different hierarchies overlap on the device. The arithmetic is exactly
 * that of stk_solve (which is built on the same phases), so a request's
 * result does not depend on which other requests share the device.
 *
 * stk_solve_begin: checks, copies b, sets x = 0 and computes ||b|| (waits
 * for `stream`'s pending work first; host-synchronous for ||b|| only). The
 * buffers must stay valid until the solve is done. Returns STK_EBUSY if a
 * solve is still in progress on h. */
stk_status stk_solve_begin(stk_hier* h, const double* b_u, const double* b_p, double* x_u, double* x_p,
                           const stk_solve_opts* opts, void* stream);

/* Continuous batching: advances the n hierarchies' solves without making
 * them wait for one another. A solve whose last enqueued phase has finished
 * on the device (its event has completed) gets its host part (Givens
 * rotations, stopping test) and its next phase enqueued at once; a solve
 * with nothing in flight gets its phase enqueued; a solve whose phase is
 * still running is left alone. If no solve could move in one pass, the call
 * waits until the first in-flight phase completes. With the environment
 * variable STK_CROSS_BATCH=1, solves of hierarchies with the same shape
 * (dimension, fine cells, levels, relaxation steps and precision /
 * preconditioner form) that are ready for an Arnoldi step at the same time
 * run their preconditioner cycles in lockstep, with one batched star-patch
 * solve launch per smoothing step of the levels below 512 workgroups for
 * all of them (up to STK_BATCH_MAX requests per launch); this pays on bursts
 * of same-shape small requests and is off by default, since on a mixed
 * stream the lockstep waits cost the other requests more than it gains.
 * Each solve's arithmetic is unchanged either way, so its result does not
 * depend on which other requests share the device.
 * Entries that are idle or done are skipped. Returns the first error met (that solve is then done with that
 * status); `stream` is unused. */
#define STK_BATCH_MAX 8
stk_status stk_step_batch(stk_hier* const* hs, int n, void* stream);

/* STK_EBUSY while the solve runs; otherwise fills info and returns the
 * solve's status (STK_OK, STK_ENOTCONV, STK_ENAN, ...). STK_EINVAL if no
 * solve was started. */
stk_status stk_poll(stk_hier* h, stk_solve_info* info);

/* Autotuning of the batched star-patch solve. The kernel exists in
 * STK_ASM_VARIANTS variants that differ only in how many packed inverse
 * elements a lane loads ahead (and so in registers and occupancy) and in
 * the cache policy of those loads (non-temporal in variant 3);
 * all perform the same multiply-adds in the same order, so results are
 * bit-identical whichever is chosen (the choice never changes a solution).
 * stk_autotune times every variant on every smoothed level (levels 1..L-1)
 * and precision in use (FP64; FP32 too if the hierarchy was set up with
 * mixed = 1) with HIP events around `reps` (1..100) back-to-back launches on
 * the level's own buffers, keeps the fastest per (level, precision), and
 * writes the choices to variants[(level - 1) * 2 + dtype] if variants is not
 * NULL (2 (L - 1) ints, -1 for a precision not in use) and the measured
 * average launch time of every variant to
 * times_ms[((level - 1) * 2 + dtype) * STK_ASM_VARIANTS + variant] if
 * times_ms is not NULL (entries of precisions not in use untouched). Timing
 * noise can make the choice differ between runs; for reproducible
 * measurements apply a recorded choice with stk_set_asm_variant instead
 * (the Python layer keeps such a table). Synchronous on
 * `stream`; drops the captured HIP graphs (they are re-captured on the next
 * solve). STK_EBUSY while a resumable solve is in progress.
 * stk_set_asm_variant fixes the variant of one (level, dtype) by hand
 * (0 <= variant < STK_ASM_VARIANTS; level >= 1). Default: variant 0. */
#define STK_ASM_VARIANTS 4
stk_status stk_autotune(stk_hier* h, int reps, int* variants, float* times_ms, void* stream);
stk_status stk_set_asm_variant(stk_hier* h, int level, int dtype, int variant);

/* Kernel timing (tracing). stk_profile(h, r), 1 <= r <= 100, clears the
 * records and starts bracketing launches of the instrumented kernel families
 * with HIP events on the launch stream; each instrumented launch is issued r
 * times back to back inside its bracket (both families are pure functions of
 * their inputs, so results are unchanged), which keeps event and launch
 * latency out of the per-launch average. stk_profile(h, 0) stops. stk_profile_read synchronises
 * the stream and returns, for family `kernel`, the number of launches, their
 * summed duration in ms and the summed algorithmic bytes:
 *   kernel 0: batched star-patch solve of the interior patches (all levels);
 *             bytes = packed inverses + patch outputs + one residual read;
 *   kernel 1: cell kernel of the A_gamma apply (all levels); bytes = velocity
 *             input + viscosity at Gauss points + element outputs;
 *   kernel 2: the launches of kernel 0 on the finest level only. */
stk_status stk_profile(stk_hier* h, int enable);
stk_status stk_profile_read(stk_hier* h, int kernel, int64_t* launches, double* total_ms,
                            double* total_bytes);

/* ---- Viscoplastic Newton loop (Section 5.3, the root of the algorithm
 * outline; hierarchy set up with coef_kind 2) ----
 * The nonlinear problem: find (u, p) with
 *   F_u = a(u; u) + gamma B^T W^{-1} B u + B^T p - b = 0,  F_p = B u = 0,
 *   a(w; v) = (2 mu_eff(eps_II(w)) eps(w), eps(v)),
 *   mu_eff  = mu_floor + min(mu0 - mu_floor, tau_y / (2 eps_II)),
 * mu0 the multi-sinker field, b = (f, phi_i) (stk_rhs). The augmented term
 * vanishes where B u = 0, so the solutions are those of the viscoplastic
 * Stokes problem. Its Jacobian at u_k is the augmented Stokes operator with
 * the fourth-order viscosity C = d tau / d eps at eps(u_k) (the law of
 * stk_viscoplastic), so every Newton step is one stk_solve on the hierarchy
 * relinearised at u_k. Readings: standard Newton (the paper's
 * stress-velocity variant differs in the tensor's rank-one term and needs an
 * update formula from another reference); coarse levels linearised at the
 * velocity injected to their nodes; x_0 = 0.
 *
 * stk_relinearize: coefficients (mu_eff, w) at the Gauss points of every
 * level from the FE velocity x_u of the finest level (stored layout;
 * injected to the coarser levels), then the star-patch inverses, the coarse
 * inverse and the Schur blocks rebuilt from them. Host-synchronous;
 * STK_ENOTSPD as for setup.
 * stk_nl_residual: (r_u, r_p) = (F_u, F_p) at (x_u, x_p) (stored layout,
 * Dirichlet entries 0; r_u must not alias x_u).
 * stk_newton: x = 0; until ||F|| <= rtol ||F(0)||: relinearise at x, solve
 * J d = -F with stk_solve (lin_rtol, restart, lin_maxit, pc, cycle, eager),
 * backtrack x + alpha d, alpha = 1, 1/2, .. until ||F|| <= (1 - 1e-4 alpha)
 * times the current norm (at most max_halvings halvings, the last trial is
 * taken regardless). Writes the last iterate to (x_u, x_p) and fills info;
 * STK_ENOTCONV after maxit steps, STK_ENAN for a non-finite residual.
 * Host-synchronous. */
#define STK_NEWTON_MAXIT 64
typedef struct {
  double rtol;        /* nonlinear residual reduction (default 1e-8) */
  int maxit;          /* Newton steps (default 30, at most STK_NEWTON_MAXIT) */
  double lin_rtol;    /* relative residual of each linear solve (default 1e-6) */
  int lin_maxit;      /* FGMRES iterations per step (default 300) */
  int restart;        /* FGMRES restart (default 30) */
  int max_halvings;   /* line-search halvings (default 10) */
  int pc;             /* as stk_solve_opts.pc */
  int cycle;          /* as stk_solve_opts.cycle */
  int eager;          /* as stk_solve_opts.eager */
} stk_newton_opts;

typedef struct {
  int iters;                            /* Newton steps taken */
  int converged;
  double rel_res;                       /* ||F(x)|| / ||F(0)|| at exit */
  double res0;                          /* ||F(0)|| */
  double t_s;                           /* wall time */
  double hist[STK_NEWTON_MAXIT + 1];    /* ||F|| / ||F(0)|| after each step */
  double alpha[STK_NEWTON_MAXIT];       /* accepted step length of each step */
  int lin_iters[STK_NEWTON_MAXIT];      /* FGMRES iterations of each step */
} stk_newton_info;

stk_status stk_relinearize(stk_hier* h, const double* x_u, void* stream);
stk_status stk_nl_residual(stk_hier* h, const double* x_u, const double* x_p, double* r_u, double* r_p,
                           void* stream);
stk_status stk_newton(stk_hier* h, double* x_u, double* x_p, const stk_newton_opts* opts, stk_newton_info* info,
                      void* stream);

/* Thread-local description of the last error (empty string if none). */
const char* stk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STK_H */
