// Host orchestration and the C ABI of libstk.so: hierarchy setup, the
// V-cycle with GMRES relaxation, the block preconditioner and FGMRES.
// Every device step is a hand-written kernel from the k_*.hip files; this file
// only allocates, sequences launches on the caller's stream and runs the
// small host-side Givens recurrences of FGMRES.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/stk.h"
#include "stk_reduce.h"
#include "stk_q3d.h"

using namespace stk;

struct stk_hier {
  Hier H;
};

namespace {

thread_local std::string g_err;

stk_status fail(stk_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(STK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define STKCHK(call)                  \
  do {                                \
    stk_status s_ = (call);           \
    if (s_ != STK_OK) return s_;      \
  } while (0)

constexpr int kPartialLen = kRedBlocks * 64;

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

stk_status validate(const stk_desc* d) {
  if (!d) return fail(STK_EINVAL, "desc is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(STK_EINVAL, "dim must be 2 or 3");
  if (d->n_levels < 2 || d->n_levels > 12) return fail(STK_EINVAL, "n_levels must be in [2, 12]");
  if (d->n_fine < 2 || d->n_fine % (1 << (d->n_levels - 1)) != 0)
    return fail(STK_EINVAL, "n_fine must be a positive multiple of 2^(n_levels-1)");
  if (d->n_fine > (d->dim == 2 ? 4096 : 256)) return fail(STK_EINVAL, "n_fine too large");
  if (d->degree != 0 && d->degree != 2 && d->degree != 3) return fail(STK_EINVAL, "degree must be 0, 2 or 3");
  const int deg = d->degree == 3 ? 3 : 2;
  if (deg == 3) {
    if (d->dim == 3 && d->n_fine > 32)
      return fail(STK_EINVAL, "degree 3 in 3D is built up to 32^3 cells (explicit 375-unknown patch inverses)");
    if (d->coef_kind != 0) return fail(STK_EINVAL, "degree 3 takes the scalar sinker viscosity (coef_kind 0)");
    if (d->mixed != 0) return fail(STK_EINVAL, "degree 3 has the FP64 form only (mixed 0)");
    if (d->qpts_1d != 0 && d->qpts_1d != 4)
      return fail(STK_EINVAL, "degree 3 uses the 4-point Gauss rule (qpts_1d 0 or 4)");
    if (d->n_fine > 2048) return fail(STK_EINVAL, "n_fine too large");
  }
  const int nc = d->n_fine >> (d->n_levels - 1);
  const int64_t n0 = (int64_t)d->dim * ipow(deg * nc - 1, d->dim);
  if (n0 > 80000) return fail(STK_EINVAL, "coarsest level too large for the dense coarse solve (80000 unknowns)");
  if (!(d->gamma >= 0.0) || !isfinite(d->gamma)) return fail(STK_EINVAL, "gamma must be finite and >= 0");
  if (d->schur != 1 && d->schur != 2) return fail(STK_EINVAL, "schur must be 1 (W = M_p) or 2 (W = M_p(1/mu))");
  if (d->coef_kind < 0 || d->coef_kind > 2)
    return fail(STK_EINVAL, "coef_kind must be 0 (sinker viscosity), 1 (viscoplastic Newton tensor at the "
                            "Fourier velocity) or 2 (viscoplastic law at an FE velocity state)");
  if (d->coef_kind == 2) {
    const stk_viscoplastic& v = d->vp;
    if (!(v.tau_y > 0.0) || !isfinite(v.tau_y)) return fail(STK_EINVAL, "vp.tau_y must be positive");
    if (!isfinite(v.mu_floor)) return fail(STK_EINVAL, "vp.mu_floor must be finite");
    if (d->schur != 1) return fail(STK_EINVAL, "the Newton state (coef_kind 2) needs W = M_p (schur = 1)");
  }
  if (deg == 2 && d->qpts_1d != 0 && d->qpts_1d != 3)
    return fail(STK_EINVAL, "qpts_1d must be 0 or 3 (the 3-point Gauss rule is the one built)");
  if (d->coef_kind == 1) {
    const stk_viscoplastic& v = d->vp;
    if (v.modes < 1 || v.modes > 8 || !v.amp) return fail(STK_EINVAL, "vp.modes must be in [1, 8] with vp.amp set");
    if (!(v.tau_y > 0.0) || !isfinite(v.tau_y)) return fail(STK_EINVAL, "vp.tau_y must be positive");
    if (!isfinite(v.eps_scale)) return fail(STK_EINVAL, "vp.eps_scale must be finite");
    if (!isfinite(v.mu_floor)) return fail(STK_EINVAL, "vp.mu_floor must be finite");
  }
  if (d->mixed != 0 && d->mixed != 1) return fail(STK_EINVAL, "mixed must be 0 (FP64 form) or 1 (mixed form)");
  if (d->nu_pre < 1 || d->nu_pre > kMaxNu || d->nu_post < 1 || d->nu_post > kMaxNu)
    return fail(STK_EINVAL, "nu_pre/nu_post must be in [1, 8]");
  const stk_sinker& s = d->sinker;
  if (s.n < 0 || s.n > 4096 || (s.n > 0 && !s.centers)) return fail(STK_EINVAL, "bad sinker list");
  if (!(s.mu_min > 0.0) || !(s.mu_max > 0.0)) return fail(STK_EINVAL, "viscosities must be positive");
  if (!(s.omega >= 0.0) || !(s.delta >= 0.0)) return fail(STK_EINVAL, "bad sinker shape parameters");
  return STK_OK;
}

// Patch classes of a level: sizes and counts (host arithmetic, used by the
// footprint and by setup).
struct ClassPlan {
  int n;
  std::vector<int> verts;
};

// Degree 3: one class of 50-unknown patches (boundary patches padded), the
// coarse-cell centre vertices first in lexicographic order of the coarse
// cell, then the other vertices in lexicographic order.
std::vector<ClassPlan> plan_patches_q3(int D, int N) {
  const int nv = N + 1, nc = N / 2;
  ClassPlan all{D == 2 ? 50 : 375, {}};
  if (D == 2) {
    for (int s = 0; s < nc * nc; ++s) all.verts.push_back((2 * (s % nc) + 1) + nv * (2 * (s / nc) + 1));
    for (int vert = 0; vert < nv * nv; ++vert) {
      const int v0 = vert % nv, v1 = vert / nv;
      if ((v0 & 1) && (v1 & 1)) continue;
      all.verts.push_back(vert);
    }
  } else {
    for (int s = 0; s < nc * nc * nc; ++s) {
      const int k0 = s % nc, k1 = (s / nc) % nc, k2 = s / (nc * nc);
      all.verts.push_back((2 * k0 + 1) + nv * ((2 * k1 + 1) + nv * (2 * k2 + 1)));
    }
    for (int vert = 0; vert < nv * nv * nv; ++vert) {
      const int v0 = vert % nv, v1 = (vert / nv) % nv, v2 = vert / (nv * nv);
      if ((v0 & 1) && (v1 & 1) && (v2 & 1)) continue;
      all.verts.push_back(vert);
    }
  }
  return {all};
}

std::vector<ClassPlan> plan_patches(int D, int N) {
  const int nv = N + 1;
  const int nvert = D == 2 ? nv * nv : nv * nv * nv;
  std::vector<ClassPlan> cls;
  ClassPlan inner{D * ipow(3, D), {}};
  // all-odd vertices first, in lexicographic order of K = (v-1)/2 (coarse cells)
  const int nc = N / 2;
  const int ncc = D == 2 ? nc * nc : nc * nc * nc;
  for (int s = 0; s < ncc; ++s) {
    const int k0 = s % nc, k1 = (s / nc) % nc, k2 = D == 3 ? s / (nc * nc) : 0;
    const int v0 = 2 * k0 + 1, v1 = 2 * k1 + 1, v2 = D == 3 ? 2 * k2 + 1 : 0;
    inner.verts.push_back(v0 + nv * (v1 + nv * v2));
  }
  std::vector<ClassPlan> bnd;
  for (int vert = 0; vert < nvert; ++vert) {
    int v[3] = {vert % nv, (vert / nv) % nv, D == 3 ? vert / (nv * nv) : 1};
    int clipped = 0;
    bool all_odd = true;
    for (int k = 0; k < D; ++k) {
      if (v[k] == 0 || v[k] == N) ++clipped;
      if ((v[k] & 1) == 0) all_odd = false;
    }
    if (clipped == 0) {
      if (!all_odd) inner.verts.push_back(vert);
      continue;
    }
    const int n = D * ipow(3, D - clipped);
    auto it = std::find_if(bnd.begin(), bnd.end(), [&](const ClassPlan& c) { return c.n == n; });
    if (it == bnd.end()) {
      bnd.push_back(ClassPlan{n, {}});
      it = bnd.end() - 1;
    }
    it->verts.push_back(vert);
  }
  cls.push_back(std::move(inner));
  std::sort(bnd.begin(), bnd.end(), [](const ClassPlan& a, const ClassPlan& b) { return a.n > b.n; });
  for (auto& c : bnd) cls.push_back(std::move(c));
  return cls;
}

int64_t packed_doubles(int n, int count) {
  const int64_t P = (int64_t)n * (n + 1) / 2;
  return ((int64_t)(count + 63) / 64) * 64 * P;
}

// Walks every allocation of a hierarchy; `alloc(bytes, ptr_to_store)`.
template <class F>
stk_status plan_allocs(const stk_desc* d, Hier& H, F&& alloc, bool build_classes) {
  const int D = d->dim;
  const int deg = d->degree == 3 ? 3 : 2;
  const int NN = ipow(deg + 1, D), NL = D * NN, NP = deg == 3 ? (D == 2 ? 6 : 10) : D + 1;
  const bool q3d = deg == 3 && D == 3;   // 375-unknown patches: tile-layout inverses
  int64_t q3ws = 0;                      // doubles of the 3D degree-3 setup workspace
  const int PU = D * ipow(2 * deg - 1, D);   // unknowns of an interior star patch
  H.dim = D;
  H.deg = deg;
  H.L = d->n_levels;
  H.lv.assign(H.L, Level{});
  for (int l = 0; l < H.L; ++l) {
    Level& L = H.lv[l];
    const int N = d->n_fine >> (H.L - 1 - l);
    L.g.N = N;
    L.g.n1 = deg * N + 1;
    L.g.nnodes = D == 2 ? (int64_t)L.g.n1 * L.g.n1 : (int64_t)L.g.n1 * L.g.n1 * L.g.n1;
    L.g.ncell = D == 2 ? (int64_t)N * N : (int64_t)N * N * N;
    L.g.h = 1.0 / N;
    L.nvert = D == 2 ? (N + 1) * (N + 1) : (N + 1) * (N + 1) * (N + 1);
    L.nvel = D * L.g.nnodes;
    L.npres = NP * L.g.ncell;
    STKCHK(alloc((size_t)NN * L.g.ncell * 8, (void**)&L.mu));
    if (d->mixed) STKCHK(alloc((size_t)NN * L.g.ncell * 4, (void**)&L.mu32));
    if (d->schur == 2) {
      STKCHK(alloc((size_t)NP * NP * L.g.ncell * 8, (void**)&L.winv));
      if (d->mixed) STKCHK(alloc((size_t)NP * NP * L.g.ncell * 4, (void**)&L.winv32));
    }
    if (d->coef_kind >= 1) {
      const int NS = D * (D + 1) / 2;
      STKCHK(alloc((size_t)NS * NN * L.g.ncell * 8, (void**)&L.cw));
      if (d->mixed) STKCHK(alloc((size_t)NS * NN * L.g.ncell * 4, (void**)&L.cw32));
    }
    STKCHK(alloc((size_t)NL * L.g.ncell * 8, (void**)&L.E));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.b));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.x));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.r));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.T));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.U));
    STKCHK(alloc((size_t)L.nvel * 8, (void**)&L.S));
    if (d->mixed) STKCHK(alloc((size_t)L.nvel * 4, (void**)&L.S32));
    STKCHK(alloc((size_t)kSmallLen * 8, (void**)&L.small));
    if (l >= 1) {
      STKCHK(alloc((size_t)(kMaxNu + 1) * L.nvel * 8, (void**)&L.V));
      STKCHK(alloc((size_t)kMaxNu * L.nvel * 8, (void**)&L.Z));
      STKCHK(alloc((size_t)PU * L.nvert * 8, (void**)&L.zbuf));
      std::vector<ClassPlan> plan = deg == 3 ? plan_patches_q3(D, N) : plan_patches(D, N);
      L.cls.assign(plan.size(), PatchClass{});
      for (size_t c = 0; c < plan.size(); ++c) {
        L.cls[c].n = plan[c].n;
        L.cls[c].count = (int)plan[c].verts.size();
        STKCHK(alloc(plan[c].verts.size() * 4, (void**)&L.cls[c].verts));
        if (q3d) {
          // 21 tiles of 64 x 64 per patch (384 padded unknowns), the 6
          // diagonal ones stored as their lower 4 x 4 blocks
          STKCHK(alloc((size_t)L.cls[c].count * stk::q3d::PS * 8, (void**)&L.cls[c].inv));
          // setup: the level's cell matrices, then one pass of full tiles and the sweep's work
          const int64_t pass = std::min<int64_t>(L.cls[c].count, stk::q3d::kPatchBatch);
          q3ws = std::max(q3ws, (int64_t)L.g.ncell * NL * NL + pass * (stk::q3d::TS + 7 * 4096));
          continue;
        }
        STKCHK(alloc((size_t)packed_doubles(plan[c].n, L.cls[c].count) * 8, (void**)&L.cls[c].inv));
        if (d->mixed)
          STKCHK(alloc((size_t)packed_doubles(plan[c].n, L.cls[c].count) * 4, (void**)&L.cls[c].inv32));
      }
    }
  }
  const Level& L0 = H.lv[0];
  H.n0 = (int64_t)D * ipow(deg * L0.g.N - 1, D);
  if (q3d) {
    q3ws = std::max(q3ws, (int64_t)L0.g.ncell * NL * NL);
    STKCHK(alloc((size_t)q3ws * 8, (void**)&H.q3cm));
  }
  {
    const size_t nb = (size_t)coarse_tiles(H.n0);
    STKCHK(alloc(nb * (nb + 1) / 2 * 4096 * 8, (void**)&H.Ainv0));
    STKCHK(alloc((2 * nb + 1) * 4096 * 8, (void**)&H.cwork));
    STKCHK(alloc(nb * 64 * 8, (void**)&H.cvec));
    STKCHK(alloc(nb * nb * 64 * 8, (void**)&H.cpart));
  }
  const Level& Lf = H.lv[H.L - 1];
  STKCHK(alloc((size_t)Lf.g.ncell * NP * NP * 8, (void**)&H.Sinv));
  STKCHK(alloc((size_t)2 * kPartialLen * 8, (void**)&H.partials));
  STKCHK(alloc(64, (void**)&H.flag));
  STKCHK(alloc((size_t)std::max(1, d->sinker.n) * D * 8, (void**)&H.centers));
  if (d->coef_kind == 1) STKCHK(alloc((size_t)D * ipow(d->vp.modes, D) * 8, (void**)&H.vp_amp));
  // FGMRES storage for the default restart length 30
  const int m = 30;
  const int64_t nvec = Lf.nvel + Lf.npres;
  H.restart_alloc = m;
  STKCHK(alloc((size_t)(m + 1) * nvec * 8, (void**)&H.fV));
  STKCHK(alloc((size_t)m * nvec * 8, (void**)&H.fZ));
  STKCHK(alloc((size_t)nvec * 8, (void**)&H.fw));
  STKCHK(alloc((size_t)2 * nvec * 8, (void**)&H.fr));
  STKCHK(alloc((size_t)(m + 1) * m * 8, (void**)&H.fH));
  STKCHK(alloc((size_t)64 * 8, (void**)&H.fy));
  STKCHK(alloc((size_t)Lf.nvel * 8, (void**)&H.pw_u));
  STKCHK(alloc((size_t)Lf.nvel * 8, (void**)&H.pw_y));
  H.mixed = d->mixed;
  if (d->mixed) {
    STKCHK(alloc((size_t)Lf.nvel * 8, (void**)&H.mb));
    STKCHK(alloc((size_t)Lf.nvel * 8, (void**)&H.mx));
  }
  if (d->coef_kind == 2) {
    STKCHK(alloc((size_t)NN * Lf.g.ncell * 8, (void**)&H.mu0));
    STKCHK(alloc((size_t)nvec * 8, (void**)&H.nl_b));
    STKCHK(alloc((size_t)nvec * 8, (void**)&H.nl_F));
    STKCHK(alloc((size_t)nvec * 8, (void**)&H.nl_d));
    STKCHK(alloc((size_t)nvec * 8, (void**)&H.nl_x));
    STKCHK(alloc((size_t)nvec * 8, (void**)&H.nl_t));
  }
  (void)build_classes;
  return STK_OK;
}

void free_all(Hier& H) {
  for (void* p : H.allocs) (void)hipFree(p);
  H.allocs.clear();
}

// ---------------------------------------------------------------------------
// Operators on a level (all asynchronous on H.stream), templated on the
// storage type R of the level vectors: double (FP64 form) or float (the
// V-cycle of the mixed form). Level work buffers are sized for doubles and
// the FP32 path reuses their memory wherever every use writes the entries it
// later reads; buffers with entries that must stay zero get FP32 copies.
template <class R>
R* rv(double* p) {
  return reinterpret_cast<R*>(p);
}

// buffer of the restriction's local solves (zero outside the coarse-cell interiors)
template <class R>
R* level_S(Level& L);
template <>
double* level_S<double>(Level& L) {
  return L.S;
}
template <>
float* level_S<float>(Level& L) {
  return L.S32;
}

// ---------------------------------------------------------------------------
// Lockstep batching of the star-patch solves across hierarchies (serving).
// Hierarchies whose Arnoldi steps issue the same sequence of patch-solve
// calls each run their step on their own host thread and stream; at every
// patch-solve call the threads meet, the last to arrive issues one batched
// launch for all of them on the first entry's stream (after every entry's
// stream has reached the call, through events), and each stream waits for
// that launch before going on. Everything else stays on each hierarchy's
// own stream, and each entry's patch solves run exactly the single-launch
// code, so results do not depend on the batch. The threads meet at a
// spinning barrier (a step has dozens of meetings of a few microseconds of
// host work each) and come from a persistent pool.
struct Cohort {
  int n = 0;
  std::atomic<int> arrived{0};
  std::atomic<long> gen{0};
  // a member whose step failed never arrives again: the others then launch
  // their own patch solves
  std::atomic<bool> broken{false};
  hipStream_t lead = nullptr;
  hipEvent_t done = nullptr;
  std::vector<const Hier*> hs;
  std::vector<const Level*> ls;
  std::vector<const void*> rs;
  std::vector<hipEvent_t> ready;
};
thread_local Cohort* t_cohort = nullptr;
thread_local int t_slot = -1;

// Workgroups of one entry of a batched patch-solve launch (64 patches per
// workgroup, 256 for the 3D boundary classes). Levels at or above
// kCohortMaxBlocks fill the device on their own and are launched without
// meeting the cohort.
constexpr int kCohortMaxBlocks = 512;
int asm_blocks(const Hier& H, const Level& L) {
  int blocks = 0;
  const int ncls = H.dim == 2 ? 3 : 4;
  for (int ci = 0; ci < ncls && ci < (int)L.cls.size(); ++ci) {
    const int per = (H.dim == 2 || ci == 0) ? 64 : 256;
    blocks += (L.cls[ci].count + per - 1) / per;
  }
  return blocks;
}

// Persistent worker threads for the cohorts: run(tasks) runs tasks[1..] on
// the workers and tasks[0] on the caller, and returns when all have ended.
class CohortPool {
 public:
  void run(std::vector<std::function<void()>>& tasks) {
    const int nw = (int)tasks.size() - 1;
    {
      std::unique_lock<std::mutex> lk(m_);
      while ((int)th_.size() < nw) th_.emplace_back([this] { work(); });
      for (int i = 1; i <= nw; ++i) q_.push_back(&tasks[i]);
      left_ = nw;
    }
    cv_.notify_all();
    tasks[0]();
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [this] { return left_ == 0; });
  }
  ~CohortPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (std::thread& t : th_) t.join();
  }

 private:
  void work() {
    for (;;) {
      std::function<void()>* f = nullptr;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [this] { return stop_ || !q_.empty(); });
        if (stop_ && q_.empty()) return;
        f = q_.back();
        q_.pop_back();
      }
      (*f)();
      std::lock_guard<std::mutex> lk(m_);
      if (--left_ == 0) done_.notify_all();
    }
  }
  std::mutex m_;
  std::condition_variable cv_, done_;
  std::vector<std::thread> th_;
  std::vector<std::function<void()>*> q_;
  int left_ = 0;
  bool stop_ = false;
};

// The patch solves of one ASM application into L.zbuf (batched with the
// other members of the calling thread's cohort, if any).
template <class R>
void asm_solves(Hier& H, Level& L, const R* r) {
  Cohort* C = t_cohort;
  // members have the same level shapes, so they all take the same branch
  if (!C || C->broken.load(std::memory_order_acquire) || H.deg == 3 || asm_blocks(H, L) >= kCohortMaxBlocks) {
    launch_asm_solves<R>(H, L, r, H.stream);
    return;
  }
  const int k = t_slot;
  (void)hipEventRecord(C->ready[k], H.stream);
  C->ls[k] = &L;
  C->rs[k] = r;
  // the generation cannot move before this member has arrived
  const long g = C->gen.load(std::memory_order_acquire);
  if (C->arrived.fetch_add(1, std::memory_order_acq_rel) + 1 == C->n) {
    for (int i = 0; i < C->n; ++i) (void)hipStreamWaitEvent(C->lead, C->ready[i], 0);
    std::vector<const R*> rr(C->n);
    for (int i = 0; i < C->n; ++i) rr[i] = static_cast<const R*>(C->rs[i]);
    launch_asm_gemv_batch<R>(C->hs.data(), C->ls.data(), rr.data(), C->n, C->lead);
    (void)hipEventRecord(C->done, C->lead);
    C->arrived.store(0, std::memory_order_relaxed);
    C->gen.fetch_add(1, std::memory_order_release);
  } else {
    while (C->gen.load(std::memory_order_acquire) == g) {
      if (C->broken.load(std::memory_order_acquire)) {
        // this generation can no longer fill up
        launch_asm_solves<R>(H, L, r, H.stream);
        return;
      }
      std::this_thread::yield();
    }
  }
  (void)hipStreamWaitEvent(H.stream, C->done, 0);
}

template <class R>
void apply_A(Hier& H, int l, const R* x, R* y) {
  Level& L = H.lv[l];
  hipEvent_t ev = nullptr;
  const int reps = prof_begin(H, H.stream, &ev);
  // pure function of x -> element buffer: a profiled call may repeat it
  for (int k = 0; k < reps; ++k) launch_elem<R>(H, L, EL_VISC | EL_AUG, x, nullptr, nullptr, H.stream);
  // algorithmic bytes of the cell kernel: u, coefficients at Gauss points, element outputs
  {
    const double nn = (double)ipow(H.deg + 1, H.dim);   // Gauss points (= nodes) per cell
    const double ncoef = L.cw ? 1.0 + H.dim * (H.dim + 1) / 2 : 1.0;   // mu [and w] per Gauss point
    prof_end(H, H.stream, PROF_ELEM, ev,
             (double)sizeof(R) * ((double)L.nvel + (double)L.g.ncell * (ncoef * nn + H.dim * nn)), reps);
  }
  launch_gather<R>(H, L, nullptr, 1.0, y, H.stream);
}

// y = A_gamma x with the partial dot products V_k . y (k < nk) for the
// Gram-Schmidt step that follows, on the partition of launch_dots.
template <class R>
void apply_A_dots(Hier& H, int l, const R* x, R* y, const R* V, int64_t ldv, int nk, double* part) {
  Level& L = H.lv[l];
  hipEvent_t ev = nullptr;
  const int reps = prof_begin(H, H.stream, &ev);
  for (int k = 0; k < reps; ++k) launch_elem<R>(H, L, EL_VISC | EL_AUG, x, nullptr, nullptr, H.stream);
  {
    const double nn = (double)ipow(H.deg + 1, H.dim);
    const double ncoef = L.cw ? 1.0 + H.dim * (H.dim + 1) / 2 : 1.0;
    prof_end(H, H.stream, PROF_ELEM, ev,
             (double)sizeof(R) * ((double)L.nvel + (double)L.g.ncell * (ncoef * nn + H.dim * nn)), reps);
  }
  launch_gather_dots<R>(H, L, y, L.nvel, V, ldv, nk, part, H.stream);
}

// 2D smoother step: z = M^{-1} v (ASM) and y = A z with the partial dots of
// y against V, the sum of the patch outputs formed inside the cell kernel.
template <class R>
void asm_apply_A_dots(Hier& H, int l, const R* v, R* z, R* y, const R* V, int64_t ldv, int nk, double* part) {
  Level& L = H.lv[l];
  asm_solves<R>(H, L, v);
  hipEvent_t ev = nullptr;
  const int reps = prof_begin(H, H.stream, &ev);
  for (int k = 0; k < reps; ++k) launch_elem_asm<R>(H, L, z, H.stream);
  {
    // algorithmic bytes: patch outputs read, z written, coefficients and
    // element vectors of every cell
    const double nn = (double)ipow(H.deg + 1, 2);
    const double ncoef = L.cw ? 4.0 : 1.0;
    prof_end(H, H.stream, PROF_ELEM, ev,
             (double)sizeof(R) * (2.0 * nn * (double)L.nvert + (double)L.nvel +
                                  (double)L.g.ncell * (ncoef * nn + 2.0 * nn)),
             reps);
  }
  launch_gather_dots<R>(H, L, y, L.nvel, V, ldv, nk, part, H.stream);
}

template <class R>
void residual(Hier& H, int l, const R* b, const R* x, R* r) {
  Level& L = H.lv[l];
  launch_elem<R>(H, L, EL_VISC | EL_AUG, x, nullptr, nullptr, H.stream);
  launch_gather<R>(H, L, b, -1.0, r, H.stream);
}

// rc = P~^T rf (fine level l -> l-1)
template <class R>
void restrict_robust(Hier& H, int l, const R* rf, R* rc) {
  Level& F = H.lv[l];
  Level& C = H.lv[l - 1];
  R* S = level_S<R>(F);
  R* U = rv<R>(F.U);
  launch_center_solve<R>(H, F, rf, S, 1.0, false, H.stream);          // S|_K = A_K^{-1} rf|_K
  launch_elem<R>(H, F, EL_AUG, S, nullptr, nullptr, H.stream);         // G S
  launch_gather<R>(H, F, rf, -1.0, U, H.stream);                       // U = rf - G S
  launch_restrict_std<R>(H, F, C, U, rc, H.stream);                    // rc = P_H^T U
}

// xf = P~ xc (coarse level l-1 -> fine level l)
template <class R>
void prolong_robust(Hier& H, int l, const R* xc, R* xf) {
  Level& F = H.lv[l];
  Level& C = H.lv[l - 1];
  R* U = rv<R>(F.U);
  launch_prolong_std<R>(H, C, F, xc, xf, H.stream);                    // xf = P_H xc
  launch_elem<R>(H, F, EL_AUG, xf, nullptr, nullptr, H.stream);
  launch_gather<R>(H, F, nullptr, 1.0, U, H.stream);                   // U = G xf
  launch_center_solve<R>(H, F, U, xf, -1.0, true, H.stream);           // xf|_K -= A_K^{-1} U|_K
}

// nu steps of right-preconditioned GMRES relaxation on A x = b.
template <class R>
void smooth(Hier& H, int l, const R* b, R* x, int nu, bool x_zero) {
  Level& L = H.lv[l];
  const int64_t n = L.nvel;
  double* p1 = H.partials;
  double* p2 = H.partials + kPartialLen;
  R* V = rv<R>(L.V);
  R* Z = rv<R>(L.Z);
  const R* r0 = b;
  if (!x_zero) {
    residual<R>(H, l, b, x, rv<R>(L.r));
    r0 = rv<R>(L.r);
  }
  launch_dots<R>(r0, n, 1, r0, n, p1, H.stream);
  launch_normalize<R>(p1, const_cast<R*>(r0), n, V, L.small + kSmallBeta, H.stream);
  for (int j = 0; j < nu; ++j) {
    R* Vj = V + (int64_t)j * n;
    R* Zj = Z + (int64_t)j * n;
    R* w = V + (int64_t)(j + 1) * n;
    if (H.dim == 2) {
      asm_apply_A_dots<R>(H, l, Vj, Zj, w, V, n, j + 1, p1);
    } else {
      asm_solves<R>(H, L, Vj);
      launch_asm_gather<R>(H, L, reinterpret_cast<const R*>(L.zbuf), Zj, H.stream);
      apply_A_dots<R>(H, l, Zj, w, V, n, j + 1, p1);
    }
    double* Hcol = L.small + kSmallH + j;
    launch_orth_update<R>(V, n, j + 1, w, n, p1, Hcol, kMaxNu, false, p2, true, H.stream);
    launch_orth_update<R>(V, n, j + 1, w, n, p2, Hcol, kMaxNu, true, p1, false, H.stream);
    // the last Arnoldi vector is not needed: its norm goes straight to the update
    if (j + 1 < nu) launch_normalize<R>(p1, w, n, w, L.small + kSmallH + (j + 1) * kMaxNu + j, H.stream);
  }
  launch_relax_update<R>(Z, n, nu, L.small, p1, x, n, x_zero, H.stream);
}

template <class R>
void coarse_solve(Hier& H, const R* b, R* x) {
  launch_coarse_apply<R>(H, H.lv[0], b, x, H.stream);
}

// One V-cycle on level l: x = V(b), from x = 0 (x_zero) or from the x passed
// in. The coarsest level is solved directly (its initial guess is unused).
template <class R>
void vcycle(Hier& H, int l, const R* b, R* x, bool x_zero = true) {
  if (l == 0) {
    coarse_solve<R>(H, b, x);
    return;
  }
  Level& L = H.lv[l];
  Level& C = H.lv[l - 1];
  smooth<R>(H, l, b, x, H.nu_pre, x_zero);
  residual<R>(H, l, b, x, rv<R>(L.r));
  restrict_robust<R>(H, l, rv<R>(L.r), rv<R>(C.b));
  vcycle<R>(H, l - 1, rv<R>(C.b), rv<R>(C.x));
  prolong_robust<R>(H, l, rv<R>(C.x), rv<R>(L.T));
  launch_axpby<R>(1.0, x, 1.0, rv<R>(L.T), x, L.nvel, H.stream);
  smooth<R>(H, l, b, x, H.nu_post, false);
}

// F-cycle on level lf (the "full" multigrid cycle of Section 5.1 and the
// algorithm outline, in the form of PETSc's full multigrid): b restricted to
// every coarser level with P~^T, the coarsest level solved, then on each
// finer level the prolongated (P~) coarser result improved by one V-cycle
// started from it. Level l's right-hand side and result live in lv[l].b and
// lv[l].x, which the V-cycles of finer levels only overwrite after use.
template <class R>
void fcycle(Hier& H, int lf, const R* b, R* x) {
  if (lf == 0) {
    coarse_solve<R>(H, b, x);
    return;
  }
  const R* bl = b;
  for (int l = lf; l >= 1; --l) {
    restrict_robust<R>(H, l, bl, rv<R>(H.lv[l - 1].b));
    bl = rv<R>(H.lv[l - 1].b);
  }
  coarse_solve<R>(H, rv<R>(H.lv[0].b), rv<R>(H.lv[0].x));
  for (int l = 1; l <= lf; ++l) {
    R* xl = l == lf ? x : rv<R>(H.lv[l].x);
    const R* bb = l == lf ? b : rv<R>(H.lv[l].b);
    prolong_robust<R>(H, l, rv<R>(H.lv[l - 1].x), xl);
    vcycle<R>(H, l, bb, xl, false);
  }
}

template <class R>
void cycle(Hier& H, int l, const R* b, R* x, bool f) {
  if (f) fcycle<R>(H, l, b, x);
  else vcycle<R>(H, l, b, x);
}

// Ahat^{-1} applied to an FP64 fine-level vector: one V- or F-cycle in FP64,
// or in the mixed form one FP32 cycle (FP32 applies, transfers and patch
// solves; FP64 coarse solve and small least-squares problems) between
// conversions.
void vcycle_fine(Hier& H, const double* b, double* x, bool mixed, bool f) {
  const int lf = H.L - 1;
  if (!mixed) {
    cycle<double>(H, lf, b, x, f);
    return;
  }
  const int64_t n = H.lv[lf].nvel;
  float* b32 = reinterpret_cast<float*>(H.mb);
  float* x32 = reinterpret_cast<float*>(H.mx);
  launch_convert<double, float>(b, b32, n, H.stream);
  cycle<float>(H, lf, b32, x32, f);
  launch_convert<float, double>(x32, x, n, H.stream);
}

// (z_u, z_p) = P (v_u, v_p), eq. (precond) with Ahat^{-1} = one V-cycle, or
// (upper) its block upper-triangular part: z_p = -Shat^{-1} v_p (mean
// removed), z_u = Ahat^{-1} (v_u - B^T z_p): one V-cycle per application.
void precond(Hier& H, const double* vu, const double* vp, double* zu, double* zp, bool mixed, bool upper,
             bool f) {
  const int lf = H.L - 1;
  Level& F = H.lv[lf];
  if (upper) {
    launch_schur_apply(H, F, nullptr, vp, zp, H.stream);             // z_p = -Shat^{-1} v_p
    launch_project_mean(H, F, zp, H.stream);
    launch_elem<double>(H, F, EL_BT, nullptr, zp, nullptr, H.stream);
    launch_gather<double>(H, F, vu, -1.0, H.pw_u, H.stream);         // v_u - B^T z_p
    vcycle_fine(H, H.pw_u, zu, mixed, f);
    return;
  }
  vcycle_fine(H, vu, H.pw_y, mixed, f);                           // y = Ahat^{-1} v_u
  launch_schur_apply(H, F, H.pw_y, vp, zp, H.stream);             // z_p = -Shat^{-1}(v_p - B y)
  launch_project_mean(H, F, zp, H.stream);
  launch_elem<double>(H, F, EL_BT, nullptr, zp, nullptr, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, H.pw_u, H.stream);   // B^T z_p
  vcycle_fine(H, H.pw_u, zu, mixed, f);                           // Ahat^{-1} B^T z_p
  launch_axpby<double>(1.0, H.pw_y, -1.0, zu, zu, F.nvel, H.stream);  // z_u = y - that
}

// y = K x on the finest level; x, y contiguous [u | p].
void stokes_apply(Hier& H, const double* x, double* y) {
  Level& F = H.lv[H.L - 1];
  launch_elem<double>(H, F, EL_VISC | EL_AUG | EL_BT | EL_BOUT, x, x + F.nvel, y + F.nvel, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, y, H.stream);
}

// One FGMRES Arnoldi step j with restart m: Z_j = P V_j, w = K Z_j,
// classical Gram-Schmidt twice against V_0..V_j, V_{j+1} = w/||w||, H column j.
void arnoldi_step(Hier& H, int j, int m, int64_t nu, int64_t nvec, bool mixed, bool upper, bool f) {
  double* Vj = H.fV + (int64_t)j * nvec;
  double* Zj = H.fZ + (int64_t)j * nvec;
  double* w = H.fV + (int64_t)(j + 1) * nvec;
  double* p1 = H.partials;
  double* p2 = H.partials + kPartialLen;
  precond(H, Vj, Vj + nu, Zj, Zj + nu, mixed, upper, f);
  // w = K Z_j with the first Gram-Schmidt pass's dot products
  Level& F = H.lv[H.L - 1];
  launch_elem<double>(H, F, EL_VISC | EL_AUG | EL_BT | EL_BOUT, Zj, Zj + nu, w + nu, H.stream);
  launch_gather_dots<double>(H, F, w, nvec, H.fV, nvec, j + 1, p1, H.stream);
  launch_orth_update<double>(H.fV, nvec, j + 1, w, nvec, p1, H.fH + j, m, false, p2, true, H.stream);
  launch_orth_update<double>(H.fV, nvec, j + 1, w, nvec, p2, H.fH + j, m, true, p1, false, H.stream);
  launch_normalize<double>(p1, w, nvec, w, H.fH + (j + 1) * m + j, H.stream);
}

void drop_graphs(Hier& H) {
  for (hipGraphExec_t g : H.steps)
    if (g) (void)hipGraphExecDestroy(g);
  H.steps.clear();
  H.steps_m = 0;
}

stk_status check_dtype(const Hier& H, int dtype) {
  if (dtype == STK_F64) return STK_OK;
  if (dtype == STK_F32 && H.mixed) return STK_OK;
  return fail(STK_EINVAL, dtype == STK_F32 ? "STK_F32 needs a hierarchy set up with mixed=1" : "unknown dtype");
}

bool solve_busy(const Hier& H) {
  return H.sv.phase == Hier::SV_ARNOLDI || H.sv.phase == Hier::SV_RESIDUAL || H.sv.phase == Hier::SV_FINISH;
}

stk_status check_level(const Hier& H, int l, int lmin) {
  if (l < lmin || l >= H.L) return fail(STK_EINVAL, "level out of range");
  return STK_OK;
}

stk_status device_norm(Hier& H, const double* x, int64_t n, double* out) {
  launch_dots<double>(x, n, 1, x, n, H.partials, H.stream);
  const int np = red_parts(n);
  std::vector<double> part(np);
  HIPCHK(hipMemcpyAsync(part.data(), H.partials, np * 8, hipMemcpyDeviceToHost, H.stream));
  HIPCHK(hipStreamSynchronize(H.stream));
  double s = 0.0;
  for (int b = 0; b < np; ++b) s += part[b];
  *out = sqrt(s);
  return STK_OK;
}

// Everything the coefficients at the Gauss points determine: the W = M_p(1/mu)
// blocks (P2), the star-patch inverses of levels >= 1, the FP32 copies (mixed
// form), the coarse inverse and the Schur blocks; host-synchronous, with the
// factorisations' pivot check (STK_ENOTSPD).
stk_status build_operators(Hier& H, hipStream_t s) {
  const int D = H.dim;
  launch_fill_int(H.flag, 0, 16, s);
  for (int l = 0; l < H.L; ++l) {
    Level& L = H.lv[l];
    if (L.winv) launch_winv_setup(H, L, s);
    if (l >= 1)
      for (PatchClass& pc : L.cls) launch_patch_setup(H, L, pc, s);
  }
  if (H.mixed) {
    // FP32 copies for the mixed form, rounded from the FP64 factors
    for (int l = 0; l < H.L; ++l) {
      Level& L = H.lv[l];
      launch_convert<double, float>(L.mu, L.mu32, (int64_t)(D == 2 ? 9 : 27) * L.g.ncell, s);
      if (L.cw)
        launch_convert<double, float>(L.cw, L.cw32, (int64_t)(D * (D + 1) / 2) * (D == 2 ? 9 : 27) * L.g.ncell, s);
      if (L.winv) launch_convert<double, float>(L.winv, L.winv32, (int64_t)(D + 1) * (D + 1) * L.g.ncell, s);
      for (PatchClass& pc : L.cls)
        launch_convert<double, float>(pc.inv, pc.inv32, packed_doubles(pc.n, pc.count), s);
    }
  }
  launch_coarse_assemble(H, H.lv[0], H.Ainv0, s);
  launch_coarse_invert(H, H.Ainv0, H.n0, H.cwork, s);
  launch_schur_setup(H, H.lv[H.L - 1], s);
  if (hipGetLastError() != hipSuccess) return fail(STK_EDEVICE, "kernel launch failed while building the operators");
  int flag = 0;
  if (hipMemcpyAsync(&flag, H.flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(STK_EDEVICE, "synchronisation failed while building the operators");
  if (flag) return fail(STK_ENOTSPD, "non-positive pivot in a patch or coarse factorisation");
  return STK_OK;
}

}  // namespace

namespace stk {

void set_last_error(const std::string& msg) { g_err = msg; }

int prof_begin(Hier& H, hipStream_t s, hipEvent_t* ev) {
  *ev = nullptr;
  if (!H.prof.on) return 1;
  Prof& P = H.prof;
  while (P.pool.size() < P.used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return 1;
    P.pool.push_back(e);
  }
  *ev = P.pool[P.used++];
  (void)hipEventRecord(*ev, s);
  return P.reps;
}

void prof_end(Hier& H, hipStream_t s, int id, hipEvent_t a, double bytes, int reps) {
  if (!H.prof.on || !a) return;
  Prof& P = H.prof;
  hipEvent_t b = P.pool[P.used++];
  (void)hipEventRecord(b, s);
  P.recs.push_back(Prof::Rec{id, a, b, bytes * reps, reps});
}

}  // namespace stk

// =========================================================================== C ABI
extern "C" {

const char* stk_last_error(void) { return g_err.c_str(); }

stk_status stk_footprint(const stk_desc* desc, size_t* bytes) {
  STKCHK(validate(desc));
  if (!bytes) return fail(STK_EINVAL, "bytes is NULL");
  Hier H;
  size_t total = 0;
  auto count = [&](size_t b, void** p) -> stk_status {
    total += (b + 255) / 256 * 256;
    *p = nullptr;
    return STK_OK;
  };
  STKCHK(plan_allocs(desc, H, count, false));
  *bytes = total;
  return STK_OK;
}

stk_status stk_setup_hierarchy(const stk_desc* desc, void* stream, stk_hier** out) {
  if (!out) return fail(STK_EINVAL, "out is NULL");
  *out = nullptr;
  STKCHK(validate(desc));
  size_t need = 0;
  STKCHK(stk_footprint(desc, &need));
  if (desc->hbm_budget && need > desc->hbm_budget)
    return fail(STK_ENOMEM, "footprint " + std::to_string(need) + " B exceeds budget " +
                                std::to_string(desc->hbm_budget) + " B");
  stk_hier* h = new stk_hier();
  Hier& H = h->H;
  H.stream = (hipStream_t)stream;
  H.nu_pre = desc->nu_pre;
  H.nu_post = desc->nu_post;
  H.gamma = desc->gamma;
  H.schur = desc->schur;
  H.n_sinkers = desc->sinker.n;
  H.omega = desc->sinker.omega;
  H.delta = desc->sinker.delta;
  H.mu_min = desc->sinker.mu_min;
  H.mu_max = desc->sinker.mu_max;
  H.beta = desc->sinker.beta;
  H.coef_kind = desc->coef_kind;
  if (H.coef_kind == 2) {
    H.vp_tau_y = desc->vp.tau_y;
    H.vp_floor = desc->vp.mu_floor > 0.0 ? desc->vp.mu_floor : desc->sinker.mu_min;
  }
  if (H.coef_kind == 1) {
    H.vp_modes = desc->vp.modes;
    H.vp_tau_y = desc->vp.tau_y;
    H.vp_scale = desc->vp.eps_scale;
    H.vp_floor = desc->vp.mu_floor > 0.0 ? desc->vp.mu_floor : desc->sinker.mu_min;
  }
  auto dev_alloc = [&](size_t b, void** p) -> stk_status {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(b, 8));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(STK_ENOMEM, "hipMalloc of " + std::to_string(b) + " B failed");
    }
    H.allocs.push_back(q);
    H.bytes += b;
    *p = q;
    return STK_OK;
  };
  stk_status st = plan_allocs(desc, H, dev_alloc, true);
  if (st != STK_OK) {
    free_all(H);
    delete h;
    return st;
  }
  auto bail = [&](stk_status s2) {
    (void)hipStreamSynchronize(H.stream);
    if (H.own) (void)hipStreamDestroy(H.own);
    free_all(H);
    delete h;
    return s2;
  };
  const int D = H.dim;
  hipStream_t s = H.stream;
  if (hipStreamCreateWithFlags(&H.own, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(STK_EDEVICE, "stream creation failed"));
  if (desc->sinker.n > 0 &&
      hipMemcpyAsync(H.centers, desc->sinker.centers, (size_t)desc->sinker.n * D * 8, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return bail(fail(STK_EDEVICE, "copy of sinker centres failed"));
  if (H.coef_kind == 1 &&
      hipMemcpyAsync(H.vp_amp, desc->vp.amp, (size_t)D * ipow(H.vp_modes, D) * 8, hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return bail(fail(STK_EDEVICE, "copy of the Fourier amplitudes failed"));
  launch_fill_int(H.flag, 0, 16, s);
  if (H.coef_kind == 1 && !(H.vp_scale > 0.0)) launch_eps_partials(H, H.lv[H.L - 1], s);
  for (int l = 0; l < H.L; ++l) {
    Level& L = H.lv[l];
    if (H.coef_kind == 1) {
      launch_coef_tensor(H, L, H.lv[H.L - 1], s);
    } else {
      // coef_kind 2 starts from the state u = 0: nothing yields, C = 2 mu0 I
      launch_mu_sinker(H, L, s);
      if (L.cw) launch_fill<double>(L.cw, 0.0, (int64_t)(D * (D + 1) / 2) * (D == 2 ? 9 : 27) * L.g.ncell, s);
    }
    launch_fill<double>(L.S, 0.0, L.nvel, s);
    if (L.S32) launch_fill<float>(L.S32, 0.0, L.nvel, s);
    launch_fill<double>(L.x, 0.0, L.nvel, s);
    if (l >= 1) {
      std::vector<ClassPlan> plan = H.deg == 3 ? plan_patches_q3(D, L.g.N) : plan_patches(D, L.g.N);
      for (size_t c = 0; c < plan.size(); ++c) {
        if (hipMemcpyAsync(L.cls[c].verts, plan[c].verts.data(), plan[c].verts.size() * 4, hipMemcpyHostToDevice,
                           s) != hipSuccess)
          return bail(fail(STK_EDEVICE, "copy of patch vertex lists failed"));
        // the host vector must outlive the copy
        if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(STK_EDEVICE, "sync failed"));
      }
    }
  }
  if (H.mu0) launch_mu_sinker_to(H, H.lv[H.L - 1], H.mu0, s);
  const stk_status st2 = build_operators(H, s);
  if (st2 != STK_OK) return bail(st2);
  *out = h;
  return STK_OK;
}

stk_status stk_profile(stk_hier* h, int enable) {
  if (!h) return fail(STK_EINVAL, "hierarchy is NULL");
  Prof& P = h->H.prof;
  if (enable < 0 || enable > 100) return fail(STK_EINVAL, "enable must be in [0, 100]");
  P.on = enable != 0;
  P.reps = enable > 0 ? enable : 1;
  P.recs.clear();
  P.used = 0;
  return STK_OK;
}

stk_status stk_profile_read(stk_hier* h, int kernel, int64_t* launches, double* total_ms, double* total_bytes) {
  if (!h) return fail(STK_EINVAL, "hierarchy is NULL");
  if (kernel < 0 || kernel > PROF_NIDS) return fail(STK_EINVAL, "unknown kernel id");
  Prof& P = h->H.prof;
  HIPCHK(hipStreamSynchronize(h->H.stream));
  // kernel PROF_NIDS: the patch-solve launches of the finest level, told
  // apart by their algorithmic bytes per launch (FP64 or FP32)
  double fine_b[2] = {0.0, 0.0};
  if (kernel == PROF_NIDS) {
    const Level& F = h->H.lv[h->H.L - 1];
    double e = (double)F.nvel;
    for (const PatchClass& pc : F.cls) e += (double)pc.count * (pc.n * (pc.n + 1) / 2 + pc.n);
    fine_b[0] = 8.0 * e;
    fine_b[1] = 4.0 * e;
  }
  int64_t n = 0;
  double ms = 0.0, by = 0.0;
  for (const Prof::Rec& r : P.recs) {
    if (kernel == PROF_NIDS) {
      if (r.id != PROF_ASM_GEMV || r.n <= 0) continue;
      const double per = r.bytes / r.n;
      if (fabs(per - fine_b[0]) > 0.5 && fabs(per - fine_b[1]) > 0.5) continue;
    } else if (r.id != kernel) {
      continue;
    }
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    n += r.n;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (total_bytes) *total_bytes = by;
  return STK_OK;
}

stk_status stk_destroy(stk_hier* h) {
  if (!h) return STK_OK;
  (void)hipStreamSynchronize(h->H.stream);
  for (hipEvent_t e : h->H.prof.pool) (void)hipEventDestroy(e);
  drop_graphs(h->H);
  if (h->H.sev) (void)hipEventDestroy(h->H.sev);
  if (h->H.bev) (void)hipEventDestroy(h->H.bev);
  if (h->H.cev) (void)hipEventDestroy(h->H.cev);
  if (h->H.hpin) (void)hipHostFree(h->H.hpin);
  if (h->H.own) {
    (void)hipStreamSynchronize(h->H.own);
    (void)hipStreamDestroy(h->H.own);
  }
  free_all(h->H);
  delete h;
  return STK_OK;
}

stk_status stk_sizes(const stk_hier* h, int level, int64_t* n_vel_stored, int64_t* n_pres) {
  if (!h) return fail(STK_EINVAL, "hierarchy is NULL");
  STKCHK(check_level(h->H, level, 0));
  if (n_vel_stored) *n_vel_stored = h->H.lv[level].nvel;
  if (n_pres) *n_pres = h->H.lv[level].npres;
  return STK_OK;
}

#define GET_H(h)                                                  \
  if (!(h)) return fail(STK_EINVAL, "hierarchy is NULL");         \
  Hier& H = (h)->H;                                               \
  H.stream = (hipStream_t)stream

// For calls that use the hierarchy's device buffers: STK_EBUSY while a
// resumable solve is in progress (its phases use the same buffers on the
// hierarchy's own stream), checked before anything is touched.
#define GET_H_IDLE(h)                                                                      \
  if (!(h)) return fail(STK_EINVAL, "hierarchy is NULL");                                  \
  if (solve_busy((h)->H)) return fail(STK_EBUSY, "a resumable solve is in progress on this hierarchy"); \
  Hier& H = (h)->H;                                                                        \
  H.stream = (hipStream_t)stream

stk_status stk_set_asm_variant(stk_hier* h, int level, int dtype, int variant) {
  if (!h) return fail(STK_EINVAL, "hierarchy is NULL");
  Hier& H = h->H;
  STKCHK(check_level(H, level, 1));
  STKCHK(check_dtype(H, dtype));
  if (variant < 0 || variant >= kAsmVariants) return fail(STK_EINVAL, "variant out of range");
  if (solve_busy(H)) return fail(STK_EBUSY, "a resumable solve is in progress on this hierarchy");
  H.lv[level].asm_variant[dtype == STK_F64 ? 0 : 1] = variant;
  drop_graphs(H);   // captured steps hold the previous variant's kernels
  return STK_OK;
}

// Times every patch-solve variant on every smoothed level (and precision in
// use) with HIP events around `reps` back-to-back launches on the level's own
// buffers, and keeps the fastest (ties: the lower index).
stk_status stk_autotune(stk_hier* h, int reps, int* variants, float* times_ms, void* stream) {
  GET_H_IDLE(h);
  if (reps < 1 || reps > 100) return fail(STK_EINVAL, "reps must be in [1, 100]");
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  stk_status st = STK_OK;
  for (int l = 1; l < H.L && st == STK_OK; ++l) {
    Level& L = H.lv[l];
    for (int dt = 0; dt < 2; ++dt) {
      if (variants) variants[(l - 1) * 2 + dt] = -1;
      if (dt == 1 && !H.mixed) continue;
      int best = 0;
      float best_ms = 0.0f;
      for (int v = 0; v < kAsmVariants; ++v) {
        L.asm_variant[dt] = v;
        // input: the level's residual buffer (any contents; only time matters)
        if (dt == 0) launch_asm_gemv<double>(H, L, L.r, 1, H.stream, nullptr);
        else launch_asm_gemv<float>(H, L, reinterpret_cast<const float*>(L.r), 1, H.stream, nullptr);
        if (hipEventRecord(a, H.stream) != hipSuccess) { st = fail(STK_EDEVICE, "event record failed"); break; }
        if (dt == 0) launch_asm_gemv<double>(H, L, L.r, reps, H.stream, nullptr);
        else launch_asm_gemv<float>(H, L, reinterpret_cast<const float*>(L.r), reps, H.stream, nullptr);
        float ms = 0.0f;
        if (hipEventRecord(b, H.stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          st = fail(STK_EDEVICE, "event timing failed");
          break;
        }
        if (times_ms) times_ms[((l - 1) * 2 + dt) * kAsmVariants + v] = ms / (float)reps;
        if (v == 0 || ms < best_ms) {
          best = v;
          best_ms = ms;
        }
      }
      L.asm_variant[dt] = best;
      if (variants) variants[(l - 1) * 2 + dt] = best;
      if (st != STK_OK) break;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  drop_graphs(H);   // captured steps hold the previous variants' kernels
  if (st == STK_OK && hipGetLastError() != hipSuccess) st = fail(STK_EDEVICE, "launch failed during tuning");
  return st;
}

stk_status stk_rhs(stk_hier* h, double* b_u, double* b_p, void* stream) {
  GET_H_IDLE(h);
  if (!b_u) return fail(STK_EINVAL, "b_u is NULL");
  Level& F = H.lv[H.L - 1];
  launch_rhs_elem(H, F, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, b_u, H.stream);
  if (b_p) launch_fill<double>(b_p, 0.0, F.npres, H.stream);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_apply_Agamma(stk_hier* h, int level, int dtype, const void* x, void* y, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_level(H, level, 0));
  STKCHK(check_dtype(H, dtype));
  if (!x || !y || x == y) return fail(STK_EINVAL, "x, y must be distinct non-NULL buffers");
  if (dtype == STK_F64) apply_A<double>(H, level, (const double*)x, (double*)y);
  else apply_A<float>(H, level, (const float*)x, (float*)y);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_apply_stokes(stk_hier* h, const double* x_u, const double* x_p, double* y_u, double* y_p,
                            void* stream) {
  GET_H_IDLE(h);
  if (!x_u || !x_p || !y_u || !y_p) return fail(STK_EINVAL, "NULL buffer");
  Level& F = H.lv[H.L - 1];
  launch_elem<double>(H, F, EL_VISC | EL_AUG | EL_BT | EL_BOUT, x_u, x_p, y_p, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, y_u, H.stream);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_asm(stk_hier* h, int level, int dtype, const void* r, void* y, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_level(H, level, 1));
  STKCHK(check_dtype(H, dtype));
  if (!r || !y) return fail(STK_EINVAL, "NULL buffer");
  if (dtype == STK_F64) launch_asm<double>(H, H.lv[level], (const double*)r, (double*)y, H.stream);
  else launch_asm<float>(H, H.lv[level], (const float*)r, (float*)y, H.stream);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_smooth(stk_hier* h, int level, int dtype, const void* b, void* x, int nsteps, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_level(H, level, 1));
  STKCHK(check_dtype(H, dtype));
  if (!b || !x || b == x) return fail(STK_EINVAL, "b, x must be distinct non-NULL buffers");
  if (nsteps < 1 || nsteps > kMaxNu) return fail(STK_EINVAL, "nsteps must be in [1, 8]");
  if (dtype == STK_F64) smooth<double>(H, level, (const double*)b, (double*)x, nsteps, false);
  else smooth<float>(H, level, (const float*)b, (float*)x, nsteps, false);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_prolong(stk_hier* h, int coarse_level, int dtype, const void* xc, void* xf, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_level(H, coarse_level + 1, 1));
  STKCHK(check_dtype(H, dtype));
  if (!xc || !xf) return fail(STK_EINVAL, "NULL buffer");
  if (dtype == STK_F64) prolong_robust<double>(H, coarse_level + 1, (const double*)xc, (double*)xf);
  else prolong_robust<float>(H, coarse_level + 1, (const float*)xc, (float*)xf);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_restrict(stk_hier* h, int fine_level, int dtype, const void* rf, void* rc, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_level(H, fine_level, 1));
  STKCHK(check_dtype(H, dtype));
  if (!rf || !rc) return fail(STK_EINVAL, "NULL buffer");
  if (dtype == STK_F64) restrict_robust<double>(H, fine_level, (const double*)rf, (double*)rc);
  else restrict_robust<float>(H, fine_level, (const float*)rf, (float*)rc);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_coarse_solve(stk_hier* h, const double* b, double* x, void* stream) {
  GET_H_IDLE(h);
  if (!b || !x || b == x) return fail(STK_EINVAL, "b, x must be distinct non-NULL buffers");
  coarse_solve<double>(H, b, x);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_vcycle(stk_hier* h, int dtype, const void* b, void* x, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_dtype(H, dtype));
  if (!b || !x || b == x) return fail(STK_EINVAL, "b, x must be distinct non-NULL buffers");
  if (dtype == STK_F64) vcycle<double>(H, H.L - 1, (const double*)b, (double*)x);
  else vcycle<float>(H, H.L - 1, (const float*)b, (float*)x);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_fcycle(stk_hier* h, int dtype, const void* b, void* x, void* stream) {
  GET_H_IDLE(h);
  STKCHK(check_dtype(H, dtype));
  if (!b || !x || b == x) return fail(STK_EINVAL, "b, x must be distinct non-NULL buffers");
  if (dtype == STK_F64) fcycle<double>(H, H.L - 1, (const double*)b, (double*)x);
  else fcycle<float>(H, H.L - 1, (const float*)b, (float*)x);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_precond(stk_hier* h, int flags, const double* v_u, const double* v_p, double* z_u, double* z_p,
                       void* stream) {
  GET_H_IDLE(h);
  if (!v_u || !v_p || !z_u || !z_p) return fail(STK_EINVAL, "NULL buffer");
  if (flags & ~(STK_PC_MIXED | STK_PC_UPPER | STK_PC_FCYCLE)) return fail(STK_EINVAL, "unknown preconditioner flags");
  const bool mixed = (flags & STK_PC_MIXED) != 0;
  if (mixed && !H.mixed) return fail(STK_EINVAL, "the mixed form needs a hierarchy set up with mixed=1");
  precond(H, v_u, v_p, z_u, z_p, mixed, (flags & STK_PC_UPPER) != 0, (flags & STK_PC_FCYCLE) != 0);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

}  // extern "C"

namespace {

// Pinned host layout: Hessenberg copy [(kMaxRestart+1) x kMaxRestart], norm
// partials [kRedBlocks], y [kMaxRestart].
constexpr int kMaxRestart = 64;
constexpr size_t kPinH = 0;
constexpr size_t kPinPart = (size_t)(kMaxRestart + 1) * kMaxRestart;
constexpr size_t kPinY = kPinPart + kRedBlocks;
constexpr size_t kPinLen = kPinY + kMaxRestart;

stk_status ensure_pinned(Hier& H) {
  if (!H.hpin) {
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, kPinLen * 8, hipHostMallocDefault));
    H.hpin = static_cast<double*>(p);
  }
  if (!H.sev) HIPCHK(hipEventCreateWithFlags(&H.sev, hipEventDisableTiming));
  return STK_OK;
}

void sv_done(Hier& H, stk_status st) {
  Hier::Solve& S = H.sv;
  S.phase = Hier::SV_DONE;
  S.status = st;
  S.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - S.t0).count();
}

// Starts a solve: checks, copies b, x = 0, ||b|| (host-synchronous on the
// hierarchy's stream, ordered after the caller's stream).
stk_status sv_begin(Hier& H, hipStream_t caller, const double* b_u, const double* b_p, double* x_u, double* x_p,
                    const stk_solve_opts* opts) {
  Hier::Solve& S = H.sv;
  if (S.phase != Hier::SV_IDLE && S.phase != Hier::SV_DONE) return fail(STK_EBUSY, "a solve is in progress");
  if (!b_u || !x_u || !x_p) return fail(STK_EINVAL, "NULL buffer");
  double rtol = 1e-8;
  int m = 30, maxit = 300;
  if (opts) {
    rtol = opts->rtol;
    m = opts->restart;
    maxit = opts->maxit;
  }
  if (!(rtol > 0.0) || m < 1 || m > kMaxRestart || maxit < 1 || maxit > 1000)
    return fail(STK_EINVAL, "bad solve options (rtol > 0, restart 1..64, maxit 1..1000)");
  const bool mixed = opts && opts->mixed;
  if (mixed && !H.mixed) return fail(STK_EINVAL, "the mixed form needs a hierarchy set up with mixed=1");
  if (opts && (opts->pc < 0 || opts->pc > 1)) return fail(STK_EINVAL, "pc must be 0 (full) or 1 (upper)");
  if (opts && (opts->cycle < 0 || opts->cycle > 1)) return fail(STK_EINVAL, "cycle must be 0 (V) or 1 (F)");
  const bool upper = opts && opts->pc == 1;
  const bool fcyc = opts && opts->cycle == 1;
  STKCHK(ensure_pinned(H));
  Level& F = H.lv[H.L - 1];
  const int64_t nu = F.nvel, np = F.npres, nvec = nu + np;
  if (m > H.restart_alloc) {
    // grow the Krylov storage
    double *nV = nullptr, *nZ = nullptr, *nH = nullptr;
    HIPCHK(hipMalloc(&nV, (size_t)(m + 1) * nvec * 8));
    HIPCHK(hipMalloc(&nZ, (size_t)m * nvec * 8));
    HIPCHK(hipMalloc(&nH, (size_t)(m + 1) * m * 8));
    H.allocs.push_back(nV);
    H.allocs.push_back(nZ);
    H.allocs.push_back(nH);
    H.fV = nV;
    H.fZ = nZ;
    H.fH = nH;
    H.restart_alloc = m;
    drop_graphs(H);
  }
  S = Hier::Solve{};
  S.m = m;
  S.maxit = maxit;
  S.rtol = rtol;
  S.mixed = mixed;
  S.upper = upper;
  S.fcycle = fcyc;
  S.graphs = !(opts && opts->eager);
  S.x_u = x_u;
  S.x_p = x_p;
  S.Hh.assign((size_t)(m + 1) * m, 0.0);
  S.cs.assign(m, 0.0);
  S.sn.assign(m, 0.0);
  S.g.assign(m + 1, 0.0);
  S.hist.assign(1, 1.0);
  S.t0 = std::chrono::steady_clock::now();
  // order the hierarchy's stream after the caller's work on b
  HIPCHK(hipEventRecord(H.sev, caller));
  HIPCHK(hipStreamWaitEvent(H.own, H.sev, 0));
  H.stream = H.own;
  hipStream_t s = H.own;
  double* bvec = H.fr + nvec;
  double* xvec = H.fw;
  double* rvec = H.fr;
  HIPCHK(hipMemcpyAsync(bvec, b_u, nu * 8, hipMemcpyDeviceToDevice, s));
  if (b_p) HIPCHK(hipMemcpyAsync(bvec + nu, b_p, np * 8, hipMemcpyDeviceToDevice, s));
  else launch_fill<double>(bvec + nu, 0.0, np, s);
  launch_fill<double>(xvec, 0.0, nvec, s);
  STKCHK(device_norm(H, bvec, nvec, &S.bnorm));
  if (!isfinite(S.bnorm)) {
    sv_done(H, STK_ENAN);
    return fail(STK_ENAN, "right-hand side is not finite");
  }
  if (S.bnorm == 0.0) {
    launch_fill<double>(x_u, 0.0, nu, s);
    launch_fill<double>(x_p, 0.0, np, s);
    HIPCHK(hipStreamSynchronize(s));
    S.converged = true;
    sv_done(H, STK_OK);
    return STK_OK;
  }
  launch_copy(bvec, rvec, nvec, s);
  S.beta = S.bnorm;
  S.g[0] = S.beta;
  S.j = 0;
  S.phase = Hier::SV_ARNOLDI;
  return STK_OK;
}

// Enqueues the device work of the current phase on the hierarchy's stream.
stk_status sv_enqueue(Hier& H) {
  Hier::Solve& S = H.sv;
  H.stream = H.own;
  hipStream_t s = H.own;
  Level& F = H.lv[H.L - 1];
  const int64_t nu = F.nvel, np = F.npres, nvec = nu + np;
  const int m = S.m;
  double* bvec = H.fr + nvec;
  double* xvec = H.fw;
  double* rvec = H.fr;
  if (S.phase == Hier::SV_ARNOLDI) {
    const int j = S.j;
    if (j == 0) launch_axpby<double>(1.0 / S.beta, rvec, 0.0, rvec, H.fV, nvec, s);
    const int key = (S.mixed ? 1 : 0) | (S.upper ? 2 : 0) | (S.fcycle ? 4 : 0);
    if (!S.graphs) {
      arnoldi_step(H, j, m, nu, nvec, S.mixed, S.upper, S.fcycle);
    } else {
      if (H.steps_m != m || H.steps_key != key) {
        drop_graphs(H);
        H.steps.assign(m, nullptr);
        H.steps_m = m;
        H.steps_key = key;
      }
      if (!H.steps[j]) {
        const bool prof_on = H.prof.on;
        H.prof.on = false;   // no event records inside captured graphs
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        arnoldi_step(H, j, m, nu, nvec, S.mixed, S.upper, S.fcycle);
        const hipError_t ce = hipStreamEndCapture(s, &graph);
        H.prof.on = prof_on;
        if (ce != hipSuccess) return fail(STK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return fail(STK_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        H.steps[j] = exec;
      }
      HIPCHK(hipGraphLaunch(H.steps[j], s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(H.hpin + kPinH, H.fH, (size_t)(m + 1) * m * 8, hipMemcpyDeviceToHost, s));
  } else if (S.phase == Hier::SV_RESIDUAL) {
    HIPCHK(hipMemcpyAsync(H.fy, H.hpin + kPinY, (size_t)S.k * 8, hipMemcpyHostToDevice, s));
    launch_combine(H.fZ, nvec, S.k, H.fy, xvec, nvec, false, s);
    // true residual r = b - K x and its norm partials
    stokes_apply(H, xvec, rvec);
    launch_axpby<double>(1.0, bvec, -1.0, rvec, rvec, nvec, s);
    launch_dots<double>(rvec, nvec, 1, rvec, nvec, H.partials, s);
    HIPCHK(hipMemcpyAsync(H.hpin + kPinPart, H.partials, (size_t)red_parts(nvec) * 8, hipMemcpyDeviceToHost, s));
  } else if (S.phase == Hier::SV_FINISH) {
    launch_project_mean(H, F, xvec + nu, s);
    HIPCHK(hipMemcpyAsync(S.x_u, xvec, nu * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(S.x_p, xvec + nu, np * 8, hipMemcpyDeviceToDevice, s));
  } else {
    return STK_OK;
  }
  HIPCHK(hipEventRecord(H.sev, s));
  S.inflight = true;
  return STK_OK;
}

// Waits for the current phase and runs its host part (Givens rotations,
// stopping tests), moving to the next phase.
stk_status sv_advance(Hier& H) {
  Hier::Solve& S = H.sv;
  if (S.phase == Hier::SV_IDLE || S.phase == Hier::SV_DONE) return STK_OK;
  HIPCHK(hipEventSynchronize(H.sev));
  S.inflight = false;
  Level& F = H.lv[H.L - 1];
  const int64_t nvec = F.nvel + F.npres;
  const int m = S.m;
  std::vector<double>& Hh = S.Hh;
  if (S.phase == Hier::SV_ARNOLDI) {
    const int j = S.j;
    const double* Hd = H.hpin + kPinH;
    for (int i = 0; i <= j + 1; ++i) Hh[i * m + j] = Hd[i * m + j];
    if (!isfinite(Hh[(j + 1) * m + j])) {
      sv_done(H, STK_ENAN);
      return fail(STK_ENAN, "non-finite value in the Arnoldi process");
    }
    for (int i = 0; i < j; ++i) {
      const double a = Hh[i * m + j], c2 = Hh[(i + 1) * m + j];
      Hh[i * m + j] = S.cs[i] * a + S.sn[i] * c2;
      Hh[(i + 1) * m + j] = -S.sn[i] * a + S.cs[i] * c2;
    }
    double c = 1.0, sv = 0.0;
    const double a = Hh[j * m + j], bb = Hh[(j + 1) * m + j];
    if (bb != 0.0) {
      const double r = hypot(a, bb);
      c = a / r;
      sv = bb / r;
    }
    S.cs[j] = c;
    S.sn[j] = sv;
    Hh[j * m + j] = c * a + sv * bb;
    Hh[(j + 1) * m + j] = 0.0;
    S.g[j + 1] = -sv * S.g[j];
    S.g[j] = c * S.g[j];
    ++S.it;
    S.hist.push_back(fabs(S.g[j + 1]) / S.bnorm);
    if (fabs(S.g[j + 1]) <= S.rtol * S.bnorm || S.it >= S.maxit || j + 1 == m) {
      // end of the cycle: y from the triangular system, then the true residual
      const int k = j + 1;
      double* y = H.hpin + kPinY;
      for (int i = k - 1; i >= 0; --i) {
        double sacc = S.g[i];
        for (int t = i + 1; t < k; ++t) sacc -= Hh[i * m + t] * y[t];
        y[i] = sacc / Hh[i * m + i];
      }
      S.k = k;
      S.phase = Hier::SV_RESIDUAL;
    } else {
      S.j = j + 1;
    }
  } else if (S.phase == Hier::SV_RESIDUAL) {
    const int np = red_parts(nvec);
    double sacc = 0.0;
    for (int b = 0; b < np; ++b) sacc += H.hpin[kPinPart + b];
    S.beta = sqrt(sacc);
    if (!isfinite(S.beta)) {
      sv_done(H, STK_ENAN);
      return fail(STK_ENAN, "non-finite residual");
    }
    if (S.beta <= S.rtol * S.bnorm) {
      S.converged = true;
      S.phase = Hier::SV_FINISH;
    } else if (S.it >= S.maxit) {
      S.phase = Hier::SV_FINISH;
    } else {
      std::fill(S.g.begin(), S.g.end(), 0.0);
      S.g[0] = S.beta;
      S.j = 0;
      S.phase = Hier::SV_ARNOLDI;
    }
  } else if (S.phase == Hier::SV_FINISH) {
    sv_done(H, S.converged ? STK_OK : STK_ENOTCONV);
  }
  return STK_OK;
}

// Enqueues the Arnoldi step of each hierarchy of `g` (same dimension, level
// count, fine mesh, relaxation steps and solve form, so the same sequence of
// patch-solve calls on levels of the same shapes) on its own stream from its
// own host thread, with the patch solves of the small levels batched across
// them (Cohort).
stk_status enqueue_cohort(const std::vector<Hier*>& g) {
  const int n = (int)g.size();
  Cohort C;
  C.n = n;
  C.hs.assign(g.begin(), g.end());
  C.ls.assign(n, nullptr);
  C.rs.assign(n, nullptr);
  C.ready.assign(n, nullptr);
  C.lead = g[0]->own;
  for (int k = 0; k < n; ++k) {
    if (!g[k]->bev) HIPCHK(hipEventCreateWithFlags(&g[k]->bev, hipEventDisableTiming));
    C.ready[k] = g[k]->bev;
  }
  C.done = g[0]->cev;
  if (!C.done) {
    HIPCHK(hipEventCreateWithFlags(&g[0]->cev, hipEventDisableTiming));
    C.done = g[0]->cev;
  }
  std::vector<stk_status> st(n, STK_OK);
  std::vector<std::string> err(n);
  std::vector<std::function<void()>> tasks(n);
  for (int k = 0; k < n; ++k)
    tasks[k] = [&, k] {
      t_cohort = &C;
      t_slot = k;
      st[k] = sv_enqueue(*g[k]);
      if (st[k] != STK_OK) {
        err[k] = g_err;
        C.broken.store(true, std::memory_order_release);
      }
      t_cohort = nullptr;
      t_slot = -1;
    };
  static CohortPool pool;
  static std::mutex pool_m;   // one cohort at a time uses the pool
  {
    std::lock_guard<std::mutex> lk(pool_m);
    pool.run(tasks);
  }
  for (int k = 0; k < n; ++k)
    if (st[k] != STK_OK) return fail(st[k], err[k]);
  return STK_OK;
}

void sv_info(const Hier& H, stk_solve_info* inf) {
  if (!inf) return;
  const Hier::Solve& S = H.sv;
  memset(inf, 0, sizeof(*inf));
  inf->iters = S.it;
  inf->converged = S.converged ? 1 : 0;
  inf->rel_res = S.bnorm > 0.0 ? S.beta / S.bnorm : 0.0;
  inf->t_solve_s = S.t_solve;
  const size_t nh = std::min<size_t>(S.hist.size(), 1001);
  for (size_t i = 0; i < nh; ++i) inf->hist[i] = S.hist[i];
  if (S.hist.empty()) inf->hist[0] = 1.0;
}

stk_status sv_final(Hier& H) {
  if (H.sv.status == STK_ENOTCONV) return fail(STK_ENOTCONV, "FGMRES reached maxit");
  if (H.sv.status == STK_ENAN) return fail(STK_ENAN, "non-finite value in the solve");
  return (stk_status)H.sv.status;
}

}  // namespace

extern "C" {

stk_status stk_solve(stk_hier* h, const double* b_u, const double* b_p, double* x_u, double* x_p,
                     const stk_solve_opts* opts, stk_solve_info* info, void* stream) {
  GET_H_IDLE(h);
  hipStream_t caller = H.stream;
  const stk_status st0 = sv_begin(H, caller, b_u, b_p, x_u, x_p, opts);
  if (st0 != STK_OK) {
    if (H.sv.phase == Hier::SV_DONE) sv_info(H, info);
    H.stream = caller;
    return st0;
  }
  while (H.sv.phase != Hier::SV_DONE) {
    stk_status st = sv_enqueue(H);
    if (st == STK_OK) st = sv_advance(H);
    if (st != STK_OK) {
      if (H.sv.phase != Hier::SV_DONE) sv_done(H, st);
      (void)hipStreamSynchronize(H.own);
      sv_info(H, info);
      H.stream = caller;
      return st;
    }
  }
  sv_info(H, info);
  H.stream = caller;
  return sv_final(H);
}

stk_status stk_solve_begin(stk_hier* h, const double* b_u, const double* b_p, double* x_u, double* x_p,
                           const stk_solve_opts* opts, void* stream) {
  GET_H(h);
  hipStream_t caller = H.stream;
  const stk_status st = sv_begin(H, caller, b_u, b_p, x_u, x_p, opts);
  H.stream = caller;
  return st;
}

stk_status stk_step_batch(stk_hier* const* hs, int n, void* stream) {
  if (n < 0 || (n > 0 && !hs)) return fail(STK_EINVAL, "bad hierarchy list");
  (void)stream;
  for (int i = 0; i < n; ++i)
    if (!hs[i]) return fail(STK_EINVAL, "NULL hierarchy in the list");
  // STK_CROSS_BATCH=1 in the environment turns the lockstep cohorts on
  // (off by default: on a mixed request stream their cross-stream waits cost
  // more than the fuller launches gain)
  const char* env = getenv("STK_CROSS_BATCH");
  const bool cross = env && env[0] == '1';
  stk_status first = STK_OK;
  auto note = [&](Hier& H, stk_status st) {
    if (st == STK_OK) return;
    if (H.sv.phase != Hier::SV_DONE) sv_done(H, st);
    if (first == STK_OK) first = st;
  };
  auto active = [](const Hier& H) { return H.sv.phase != Hier::SV_IDLE && H.sv.phase != Hier::SV_DONE; };
  for (int pass = 0; pass < 2; ++pass) {
    bool moved = false;
    // 1. host parts of the phases that have finished on the device
    for (int i = 0; i < n; ++i) {
      Hier& H = hs[i]->H;
      if (!active(H) || !H.sv.inflight) continue;
      const hipError_t q = hipEventQuery(H.sev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        note(H, fail(STK_EDEVICE, std::string("phase event: ") + hipGetErrorString(q)));
        continue;
      }
      note(H, sv_advance(H));
      moved = true;
    }
    // 2. next phases of every solve with nothing in flight; Arnoldi steps of
    //    same-shape plain-launch solves go out as lockstep cohorts
    std::map<std::tuple<int, int, int, int, int, int>, std::vector<Hier*>> groups;
    for (int i = 0; i < n; ++i) {
      Hier& H = hs[i]->H;
      if (!active(H) || H.sv.inflight) continue;
      const Hier::Solve& S = H.sv;
      if (cross && S.phase == Hier::SV_ARNOLDI && !S.graphs && !H.prof.on) {
        const int form = (S.mixed ? 1 : 0) | (S.upper ? 2 : 0) | (S.fcycle ? 4 : 0) | (H.deg == 3 ? 8 : 0);
        groups[std::make_tuple(H.dim, H.L, H.lv.back().g.N, H.nu_pre, H.nu_post, form)].push_back(&H);
        continue;
      }
      note(H, sv_enqueue(H));
      moved = true;
    }
    for (auto& kv : groups) {
      std::vector<Hier*>& g = kv.second;
      for (size_t k0 = 0; k0 < g.size(); k0 += kAsmBatchMax) {
        const size_t kn = std::min(g.size() - k0, (size_t)kAsmBatchMax);
        std::vector<Hier*> part(g.begin() + k0, g.begin() + k0 + kn);
        if (kn == 1) {
          note(*part[0], sv_enqueue(*part[0]));
        } else {
          const stk_status st = enqueue_cohort(part);
          if (st != STK_OK) {
            for (Hier* H : part) note(*H, st);
          }
        }
        moved = true;
      }
    }
    if (moved || pass == 1) break;
    // 3. nothing could move: wait for the first in-flight phase to finish
    bool any = false;
    for (int i = 0; i < n; ++i) any = any || (active(hs[i]->H) && hs[i]->H.sv.inflight);
    if (!any) break;
    for (;;) {
      bool ready = false;
      for (int i = 0; i < n && !ready; ++i) {
        Hier& H = hs[i]->H;
        if (active(H) && H.sv.inflight && hipEventQuery(H.sev) != hipErrorNotReady) ready = true;
      }
      if (ready) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  return first;
}

stk_status stk_poll(stk_hier* h, stk_solve_info* info) {
  if (!h) return fail(STK_EINVAL, "hierarchy is NULL");
  Hier& H = h->H;
  const int ph = H.sv.phase;
  if (ph == Hier::SV_IDLE) return fail(STK_EINVAL, "no solve was started");
  if (ph != Hier::SV_DONE) return STK_EBUSY;
  sv_info(H, info);
  return sv_final(H);
}

}  // extern "C"

// =========================================================================== viscoplastic Newton
namespace {

// F = (F_u, F_p) of the viscoplastic problem at (u, p): F_u = a(u; u) +
// gamma B^T W^{-1} B u + B^T p - b, F_p = B u; b the velocity right-hand side.
void nl_residual(Hier& H, const double* u, const double* p, const double* b, double* Fu, double* Fp) {
  Level& F = H.lv[H.L - 1];
  launch_nl_elem(H, F, u, p, Fp, H.stream);
  launch_gather<double>(H, F, b, -1.0, Fu, H.stream);                 // b - a(u; u) - ...
  launch_axpby<double>(-1.0, Fu, 0.0, Fu, Fu, F.nvel, H.stream);
}

// Coefficients of the linearisation at the fine velocity u on every level
// (coarser levels take the velocity injected to their nodes), then every
// operator built from them.
stk_status relinearize(Hier& H, const double* u) {
  hipStream_t s = H.stream;
  const double* ul = u;
  for (int l = H.L - 1; l >= 0; --l) {
    Level& L = H.lv[l];
    launch_coef_fe(H, L, ul, s);
    if (l > 0) {
      launch_inject(H, L, H.lv[l - 1], ul, H.lv[l - 1].T, s);
      ul = H.lv[l - 1].T;
    }
  }
  return build_operators(H, s);
}

stk_status newton_check(const Hier& H) {
  if (H.coef_kind != 2) return fail(STK_EINVAL, "the hierarchy holds no viscoplastic state (set up with coef_kind 2)");
  return STK_OK;
}

}  // namespace

extern "C" {

stk_status stk_relinearize(stk_hier* h, const double* x_u, void* stream) {
  GET_H_IDLE(h);
  STKCHK(newton_check(H));
  if (!x_u) return fail(STK_EINVAL, "x_u is NULL");
  return relinearize(H, x_u);
}

stk_status stk_nl_residual(stk_hier* h, const double* x_u, const double* x_p, double* r_u, double* r_p,
                           void* stream) {
  GET_H_IDLE(h);
  STKCHK(newton_check(H));
  if (!x_u || !x_p || !r_u || !r_p || x_u == r_u) return fail(STK_EINVAL, "bad buffers");
  Level& F = H.lv[H.L - 1];
  launch_rhs_elem(H, F, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, H.nl_b, H.stream);
  nl_residual(H, x_u, x_p, H.nl_b, r_u, r_p);
  HIPCHK(hipGetLastError());
  return STK_OK;
}

stk_status stk_newton(stk_hier* h, double* x_u, double* x_p, const stk_newton_opts* opts, stk_newton_info* info,
                      void* stream) {
  GET_H_IDLE(h);
  STKCHK(newton_check(H));
  if (!x_u || !x_p) return fail(STK_EINVAL, "NULL buffer");
  stk_newton_opts o{1e-8, 30, 1e-6, 300, 30, 10, 0, 0, 0};
  if (opts) o = *opts;
  if (!(o.rtol > 0.0) || o.maxit < 1 || o.maxit > STK_NEWTON_MAXIT || !(o.lin_rtol > 0.0) || o.lin_maxit < 1 ||
      o.max_halvings < 0 || o.max_halvings > 30 || o.restart < 1 || o.restart > 64)
    return fail(STK_EINVAL, "bad Newton options");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t caller = H.stream;
  Level& F = H.lv[H.L - 1];
  const int64_t nu = F.nvel, np = F.npres, nvec = nu + np;
  double *b = H.nl_b, *R = H.nl_F, *d = H.nl_d, *x = H.nl_x, *t = H.nl_t;
  if (info) memset(info, 0, sizeof(*info));
  // right-hand side, x = 0, F(x), ||F||
  launch_rhs_elem(H, F, H.stream);
  launch_gather<double>(H, F, nullptr, 1.0, b, H.stream);
  launch_fill<double>(x, 0.0, nvec, H.stream);
  nl_residual(H, x, x + nu, b, R, R + nu);
  double fn = 0.0;
  STKCHK(device_norm(H, R, nvec, &fn));
  if (!isfinite(fn)) return fail(STK_ENAN, "non-finite nonlinear residual");
  const double f0 = fn;
  stk_solve_opts so{o.lin_rtol, o.restart, o.lin_maxit, o.eager, 0, o.pc, o.cycle};
  int k = 0;
  bool converged = f0 == 0.0;
  if (info) info->hist[0] = 1.0;
  stk_status st = STK_OK;
  while (!converged && k < o.maxit) {
    STKCHK(relinearize(H, x));
    // Newton step: J d = -F
    launch_axpby<double>(-1.0, R, 0.0, R, t, nvec, H.stream);
    stk_solve_info li;
    const stk_status ls = stk_solve(h, t, t + nu, d, d + nu, &so, &li, caller);
    H.stream = caller;
    if (ls != STK_OK && ls != STK_ENOTCONV) return ls;
    // backtracking on the residual norm
    double alpha = 1.0, ft = 0.0;
    for (int hv = 0; hv <= o.max_halvings; ++hv) {
      launch_axpby<double>(1.0, x, alpha, d, t, nvec, H.stream);
      nl_residual(H, t, t + nu, b, R, R + nu);
      STKCHK(device_norm(H, R, nvec, &ft));
      if (!isfinite(ft)) return fail(STK_ENAN, "non-finite nonlinear residual");
      if (ft <= (1.0 - 1e-4 * alpha) * fn || hv == o.max_halvings) break;
      alpha *= 0.5;
    }
    launch_copy(t, x, nvec, H.stream);
    fn = ft;
    if (info) {
      info->lin_iters[k] = li.iters;
      info->alpha[k] = alpha;
      info->hist[k + 1] = fn / f0;
    }
    ++k;
    converged = fn <= o.rtol * f0;
  }
  HIPCHK(hipMemcpyAsync(x_u, x, nu * 8, hipMemcpyDeviceToDevice, H.stream));
  HIPCHK(hipMemcpyAsync(x_p, x + nu, np * 8, hipMemcpyDeviceToDevice, H.stream));
  HIPCHK(hipStreamSynchronize(H.stream));
  if (info) {
    info->iters = k;
    info->converged = converged ? 1 : 0;
    info->rel_res = f0 > 0.0 ? fn / f0 : 0.0;
    info->res0 = f0;
    info->t_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!converged) st = fail(STK_ENOTCONV, "Newton reached maxit");
  return st;
}

}  // extern "C"
