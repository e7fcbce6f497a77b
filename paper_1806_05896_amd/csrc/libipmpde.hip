// libipmpde: host driver and C ABI.
//
// One translation unit: the kernel files are included here so that every
// launch site sees its kernel.  The interior point loop (Appendix,
// Algorithm A.1) runs on the host; every vector operation of it runs in the
// kernels on the caller's stream.  Work is organised in groups: a device
// array of instance descriptors that every kernel indexes with blockIdx.z,
// so one launch advances all instances of a batch; a single problem is a
// group of one.  The only device-to-host traffic is a few scalars per
// instance per IPM iteration and per Krylov chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/ipmpde.h"
#include "common.h"
#include "kernels_ipm.hip"
#include "kernels_krylov.hip"
#include "kernels_mg.hip"
#include "kernels_mg_p2.hip"
#include "kernels_mg_p3.hip"
#include "kernels_mg_f3.hip"
#include "kernels_persist.hip"
#include "kernels_fgmres.hip"

using namespace ipm;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err = "";

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(IPMPDE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));              \
  } while (0)

#define TRY(expr)                     \
  do {                                \
    int rc_ = (expr);                 \
    if (rc_ != IPMPDE_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------------------
// allocator

static ipmpde_alloc_fn g_alloc = nullptr;
static ipmpde_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

struct Alloc {
  void* p;
  ipmpde_free_fn fr;
  void* ctx;
};

struct AllocList {
  std::vector<Alloc> a;
  int alloc(void** out, size_t bytes) {
    void* p = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    if (g_alloc) {
      p = g_alloc(bytes, g_alloc_ctx);
      if (!p) return fail(IPMPDE_ENOMEM, "allocator callback returned NULL");
      a.push_back({p, g_free, g_alloc_ctx});
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) return fail(IPMPDE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      a.push_back({p, nullptr, nullptr});
    }
    *out = p;
    return IPMPDE_OK;
  }
  template <typename T>
  int alloc_t(T** out, size_t count) {
    return alloc((void**)out, count * sizeof(T));
  }
  void release() {
    for (auto& x : a) {
      if (x.fr) x.fr(x.p, x.ctx);
      else (void)hipFree(x.p);
    }
    a.clear();
  }
};

// ---------------------------------------------------------------------------
// groups

// A captured chunk of Krylov iterations is valid for one launch geometry:
// the options, the descriptor count and the group's size maxima.
struct GraphKey {
  int mg_fp32, nu_pre, nu_post, chunk, maxit, zc, max_n, max_nlev, max_cl, flags;
  size_t coarse_lds;
  double omega, tol;
  // FGMRES: 1 + the preconditioner kind, the first Arnoldi step of the
  // captured range and the vcycles (0 for MINRES chunks)
  int fg = 0, j0 = 0, vcycles = 0;
  bool operator<(const GraphKey& o) const {
    return std::tie(mg_fp32, nu_pre, nu_post, chunk, maxit, zc, max_n, max_nlev, max_cl, flags, coarse_lds, omega, tol,
                    fg, j0, vcycles) <
           std::tie(o.mg_fp32, o.nu_pre, o.nu_post, o.chunk, o.maxit, o.zc, o.max_n, o.max_nlev, o.max_cl, o.flags,
                    o.coarse_lds, o.omega, o.tol, o.fg, o.j0, o.vcycles);
  }
};
static constexpr size_t kMaxGraphs = 64;

struct ipmpde_problem;

// A set of instances advanced together.  Each descriptor is a copy of its
// problem's template with the group's own scalar areas (ctrl, stat) and the
// per-step fields (mu, active, multigrid selection) filled in.
struct Group {
  std::vector<ipmpde_problem*> probs;
  int count = 0, dim = 0;
  int cap = 0;  // descriptor capacity
  int zc = 0;   // descriptors per launch (blockIdx.z extent); [count, zc) are inactive
  Inst* D = nullptr;             // device descriptors
  Inst* H = nullptr;             // pinned host copies
  KrylovCtrl* ctrl_d = nullptr;
  KrylovCtrl* ctrl_h = nullptr;  // pinned (the prefix up to hcol is copied back)
  double* stat_d = nullptr;
  double* stat_h = nullptr;      // pinned, 16 per instance
  hipStream_t cap_stream = nullptr;  // created at the first capture unless set (then not owned)
  bool own_cap = true;
  std::map<GraphKey, hipGraphExec_t> graphs;
  AllocList mem;
  // grid sizes (maxima over instances) after group_select
  int max_n = 0, max_nlev = 0, max_cl = 0;
  int maxN[kMaxLev] = {0};
  long maxn[kMaxLev] = {0};
  size_t coarse_lds = 0;
  bool p2 = false;   // some instance is 2D Poisson (padded coarse kernel)
  bool gen = false;  // some instance uses the generic (unpadded) level and coarse kernels
  bool cd = false;   // some instance is 2D convection-diffusion (its own coarse kernel)
  bool f3 = false;   // some instance takes the 3D finite-difference Poisson coarse kernel
  bool p3 = false;   // 3D, every instance finite-difference Poisson: the fused level kernels
  int max_cpack = 0; // longest coarse LDS image (Poisson instances)
  bool any_small = false;  // some instance runs its whole hierarchy in the coarse kernel
  bool persist = false;    // some instance takes the persistent single-workgroup MINRES kernel
  int outsel = 1;    // level-0 output buffer of a V-cycle (x2 = 1)
  bool heat = false; // heat-equation problems (a group holds only heat problems or none)
  bool q1 = false;   // Q1 finite-element problems (likewise): generic multigrid path
  int sel_pre = 0;   // 3D path: buffer holding the pre-smoothed iterate
  bool fp32 = true;
  int tile = IPMPDE_TILE_AUTO;  // tile policy of the 2D Poisson level kernels (options.mg_tile)
};

struct ipmpde_problem {
  Inst I;  // template descriptor (device pointers, problem data)
  int dim = 0, N = 0, n = 0, pde = 0;
  double eps = 1.0, alpha = 0.0, beta = 0.0;
  bool has_y = false;
  AllocList mem;   // problem data, iterates, barrier diagonals (lifetime of the handle)
  AllocList work;  // Newton/Krylov vectors, multigrid levels, reduction partials
  bool have_work = false;
  bool need_init = true;   // iterates not yet at the starting point
  bool in_engine = false;  // queued or running in a serving engine
  double* obs = nullptr;   // observation weights (device), nullptr: observed everywhere
  double* eobs = nullptr;  // Q1: observed-element weights (device), nullptr: observed everywhere
  bool obs_zero = false;   // some node is unobserved
  int nlev = 0;
  Level lv32[kMaxLev];
  Level lv64[kMaxLev];
  Level* lvd32 = nullptr;
  Level* lvd64 = nullptr;
  bool have32 = false, have64 = false;
  int coarse32 = 0, coarse64 = 0;
  void* cpack32 = nullptr;  // LDS image of the Poisson coarse levels (per precision)
  void* cpack64 = nullptr;
  void* kc32[3] = {nullptr, nullptr, nullptr};  // k-cycle level-0 arrays: b0, s[0], s[1]
  void* kc64[3] = {nullptr, nullptr, nullptr};
  int cpack_elems32 = 0, cpack_elems64 = 0;
  int f_restart = 0;
  Group* self = nullptr;  // the group of one used by the single-problem entry points
  // heat equation: nt time steps of length tau; every multigrid solve runs
  // step by step on per-step descriptors (a 2D Poisson-type instance each,
  // pointing into the space-time arrays), launched through hview
  int nt = 1;
  double tau = 0.0;
  Inst* hs_h = nullptr;  // pinned host copies of the per-step descriptors
  Inst* hs_d = nullptr;
  Group hview;           // D = hs_d + t (one step, zc = 1) or hs_d (all steps, zc = nt)
  ipmpde_stats stats;
  double mu = 1.0;
  // w of the options last applied: 1 for the unit form, the lumped mass h^dim
  // of a node under IPMPDE_MASS_HD (reported mu, measures, multipliers and
  // Theta are w times the internal unit-form values)
  double rep = 1.0;
  bool setup_done = false;
  int setup_fp32 = -1;
  const Group* setup_group = nullptr;  // group whose descriptors hold the last Newton setup
};

static bool is_pow2m1(int N) { return N >= 3 && ((N + 1) & N) == 0; }

static int level_count(int N) {
  int c = 1;
  while (N > 1) { N = (N - 1) / 2; ++c; }
  return c;
}

static size_t pow_dim(int N, int dim) { return dim == 2 ? (size_t)N * N : (size_t)N * N * N; }

// Blocks of a node-parallel launch, a multiple of 8 (one per XCD; see xcd_node).
static int nblk(long n) { return (div_up(n, kBS) + 7) & ~7; }

// LDS budget of the single-workgroup coarse kernel (gfx950 has 160 KB of
// LDS per CU), and the largest grid it takes; finer levels run as
// grid-wide kernels.
static constexpr size_t kCoarseLds = 150 * 1024;
// the FP64 kernels size their per-thread arrays for coarse levels of at most 31 x 31
static_assert((size_t)coarse_p2_elems(63) * 8 > kCoarseLds, "an FP64 63 x 63 level must not fit the coarse kernel");

// Coarse kernel kinds: the padded 2D Poisson one (finite differences and
// Q1), the 2D convection-diffusion one with staged stencil coefficients and
// the padded 3D Poisson one (finite differences and Q1).
enum { kCoarseP2 = 1, kCoarseCD = 2, kCoarseF3 = 3 };

static size_t coarse_level_elems(const Level& L, int kind) {
  if (kind == kCoarseP2) return (size_t)coarse_p2_elems(L.N);
  if (kind == kCoarseCD) return (size_t)kCoarseCDArrays * L.n;
  return (size_t)coarse_f3_elems(L.N);  // kCoarseF3
}

// Largest grid of each coarse kernel: the convection-diffusion stencil costs
// several wind evaluations per node to stage, so its 63 x 63 level runs on
// the grid-wide level kernels instead.
static int coarse_max_N(int dim, int kind) {
  if (dim == 3) return 15;
  return kind == kCoarseCD ? 31 : kCoarseP2MaxN;
}

// Elements of the 2D Poisson coarse image after its levels: the inverse of
// the 7 x 7 level's operator when the hierarchy has that level.
static size_t coarse_p2_tail(const Level* lv, int nlev, int kind) {
  if (kind != kCoarseP2 && kind != kCoarseCD) return 0;
  for (int l = 0; l < nlev; ++l)
    if (lv[l].N == kCoarseInvN) return (size_t)kCoarseInvN * kCoarseInvN * kCoarseInvN * kCoarseInvN;
  return 0;
}

static int pick_coarse(const Level* lv, int nlev, size_t elem, int dim, int kind) {
  const int nmax = coarse_max_N(dim, kind);
  int cl = nlev - 1;
  size_t need = coarse_p2_tail(lv, nlev, kind) * elem;
  for (int l = nlev - 1; l >= 0; --l) {
    need += coarse_level_elems(lv[l], kind) * elem;
    if (need > kCoarseLds || lv[l].N > nmax) break;
    cl = l;
  }
  return cl;
}

static size_t coarse_lds_bytes(const Level* lv, int nlev, int cl, size_t elem, int kind) {
  size_t need = coarse_p2_tail(lv, nlev, kind) * elem;
  for (int l = cl; l < nlev; ++l) need += coarse_level_elems(lv[l], kind) * elem;
  return need;
}

// Allow the coarse kernels more than the default 64 KB of dynamic LDS.
static int set_coarse_lds_limit() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    const void* fns[] = {(const void*)k_mg_coarse_cd<float>, (const void*)k_mg_coarse_cd<double>,
                         (const void*)k_minres_small<float>, (const void*)k_minres_small<double>,
                         (const void*)k_mg_coarse_p2<float>, (const void*)k_mg_coarse_p2<double>,
                         (const void*)k_mg_coarse_f3<float>, (const void*)k_mg_coarse_f3<double>,
                         (const void*)k_heat_sweep_p2<float>, (const void*)k_heat_sweep_p2<double>};
    for (const void* f : fns) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoarseLds);
      if (e != hipSuccess) err = e;
    }
  });
  if (err != hipSuccess) return fail(IPMPDE_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(err));
  return IPMPDE_OK;
}

static bool is_p2(const ipmpde_problem* P) { return P->dim == 2 && P->pde == IPMPDE_POISSON; }
// The padded single-workgroup coarse kernel: 2D Poisson (five-point) and Q1 (nine-point).
static bool padded_coarse(const ipmpde_problem* P) { return is_p2(P) || (P->dim == 2 && P->pde == IPMPDE_POISSON_Q1); }
static int coarse_kind(const ipmpde_problem* P) {
  if (padded_coarse(P)) return kCoarseP2;
  return P->pde == IPMPDE_CONVDIFF ? kCoarseCD : kCoarseF3;  // 3D: Poisson, finite differences or Q1
}

// The fused 3D level kernels stage cubes of (2 TC + 1 + 2 nu)^3 (descent,
// TC = 4 coarse nodes per axis) and (TF + 2 nu)^3 nodes (ascent, TF = 8) in
// static LDS; a sweep count is served when both fit (FP32: nu <= 3, FP64:
// nu = 1).  Smaller cubes recompute so much halo that the one-node-per-thread
// kernels are faster (measured: FP64 with 2^3-node cubes, 2.28 against 2.52
// solves/s at 127^3), so the other cases take those.
static bool p3_fits(size_t el, int nu) {
  if (nu < 1 || nu > 6) return false;
  const size_t wd = 9 + 2 * nu, wu = 8 + 2 * nu, wc = wu / 2 + 2;
  return 4 * el * wd * wd * wd <= 65536 && el * (4 * wu * wu * wu + wc * wc * wc) <= 65536;
}

// Elements between two reaction-term slots' coarse images: a multiple of 4,
// so every slot's image starts on 16 bytes (the coarse kernel copies it in
// 16-byte pieces).
static int cpack_stride(int elems) { return (elems + 3) & ~3; }

// Reaction-term slots of every multigrid level (see k_mg_select): the
// Schur-approximation operator's, and the two extra operators of P_Pi.
static constexpr int kReactionSlots = 3;

// Heat equation: every level array holds all nt time steps (step t at
// offset t n_l); one reaction-term slot (I/tau + M_hat restricted); the
// coarse LDS image once per step.
static int ensure_mg_heat(ipmpde_problem* P, bool fp32) {
  bool& have = fp32 ? P->have32 : P->have64;
  Level* lv = fp32 ? P->lv32 : P->lv64;
  if (have) return IPMPDE_OK;
  const size_t el = fp32 ? 4 : 8, nt = (size_t)P->nt;
  int N = P->N;
  for (int l = 0; l < P->nlev; ++l) {
    lv[l].N = N;
    lv[l].n = N * N;
    lv[l].h = 1.0 / (N + 1);
    lv[l].invN = 1.0f / (float)N;
    const size_t nb = (size_t)lv[l].n * el * nt;
    TRY(P->work.alloc(&lv[l].x, nb));
    TRY(P->work.alloc(&lv[l].x2, nb));
    TRY(P->work.alloc(&lv[l].b, nb));
    TRY(P->work.alloc(&lv[l].mh, nb));
    lv[l].mhb = lv[l].mh;
    for (void* a : {lv[l].x, lv[l].x2, lv[l].b, lv[l].mh}) HIP_TRY(hipMemset(a, 0, nb));
    N = (N - 1) / 2;
  }
  for (void*& a : (fp32 ? P->kc32 : P->kc64)) TRY(P->work.alloc(&a, (size_t)lv[0].n * el * nt));
  const int cl = pick_coarse(lv, P->nlev, el, 2, kCoarseP2);
  (fp32 ? P->coarse32 : P->coarse64) = cl;
  // per step: the levels and the inverse of the 7 x 7 level's operator
  int elems = (int)coarse_p2_tail(lv, P->nlev, kCoarseP2);
  for (int l = cl; l < P->nlev; ++l) elems += coarse_p2_elems(lv[l].N);
  void*& pk = fp32 ? P->cpack32 : P->cpack64;
  TRY(P->work.alloc(&pk, nt * elems * el));
  (fp32 ? P->cpack_elems32 : P->cpack_elems64) = elems;
  Level*& lvd = fp32 ? P->lvd32 : P->lvd64;
  TRY(P->work.alloc_t(&lvd, kMaxLev));
  HIP_TRY(hipMemcpy(lvd, lv, sizeof(Level) * kMaxLev, hipMemcpyHostToDevice));
  have = true;
  return IPMPDE_OK;
}

static int ensure_mg(ipmpde_problem* P, bool fp32) {
  TRY(set_coarse_lds_limit());
  if (P->pde == IPMPDE_HEAT) return ensure_mg_heat(P, fp32);
  bool& have = fp32 ? P->have32 : P->have64;
  Level* lv = fp32 ? P->lv32 : P->lv64;
  if (have) return IPMPDE_OK;
  const size_t el = fp32 ? 4 : 8;
  int N = P->N;
  for (int l = 0; l < P->nlev; ++l) {
    lv[l].N = N;
    lv[l].n = (int)pow_dim(N, P->dim);
    lv[l].h = 1.0 / (N + 1);
    lv[l].invN = 1.0f / (float)N;
    const size_t nb = (size_t)lv[l].n * el;
    TRY(P->work.alloc(&lv[l].x, nb));
    TRY(P->work.alloc(&lv[l].x2, nb));
    TRY(P->work.alloc(&lv[l].b, nb));
    TRY(P->work.alloc(&lv[l].mh, kReactionSlots * nb));  // slot 2 stays zero
    lv[l].mhb = lv[l].mh;
    HIP_TRY(hipMemset(lv[l].x, 0, nb));
    HIP_TRY(hipMemset(lv[l].x2, 0, nb));
    HIP_TRY(hipMemset(lv[l].b, 0, nb));
    HIP_TRY(hipMemset(lv[l].mh, 0, kReactionSlots * nb));
    N = (N - 1) / 2;
  }
  for (void*& a : (fp32 ? P->kc32 : P->kc64)) TRY(P->work.alloc(&a, (size_t)lv[0].n * el));
  const int cl = pick_coarse(lv, P->nlev, el, P->dim, coarse_kind(P));
  (fp32 ? P->coarse32 : P->coarse64) = cl;
  if (padded_coarse(P) || coarse_kind(P) == kCoarseCD) {
    // the coarse kernel's LDS image per reaction-term slot
    int elems = 0;
    if (padded_coarse(P)) {
      elems = (int)coarse_p2_tail(lv, P->nlev, kCoarseP2);
      for (int l = cl; l < P->nlev; ++l) elems += coarse_p2_elems(lv[l].N);
    } else {
      elems = (int)coarse_p2_tail(lv, P->nlev, kCoarseCD);
      for (int l = cl; l < P->nlev; ++l) elems += (int)coarse_level_elems(lv[l], kCoarseCD);
    }
    void*& pk = fp32 ? P->cpack32 : P->cpack64;
    TRY(P->work.alloc(&pk, (size_t)kReactionSlots * cpack_stride(elems) * el));
    (fp32 ? P->cpack_elems32 : P->cpack_elems64) = elems;
  }
  Level*& lvd = fp32 ? P->lvd32 : P->lvd64;
  TRY(P->work.alloc_t(&lvd, kMaxLev));
  HIP_TRY(hipMemcpy(lvd, lv, sizeof(Level) * kMaxLev, hipMemcpyHostToDevice));
  have = true;
  return IPMPDE_OK;
}

static int ensure_fgmres(ipmpde_problem* P, int restart) {
  if (P->I.fV && P->f_restart >= restart) return IPMPDE_OK;
  const size_t n4 = 4 * (size_t)P->n;
  TRY(P->work.alloc_t(&P->I.fV, (size_t)(restart + 1) * n4));
  TRY(P->work.alloc_t(&P->I.fZ, (size_t)restart * n4));
  P->f_restart = restart;
  return IPMPDE_OK;
}

// partial-sum capacity for reductions over `blocks` blocks (3 values each)
// and for the FGMRES block dot products (61 x 256)
static int partials_words(int blocks) { return std::max(4 * blocks, 64 * kBS) + 64; }
static int ensure_partials(ipmpde_problem* P, int blocks) {
  const int need = partials_words(blocks);
  if (P->I.nparts >= need) return IPMPDE_OK;
  TRY(P->work.alloc_t(&P->I.partials, (size_t)need));
  P->I.nparts = need;
  return IPMPDE_OK;
}

// The Newton right-hand side, direction and Krylov vectors (4n each).
static constexpr int kKrylovVecs = 11;
static void krylov_vecs(Inst& I, double** v[kKrylovVecs]) {
  double** all[kKrylovVecs] = {&I.rhs, &I.X, &I.Q, &I.R, &I.Rt, &I.V[0], &I.V[1], &I.Z[0], &I.Z[1],
                               &I.W[0], &I.W[1]};
  std::copy(all, all + kKrylovVecs, v);
}

// Workspace of the Newton solves; allocated on first use (or admission to a
// serving engine) and released when the problem leaves the engine.
static int ensure_work(ipmpde_problem* P) {
  if (P->have_work) return IPMPDE_OK;
  const size_t n4 = 4 * (size_t)P->n;
  double** v[kKrylovVecs];
  krylov_vecs(P->I, v);
  for (double** p : v) TRY(P->work.alloc_t(p, n4));
  for (double** p : v) HIP_TRY(hipMemset(*p, 0, n4 * sizeof(double)));
  TRY(ensure_partials(P, nblk((long)P->n)));
  P->have_work = true;
  return IPMPDE_OK;
}

static void release_work(ipmpde_problem* P) {
  P->work.release();
  Inst& I = P->I;
  double** v[kKrylovVecs];
  krylov_vecs(I, v);
  for (double** p : v) *p = nullptr;
  I.fV = I.fZ = nullptr;
  I.partials = nullptr;
  I.nparts = 0;
  P->f_restart = 0;
  P->have32 = P->have64 = false;
  P->lvd32 = P->lvd64 = nullptr;
  P->cpack32 = P->cpack64 = nullptr;
  for (int k = 0; k < 3; ++k) P->kc32[k] = P->kc64[k] = nullptr;
  P->cpack_elems32 = P->cpack_elems64 = 0;
  for (int l = 0; l < kMaxLev; ++l) P->lv32[l] = P->lv64[l] = Level{};
  P->have_work = false;
  P->setup_done = false;
}

static void group_release(Group* G) {
  if (!G) return;
  for (auto& kv : G->graphs) (void)hipGraphExecDestroy(kv.second);
  G->graphs.clear();
  G->mem.release();
  if (G->H) (void)hipHostFree(G->H);
  if (G->ctrl_h) (void)hipHostFree(G->ctrl_h);
  if (G->stat_h) (void)hipHostFree(G->stat_h);
  if (G->cap_stream && G->own_cap) (void)hipStreamDestroy(G->cap_stream);
  delete G;
}

// A group with room for `cap` descriptors holding `probs` (cap >= size).
static int group_create(const std::vector<ipmpde_problem*>& probs, int cap, int dim, Group** out) {
  Group* G = new Group();
  G->probs = probs;
  G->count = (int)probs.size();
  G->cap = cap;
  G->zc = G->count;
  G->dim = dim;
  G->heat = !probs.empty() && probs[0]->pde == IPMPDE_HEAT;
  G->q1 = !probs.empty() && probs[0]->pde == IPMPDE_POISSON_Q1;
  auto bail = [&](int rc) { group_release(G); return rc; };
  int rc;
  if ((rc = G->mem.alloc_t(&G->D, cap))) return bail(rc);
  if ((rc = G->mem.alloc_t(&G->ctrl_d, cap))) return bail(rc);
  if ((rc = G->mem.alloc_t(&G->stat_d, 16 * (size_t)cap))) return bail(rc);
  hipError_t e;
  if ((e = hipMemset(G->ctrl_d, 0, sizeof(KrylovCtrl) * cap)) != hipSuccess ||
      (e = hipMemset(G->stat_d, 0, 16 * sizeof(double) * cap)) != hipSuccess ||
      (e = hipHostMalloc((void**)&G->H, sizeof(Inst) * cap, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&G->ctrl_h, sizeof(KrylovCtrl) * cap, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&G->stat_h, 16 * sizeof(double) * cap, hipHostMallocDefault)) != hipSuccess)
    return bail(fail(IPMPDE_EDEVICE, std::string("group setup: ") + hipGetErrorString(e)));
  std::memset(G->ctrl_h, 0, sizeof(KrylovCtrl) * cap);
  std::memset(G->stat_h, 0, 16 * sizeof(double) * cap);
  std::memset((void*)G->H, 0, sizeof(Inst) * cap);  // active = 0
  for (int i = 0; i < G->count; ++i) {
    G->H[i] = probs[i]->I;
    G->H[i].ctrl = G->ctrl_d + i;
    G->H[i].stat = G->stat_d + 16 * (size_t)i;
    G->H[i].active = 1;
    G->H[i].mu = 1.0;
    G->H[i].alpha0 = 0.995;
  }
  *out = G;
  return IPMPDE_OK;
}

// The coarse kernel's copies of its level fields (after lv, nlev and
// coarse_lev are set).
static void coarse_copies(Inst& d) {
  const int cl = d.coarse_lev;
  d.cN0 = d.lv[cl].N;
  d.cb = d.lv[cl].b;
  d.cx = d.lv[cl].x;
  for (int q = 0; q < kCoarseLevels; ++q) {
    const int N = ((d.cN0 + 1) >> q) - 1;
    const double h = 1.0 / (N + 1);  // as lv[].h
    d.cih2[q] = N > 0 ? 1.0 / (h * h) : 0.0;
  }
}

// Heat equation: the per-time-step descriptors (from the problem's filled
// descriptor d) and the launch view over them.  Step t is a 2D Poisson-type
// instance with operator I/tau + A_h + M_hat_t whose arrays are the t-th
// slices of the space-time arrays.
static void heat_steps(ipmpde_problem* P, const Inst& d, bool fp32) {
  const Level* lv = fp32 ? P->lv32 : P->lv64;
  const size_t el = fp32 ? 4 : 8;
  const int n2 = P->N * P->N;
  void* const* kc = fp32 ? P->kc32 : P->kc64;
  char* pk = (char*)(fp32 ? P->cpack32 : P->cpack64);
  const int pe = fp32 ? P->cpack_elems32 : P->cpack_elems64;
  auto at = [](void* base, size_t off) { return (void*)((char*)base + off); };
  for (int t = 0; t < P->nt; ++t) {
    Inst& S = P->hs_h[t];
    S = d;
    S.pde = IPMPDE_POISSON;
    S.n = n2;
    S.nt = 1;
    for (int l = 0; l < P->nlev; ++l) {
      const size_t off = (size_t)t * lv[l].n * el;
      S.lv[l] = lv[l];
      S.lv[l].x = at(lv[l].x, off);
      S.lv[l].x2 = at(lv[l].x2, off);
      S.lv[l].b = at(lv[l].b, off);
      S.lv[l].mh = at(lv[l].mh, off);
      S.lv[l].mhb = S.lv[l].mh;
    }
    const size_t o2 = (size_t)t * n2;
    S.ty = d.ty + o2;
    S.tw = d.tw + o2;
    S.tv = d.tv + o2;
    S.obs = d.obs ? d.obs + o2 : nullptr;
    S.kc_b0 = at(kc[0], o2 * el);
    S.kc_s[0] = at(kc[1], o2 * el);
    S.kc_s[1] = at(kc[2], o2 * el);
    S.coarse_p2 = 1;
    S.cpack = pk + (size_t)t * pe * el;
    S.cpackb = S.cpack;
    S.cpack_slot = pe;
    S.cpack_elems = pe;
    S.ppi = 0;
    S.lvd = nullptr;
    coarse_copies(S);
  }
  Group& V = P->hview;
  V.count = 1;
  V.dim = 2;
  V.zc = 1;
  V.D = P->hs_d;
  V.H = P->hs_h;
  V.fp32 = fp32;
  V.max_n = n2;
  V.max_nlev = P->nlev;
  V.max_cl = d.coarse_lev;
  std::fill(V.maxN, V.maxN + kMaxLev, 0);
  std::fill(V.maxn, V.maxn + kMaxLev, 0);
  for (int l = 0; l < P->nlev; ++l) {
    V.maxN[l] = lv[l].N;
    V.maxn[l] = lv[l].n;
  }
  V.coarse_lds = coarse_lds_bytes(lv, P->nlev, d.coarse_lev, el, kCoarseP2);
  V.p2 = true;
  V.gen = false;
  V.max_cpack = pe;
  V.any_small = d.coarse_lev == 0;
  V.outsel = 1;
}

// Refresh the descriptors from the problems' templates (keeping the
// per-step fields) and select the multigrid precision and schedule.
static int group_select(Group* G, const ipmpde_options& o) {
  const bool fp32 = o.mg_precision == IPMPDE_FP32;
  G->fp32 = fp32;
  G->tile = o.mg_tile;
  G->max_n = 0;
  G->max_nlev = 0;
  G->max_cl = 0;
  G->coarse_lds = 0;
  G->p2 = false;
  G->gen = false;
  G->cd = false;
  G->f3 = false;
  G->p3 = false;
  G->any_small = false;
  G->persist = false;
  G->max_cpack = 0;
  std::fill(G->maxN, G->maxN + kMaxLev, 0);
  std::fill(G->maxn, G->maxn + kMaxLev, 0);
  for (int i = 0; i < G->count; ++i) {
    ipmpde_problem* P = G->probs[i];
    TRY(ensure_work(P));
    TRY(ensure_mg(P, fp32));
    if (o.krylov == IPMPDE_FGMRES) TRY(ensure_fgmres(P, o.restart));
  }
  for (int i = 0; i < G->count; ++i) TRY(ensure_partials(G->probs[i], nblk(std::max(G->max_n, G->probs[i]->n))));
  for (int i = 0; i < G->count; ++i) G->max_n = std::max(G->max_n, G->probs[i]->n);
  for (int i = 0; i < G->count; ++i) TRY(ensure_partials(G->probs[i], nblk(G->max_n)));
  for (int i = 0; i < G->count; ++i) {
    ipmpde_problem* P = G->probs[i];
    Inst& d = G->H[i];
    const int active = d.active;
    const double mu = d.mu, a0 = d.alpha0;
    d = P->I;
    d.ctrl = G->ctrl_d + i;
    d.stat = G->stat_d + 16 * (size_t)i;
    d.active = active;
    d.mu = mu;
    d.alpha0 = a0;
    const Level* lv = fp32 ? P->lv32 : P->lv64;
    for (int l = 0; l < P->nlev; ++l) d.lv[l] = lv[l];
    d.nlev = P->nlev;
    d.coarse_lev = fp32 ? P->coarse32 : P->coarse64;
    d.lvd = fp32 ? P->lvd32 : P->lvd64;
    d.mg_fp32 = fp32 ? 1 : 0;
    d.nu_pre = o.nu_pre;
    d.nu_post = o.nu_post;
    d.vcycles = o.vcycles;
    d.omega = o.omega > 0 ? o.omega : (P->dim == 2 ? 0.8 : 6.0 / 7.0);
    G->max_nlev = std::max(G->max_nlev, P->nlev);
    G->max_cl = std::max(G->max_cl, d.coarse_lev);
    G->any_small = G->any_small || d.coarse_lev == 0;
    G->persist = G->persist || (is_p2(P) && d.coarse_lev == 0 && o.krylov == IPMPDE_MINRES && o.precond == IPMPDE_PD &&
                                o.vcycles == 1 && !P->obs && P->pde != IPMPDE_HEAT);
    for (int l = 0; l < P->nlev; ++l) {
      G->maxN[l] = std::max(G->maxN[l], lv[l].N);
      G->maxn[l] = std::max(G->maxn[l], (long)lv[l].n);
    }
    d.coarse_p2 = is_p2(P) ? 1 : (padded_coarse(P) ? 2 : 0);
    d.cpack = fp32 ? P->cpack32 : P->cpack64;
    d.cpackb = d.cpack;
    d.cpack_slot = cpack_stride(fp32 ? P->cpack_elems32 : P->cpack_elems64);
    d.obs = P->obs;
    d.eobs = P->eobs;
    d.ppi = o.precond == IPMPDE_PPI ? 1 : 0;
    void* const* kc = fp32 ? P->kc32 : P->kc64;
    d.kc_b0 = kc[0];
    d.kc_s[0] = kc[1];
    d.kc_s[1] = kc[2];
    d.cpack_elems = fp32 ? P->cpack_elems32 : P->cpack_elems64;
    coarse_copies(d);
    G->max_cpack = std::max(G->max_cpack, d.cpack_elems);
    G->p2 = G->p2 || padded_coarse(P);
    G->gen = G->gen || !padded_coarse(P);
    G->cd = G->cd || coarse_kind(P) == kCoarseCD;
    G->f3 = G->f3 || coarse_kind(P) == kCoarseF3;
    G->coarse_lds = std::max(G->coarse_lds, coarse_lds_bytes(lv, P->nlev, d.coarse_lev, fp32 ? 4 : 8, coarse_kind(P)));
  }
  if (G->heat)
    for (int i = 0; i < G->count; ++i) {
      heat_steps(G->probs[i], G->H[i], fp32);
      G->H[i].hsteps = G->probs[i]->hs_d;
    }
  G->p3 = G->dim == 3 && !G->heat && p3_fits(fp32 ? 4 : 8, o.nu_pre) && p3_fits(fp32 ? 4 : 8, o.nu_post);
  for (int i = 0; i < G->count; ++i) G->p3 = G->p3 && G->probs[i]->pde == IPMPDE_POISSON;
  if (G->dim == 2 || G->p3) {
    G->outsel = 1;
  } else {
    G->sel_pre = o.nu_pre & 1;
    G->outsel = G->sel_pre ^ (o.nu_post & 1);
  }
  return IPMPDE_OK;
}

// Upload the descriptors.  The copy reads the pinned host array when it
// executes, not when it is enqueued: the host copies must not be edited
// again until the stream has been synchronised past it (every caller's next
// edit follows a read-back that does so, or an explicit wait).
static int group_sync(Group* G, hipStream_t s) {
  for (int i = G->count; i < G->zc; ++i) G->H[i].active = 0;
  HIP_TRY(hipMemcpyAsync(G->D, G->H, sizeof(Inst) * G->zc, hipMemcpyHostToDevice, s));
  if (G->heat)
    for (int i = 0; i < G->count; ++i) {
      const ipmpde_problem* P = G->probs[i];
      HIP_TRY(hipMemcpyAsync(P->hs_d, P->hs_h, sizeof(Inst) * P->nt, hipMemcpyHostToDevice, s));
    }
  return IPMPDE_OK;
}

static dim3 gz(const Group* G, long nthreads, int y = 1) { return dim3(nblk(std::max(nthreads, 1L)), y, G->zc); }

static int read_ctrl(Group* G, hipStream_t s) {
  HIP_TRY(hipMemcpy2DAsync(G->ctrl_h, sizeof(KrylovCtrl), G->ctrl_d, sizeof(KrylovCtrl), offsetof(KrylovCtrl, hcol),
                           G->count, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IPMPDE_OK;
}

static int read_stat(Group* G, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(G->stat_h, G->stat_d, 16 * sizeof(double) * G->count, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// options

extern "C" int ipmpde_default_options(ipmpde_options* o) {
  if (!o) return fail(IPMPDE_EINVAL, "opts is NULL");
  o->sigma = 0.2;
  o->alpha0 = 0.995;
  o->eps_p = o->eps_d = o->eps_c = 1e-6;
  o->mu0 = 1.0;
  o->ipm_maxit = 200;
  o->fixed_nli = 0;
  o->krylov = IPMPDE_MINRES;
  o->precond = IPMPDE_PD;
  o->restart = 30;
  o->krylov_tol = 1e-10;
  o->krylov_maxit = 500;
  o->vcycles = 1;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->omega = 0.0;
  o->mg_precision = IPMPDE_FP32;
  o->chunk = 8;
  o->use_graphs = 1;
  o->mu_rule = IPMPDE_MU_PAPER;
  o->mass_scaling = IPMPDE_MASS_UNIT;
  o->mg_tile = IPMPDE_TILE_AUTO;
  o->lanes = 1;
  return IPMPDE_OK;
}

// Largest number of lanes (concurrent sub-batches) of a batch solve.
static constexpr int kMaxLanes = 16;

static int check_options(const ipmpde_options& o) {
  if (!(o.sigma > 0 && o.sigma < 1)) return fail(IPMPDE_EINVAL, "sigma must lie in (0,1)");
  if (!(o.alpha0 > 0 && o.alpha0 < 1)) return fail(IPMPDE_EINVAL, "alpha0 must lie in (0,1)");
  if (!(o.eps_p > 0 && o.eps_d > 0 && o.eps_c > 0)) return fail(IPMPDE_EINVAL, "tolerances must be positive");
  if (!(o.mu0 > 0)) return fail(IPMPDE_EINVAL, "mu0 must be positive");
  if (o.ipm_maxit < 1 || o.ipm_maxit > IPMPDE_MAX_HIST - 1) return fail(IPMPDE_EINVAL, "ipm_maxit out of range");
  if (o.fixed_nli < 0 || o.fixed_nli > IPMPDE_MAX_HIST - 1) return fail(IPMPDE_EINVAL, "fixed_nli out of range");
  if (o.krylov != IPMPDE_MINRES && o.krylov != IPMPDE_FGMRES) return fail(IPMPDE_EINVAL, "unknown krylov");
  if (o.precond != IPMPDE_PD && o.precond != IPMPDE_PT && o.precond != IPMPDE_PPI)
    return fail(IPMPDE_EINVAL, "unknown precond");
  if (o.precond == IPMPDE_PPI && o.krylov != IPMPDE_FGMRES)
    return fail(IPMPDE_EINVAL, "P_Pi is not symmetric: it requires FGMRES");
  if (o.precond == IPMPDE_PT && o.krylov != IPMPDE_FGMRES)
    return fail(IPMPDE_EINVAL, "the block-triangular preconditioner needs FGMRES");
  if (o.restart < 1 || o.restart > 60) return fail(IPMPDE_EINVAL, "restart must be in [1,60]");
  if (!(o.krylov_tol > 0 && o.krylov_tol < 1)) return fail(IPMPDE_EINVAL, "krylov_tol must be in (0,1)");
  if (o.krylov_maxit < 1) return fail(IPMPDE_EINVAL, "krylov_maxit must be >= 1");
  if (o.vcycles < 1 || o.vcycles > 8) return fail(IPMPDE_EINVAL, "vcycles must be in [1, 8]");
  if (o.nu_pre < 1 || o.nu_pre > 6 || o.nu_post < 1 || o.nu_post > 6) return fail(IPMPDE_EINVAL, "nu out of [1,6]");
  if (o.krylov == IPMPDE_MINRES && o.nu_pre != o.nu_post)
    return fail(IPMPDE_EINVAL, "MINRES needs nu_pre == nu_post (symmetric preconditioner)");
  if (!(o.omega >= 0 && o.omega < 1.5)) return fail(IPMPDE_EINVAL, "omega out of range");
  if (o.mg_precision != IPMPDE_FP32 && o.mg_precision != IPMPDE_FP64) return fail(IPMPDE_EINVAL, "bad mg_precision");
  if (o.chunk < 2 || o.chunk > 64 || (o.chunk & 1)) return fail(IPMPDE_EINVAL, "chunk must be even in [2,64]");
  if (o.mu_rule != IPMPDE_MU_PAPER && o.mu_rule != IPMPDE_MU_CENTRAL) return fail(IPMPDE_EINVAL, "bad mu_rule");
  if (o.mass_scaling != IPMPDE_MASS_UNIT && o.mass_scaling != IPMPDE_MASS_HD)
    return fail(IPMPDE_EINVAL, "bad mass_scaling");
  if (o.mg_tile != IPMPDE_TILE_AUTO && o.mg_tile != IPMPDE_TILE_SMALL && o.mg_tile != IPMPDE_TILE_LARGE)
    return fail(IPMPDE_EINVAL, "bad mg_tile");
  if (o.lanes < 0 || o.lanes > kMaxLanes) return fail(IPMPDE_EINVAL, "lanes must be in [0, 16]");
  return IPMPDE_OK;
}

static int resolve_opts(const ipmpde_options* in, ipmpde_options* out) {
  if (in) *out = *in;
  else ipmpde_default_options(out);
  return check_options(*out);
}

// The literal weighting of eq. (pb_fe_lin) multiplies the objective and the
// state equation by the lumped mass w = h^dim of a node; the device always
// runs the unit form (everything divided by w), which takes the same Newton
// steps when mu0 and the tolerances are divided by w.  Returns the unit-form
// options and records w for reporting.
static int unit_form(ipmpde_problem* P, const ipmpde_options& o, ipmpde_options* u) {
  *u = o;
  P->rep = 1.0;
  if (o.mass_scaling != IPMPDE_MASS_HD) return IPMPDE_OK;
  if (P->pde == IPMPDE_HEAT) return fail(IPMPDE_EINVAL, "the h^d weighting is defined for the stationary problems");
  const double h = 1.0 / (P->N + 1);
  const double w = P->dim == 3 ? h * h * h : h * h;
  u->mu0 /= w;
  u->eps_p /= w;
  u->eps_d /= w;
  u->eps_c /= w;
  P->rep = w;
  return IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// multigrid launch sequence (all instances of the group)

template <typename T>
static void launch_coarse(Group* G, int transpose, int guard, hipStream_t s) {
  // each instance takes the kernel it would take alone (the other one
  // returns at once for it), so batched and solo solves round alike
  if (G->p2) hipLaunchKernelGGL(k_mg_coarse_p2<T>, dim3(1, 1, G->zc), dim3(kCoarseBS), G->coarse_lds, s, G->D, guard);
  if (G->f3) hipLaunchKernelGGL(k_mg_coarse_f3<T>, dim3(1, 1, G->zc), dim3(kCoarseBS), G->coarse_lds, s, G->D, guard);
  if (G->cd)
    hipLaunchKernelGGL(k_mg_coarse_cd<T>, dim3(1, 1, G->zc), dim3(kCoarseBS), G->coarse_lds, s, G->D, transpose,
                       guard);
}

// 3D (generic) V-cycle: per level nu_pre sweeps, residual + restriction,
// coarse kernel, prolongation + nu_post sweeps.  Level-0 output: G->outsel.
template <typename T>
static void mg_vcycle_generic(Group* G, int transpose, int guard, hipStream_t s) {
  const int nu_pre = G->H[0].nu_pre, nu_post = G->H[0].nu_post;
  // the LDS-blocked sweep and residual (the 3D operators are symmetric: transpose changes nothing)
  auto g3 = [&](int l) { return dim3((mg3_blocks(G->maxN[l]) + 7) & ~7, 1, G->zc); };
  auto sweep = [&](int l, int a, int c, int first) {
    hipLaunchKernelGGL(k_mg_level3<T>, g3(l), dim3(kBS), 0, s, G->D, l, a, c, first, 0, guard);
  };
  for (int l = 0; l < G->max_cl; ++l) {
    int a = 0, c = 1;
    for (int sw = 0; sw < nu_pre; ++sw) {
      sweep(l, a, c, sw == 0 ? 1 : 0);
      std::swap(a, c);
    }
    hipLaunchKernelGGL(k_mg_level3<T>, g3(l), dim3(kBS), 0, s, G->D, l, a, c, 0, 1, guard);
    hipLaunchKernelGGL(k_mg_restrict_r<T>, gz(G, G->maxn[l + 1]), dim3(kBS), 0, s, G->D, l, c, guard);
  }
  launch_coarse<T>(G, transpose, guard, s);
  for (int l = G->max_cl - 1; l >= 0; --l) {
    int a = G->sel_pre, c = 1 - a;
    hipLaunchKernelGGL(k_mg_prolong<T>, gz(G, G->maxn[l]), dim3(kBS), 0, s, G->D, l, a, G->outsel, guard);
    for (int sw = 0; sw < nu_post; ++sw) {
      sweep(l, a, c, 0);
      std::swap(a, c);
    }
  }
}

template <typename T>
static void launch_down2d(int nu, dim3 g, size_t lds, hipStream_t s, const Inst* D, int l, int scaled, int tr, int guard) {
  switch (nu) {
#define D_(NU) case NU: hipLaunchKernelGGL((k_mg_down2d<T, NU>), g, dim3(kBS), lds, s, D, l, scaled, tr, guard); break;
    D_(1) D_(2) D_(3) D_(4) D_(5) D_(6)
#undef D_
  }
}
template <typename T>
static void launch_up2d(int nu, dim3 g, size_t lds, hipStream_t s, const Inst* D, int l, int tr, int guard) {
  switch (nu) {
#define U_(NU) case NU: hipLaunchKernelGGL((k_mg_up2d<T, NU>), g, dim3(kBS), lds, s, D, l, tr, guard); break;
    U_(1) U_(2) U_(3) U_(4) U_(5) U_(6)
#undef U_
  }
}

// Tile choice of the Poisson level kernels: the large tiles recompute less
// halo but make fewer workgroups, so they are taken when the launch still
// has at least this many.
static constexpr long kBigTileMinGroups = 2048;

// Large tiles for a launch of `groups` large-tile workgroups under the
// group's policy (options.mg_tile): by the workgroup count, or forced.
static bool big_tiles(const Group* G, long groups) {
  if (G->tile == IPMPDE_TILE_SMALL) return false;
  if (G->tile == IPMPDE_TILE_LARGE) return true;
  return groups >= kBigTileMinGroups;
}

// Workgroups of a Poisson level launch: each takes a run of tiles, as many as
// keep the launch near this many workgroups, so that a workgroup loads its
// next tile while it smooths the current one instead of a new workgroup
// waiting for its first loads.  Measured on the batched 8 x 511^2 solve
// (runs of 8 / 4 / 2 tiles at the finest level): 512 workgroups 229.9 ms,
// 1024 198.6 ms, 2048 189.3 ms, 4096 186.3 ms.
static constexpr long kTileRunGroups = 4096;
// Threads per workgroup of the large tiles (their regions hold 37^2 / 36^2
// nodes, about three per thread per phase at 512 threads).
static constexpr int kP2BigBS = 512;
static int tile_run_length(int nt, int zc) {
  return std::max(1, div_up((long)nt * nt * zc, kTileRunGroups));
}

template <typename T, int NU, int ST>
static void launch_down_p2_nu(const Group* G, int l, int scaled, int guard, hipStream_t s) {
  const int Nc = G->maxN[l + 1];
  if constexpr (p2_down_lds<T, NU, 16>() <= kStaticLdsMax) {
    const int nt = div_up(Nc, 16);
    if (big_tiles(G, (long)nt * nt * G->zc)) {
      const int tpw = tile_run_length(nt, G->zc);
      hipLaunchKernelGGL((k_mg_down_p2<T, NU, 16, ST, kP2BigBS>), dim3(div_up((long)nt * nt, tpw), 1, G->zc),
                         dim3(kP2BigBS), 0, s, G->D, l, scaled, guard, nt, tpw);
      return;
    }
  }
  const int nt = div_up(Nc, 8);
  const int tpw = tile_run_length(nt, G->zc);
  hipLaunchKernelGGL((k_mg_down_p2<T, NU, 8, ST>), dim3(div_up((long)nt * nt, tpw), 1, G->zc), dim3(kBS), 0, s, G->D,
                     l, scaled, guard, nt, tpw);
}

template <typename T, int NU, int ST>
static void launch_up_p2_nu(const Group* G, int l, int guard, hipStream_t s) {
  const int N = G->maxN[l];
  if constexpr (p2_up_lds<T, NU, 32>() <= kStaticLdsMax) {
    const int nt = div_up(N, 32);
    if (big_tiles(G, (long)nt * nt * G->zc)) {
      const int tpw = tile_run_length(nt, G->zc);
      hipLaunchKernelGGL((k_mg_up_p2<T, NU, 32, ST, kP2BigBS>), dim3(div_up((long)nt * nt, tpw), 1, G->zc),
                         dim3(kP2BigBS), 0, s, G->D, l, guard, nt, tpw);
      return;
    }
  }
  const int nt = div_up(N, 16);
  const int tpw = tile_run_length(nt, G->zc);
  hipLaunchKernelGGL((k_mg_up_p2<T, NU, 16, ST>), dim3(div_up((long)nt * nt, tpw), 1, G->zc), dim3(kBS), 0, s, G->D,
                     l, guard, nt, tpw);
}

// One descent (smoothing + residual + restriction) of level l for every
// instance: the Poisson kernels for the Poisson instances, the generic ones
// for the others (each kernel returns at once for the other kind).
template <typename T>
static void launch_down_level(const Group* G, int l, int scaled, int transpose, int guard, hipStream_t s) {
  const int nu = G->H[0].nu_pre;
  if (G->gen) {
    const size_t ldd = 4 * (size_t)down_width(nu) * down_width(nu) * sizeof(T);
    const int nt = div_up(G->maxN[l + 1], kTC);
    launch_down2d<T>(nu, dim3(nt, nt, G->zc), ldd, s, G->D, l, scaled, transpose, guard);
  }
  if (G->p2) {
    switch (nu) {
#define D_(NU)                                                      \
  case NU:                                                          \
    if (G->q1) launch_down_p2_nu<T, NU, 9>(G, l, scaled, guard, s); \
    else launch_down_p2_nu<T, NU, 5>(G, l, scaled, guard, s);       \
    break;
      D_(1) D_(2) D_(3) D_(4) D_(5) D_(6)
#undef D_
    }
  }
}

// One ascent (prolongation + smoothing) of level l for every instance.
template <typename T>
static void launch_up_level(const Group* G, int l, int transpose, int guard, hipStream_t s) {
  const int nu = G->H[0].nu_post;
  if (G->gen) {
    const size_t ldu = 4 * (size_t)up_width(nu) * up_width(nu) * sizeof(T);
    const int nt = div_up(G->maxN[l], kTF);
    launch_up2d<T>(nu, dim3(nt, nt, G->zc), ldu, s, G->D, l, transpose, guard);
  }
  if (G->p2) {
    switch (nu) {
#define U_(NU)                                              \
  case NU:                                                  \
    if (G->q1) launch_up_p2_nu<T, NU, 9>(G, l, guard, s);   \
    else launch_up_p2_nu<T, NU, 5>(G, l, guard, s);         \
    break;
      U_(1) U_(2) U_(3) U_(4) U_(5) U_(6)
#undef U_
    }
  }
}

// 2D V-cycle with the fused level kernels: per level one descent launch
// (smoothing + residual + restriction) and one ascent launch (prolongation +
// smoothing).  scaled: the level-0 right-hand side is (1 + Theta_y) times the
// previous V-cycle's output.  Output: level 0's x2 (x for instances whose
// whole hierarchy fits the coarse kernel).
template <typename T>
static void mg_vcycle_2d(Group* G, int transpose, int guard, int scaled, hipStream_t s) {
  for (int l = 0; l < G->max_cl; ++l) launch_down_level<T>(G, l, (l == 0) ? scaled : 0, transpose, guard, s);
  launch_coarse<T>(G, transpose, guard, s);
  for (int l = G->max_cl - 1; l >= 0; --l) launch_up_level<T>(G, l, transpose, guard, s);
}

template <typename T, int NU>
static void launch_down_p3_nu(const Group* G, int l, int scaled, int guard, hipStream_t s) {
  const int Nc = G->maxN[l + 1];
  // the cubes' own fine nodes 2 J ... 2 J + 2 TC - 1 must cover the N = 2 Nc + 1 fine nodes
#define L_(TC)                                                                                                 \
  {                                                                                                            \
    const int nt = div_up(Nc + 1, TC);                                                                         \
    hipLaunchKernelGGL((k_mg_down_p3<T, NU, TC>), dim3(nt, nt * nt, G->zc), dim3(kP3BS), 0, s, G->D, l, scaled, \
                       guard);                                                                                 \
  }
  // (5^3 coarse nodes per cube, 54 KB of LDS in FP32, measured slower: fewer workgroups fit a CU)
  if constexpr (p3_down_lds<T, NU, 4>() <= kStaticLdsMax) L_(4)  // else never called: p3_fits excludes it
#undef L_
}

template <typename T, int NU>
static void launch_up_p3_nu(const Group* G, int l, int guard, hipStream_t s) {
  const int N = G->maxN[l];
#define L_(TF)                                                                                                     \
  {                                                                                                                \
    const int nt = div_up(N, TF);                                                                                  \
    hipLaunchKernelGGL((k_mg_up_p3<T, NU, TF>), dim3(nt, nt * nt, G->zc), dim3(kP3BS), 0, s, G->D, l, guard);       \
  }
  if constexpr (p3_up_lds<T, NU, 8>() <= kStaticLdsMax) L_(8)  // else never called: p3_fits excludes it
#undef L_
}

// 3D finite-difference V-cycle with the fused level kernels (as the 2D one).
// Output: level 0's x2 (x for instances whose whole hierarchy fits the coarse
// kernel).
template <typename T>
static void mg_vcycle_p3(Group* G, int transpose, int guard, int scaled, hipStream_t s) {
  const int nu_pre = G->H[0].nu_pre, nu_post = G->H[0].nu_post;
  for (int l = 0; l < G->max_cl; ++l) {
    const int sc = l == 0 ? scaled : 0;
    switch (nu_pre) {
#define D_(NU) case NU: launch_down_p3_nu<T, NU>(G, l, sc, guard, s); break;
      D_(1) D_(2) D_(3) D_(4) D_(5) D_(6)
#undef D_
    }
  }
  launch_coarse<T>(G, transpose, guard, s);
  for (int l = G->max_cl - 1; l >= 0; --l) {
    switch (nu_post) {
#define U_(NU) case NU: launch_up_p3_nu<T, NU>(G, l, guard, s); break;
      U_(1) U_(2) U_(3) U_(4) U_(5) U_(6)
#undef U_
    }
  }
}

// One V-cycle of the group's multigrid path.
template <typename T>
static void mg_vcycle(Group* G, int transpose, int guard, int scaled, hipStream_t s) {
  if (G->dim == 2) mg_vcycle_2d<T>(G, transpose, guard, scaled, s);
  else if (G->p3) mg_vcycle_p3<T>(G, transpose, guard, scaled, s);
  else mg_vcycle_generic<T>(G, transpose, guard, s);
}

// One multigrid solve with A + M_hat (transpose: its transpose) from level
// 0's b: vcycles V-cycles as a k-cycle iteration (the first may take the
// scaled right-hand side: the 2D and fused 3D paths).  Output: the level-0
// output array.
template <typename T>
static void mg_solve(Group* G, int transpose, int guard, int scaled, hipStream_t s) {
  const int k = G->H[0].vcycles;
  for (int j = 1; j <= k; ++j) {
    if (j > 1)
      hipLaunchKernelGGL(k_mg_kc_resid<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, transpose, j - 1, guard);
    mg_vcycle<T>(G, transpose, guard, j == 1 ? scaled : 0, s);
  }
  if (k > 1) hipLaunchKernelGGL(k_mg_kc_final<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, k, guard);
}

// Heat equation (Sec. 4.4): S_hat^-1 = (L + M_hat)^-T (O + Theta_y)
// (L + M_hat)^-1 with the block lower bidiagonal L + M_hat solved by block
// forward substitution, each diagonal block I/tau + A_h + M_hat_t by the
// multigrid solve of its time step, and the transpose by block backward
// substitution with the same per-step solves.
// Heat groups whose every step hierarchy fits one workgroup, one V-cycle per
// step: each substitution is one launch, one workgroup per instance.
static bool heat_one_launch(const Group* G) {
  for (int i = 0; i < G->count; ++i) {
    const Group& V = G->probs[i]->hview;
    if (!V.any_small || G->H[i].vcycles != 1) return false;
  }
  return true;
}

template <typename T>
static void heat_schur_inv(Group* G, int guard, hipStream_t s) {
  if (heat_one_launch(G)) {
    size_t lds = 0;
    for (int i = 0; i < G->count; ++i) lds = std::max(lds, G->probs[i]->hview.coarse_lds);
    const dim3 grid(1, 1, G->zc);
    hipLaunchKernelGGL(k_heat_sweep_p2<T>, grid, dim3(kCoarseBS), lds, s, G->D, 1, guard);
    hipLaunchKernelGGL(k_mg_scale_ty<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, guard);
    hipLaunchKernelGGL(k_heat_sweep_p2<T>, grid, dim3(kCoarseBS), lds, s, G->D, -1, guard);
    return;
  }
  // per-step launches (a group of one: the checks at Newton setup)
  ipmpde_problem* P = G->probs[0];
  Group* V = &P->hview;
  V->zc = 1;
  for (int t = 0; t < P->nt; ++t) {
    V->D = P->hs_d + t;
    if (t > 0) hipLaunchKernelGGL(k_heat_couple<T>, gz(V, V->max_n), dim3(kBS), 0, s, V->D, 1, G->outsel, guard);
    mg_solve<T>(V, 0, guard, 0, s);
  }
  hipLaunchKernelGGL(k_mg_scale_ty<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, guard);
  for (int t = P->nt - 1; t >= 0; --t) {
    V->D = P->hs_d + t;
    if (t < P->nt - 1) hipLaunchKernelGGL(k_heat_couple<T>, gz(V, V->max_n), dim3(kBS), 0, s, V->D, -1, G->outsel, guard);
    mg_solve<T>(V, 1, guard, 0, s);
  }
  V->D = P->hs_d;
}

// S_hat^-1 applied to every instance's lv[0].b (Sec. 4.2): solve with
// A + M_hat, scale by 1 + Theta_y, solve with (A + M_hat)^T.  The result is
// the level-0 output array (selected in the kernels with G->outsel).
template <typename T>
static void schur_inv(Group* G, int guard, hipStream_t s) {
  if (G->heat) {
    heat_schur_inv<T>(G, guard, s);
    return;
  }
  if ((G->dim == 2 && !G->q1) || G->p3) {  // Q1: the middle factor M + Theta_y is a stencil, applied below
    mg_solve<T>(G, 0, guard, 0, s);
    // instances whose whole hierarchy is in the coarse kernel never run a
    // descent kernel, so their scaled right-hand side is formed here; the
    // others form it inside their first descent kernel
    if (G->any_small) hipLaunchKernelGGL(k_mg_scale_ty_small<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, guard);
    mg_solve<T>(G, 1, guard, 1, s);
    return;
  }
  mg_solve<T>(G, 0, guard, 0, s);
  if (G->dim == 3 && G->q1)  // the 27-point Q1 mass summed from an LDS-staged block (mode 2)
    hipLaunchKernelGGL(k_mg_level3<T>, dim3((mg3_blocks(G->maxN[0]) + 7) & ~7, 1, G->zc), dim3(kBS), 0, s, G->D, 0,
                       G->outsel, 0, 0, 2, guard);
  else
    hipLaunchKernelGGL(k_mg_scale_ty<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, guard);
  mg_solve<T>(G, 1, guard, 0, s);
}

// ---------------------------------------------------------------------------
// Krylov solves (all instances; each stops on its own)

// Attainable accuracy: a relative residual below c eps |(|K||x| + |b|)| / |b|
// cannot be resolved by evaluating b - K x in FP64; the Krylov solves accept
// it as converged when the requested tolerance lies below that floor.
static double floor_factor() { return 16.0 * 2.220446049250313e-16; }

// Chebyshev steps for the Q1 mass block (the paper's 20).
static constexpr int kChebSteps = 20;

// z_y = (M + Theta_y)^-1 r_y for every Q1 instance by Chebyshev
// semi-iteration (Sec. 4.1) on the spectrum of the diagonally scaled Q1
// mass, [1/4, 9/4] in 2D and [1/8, 27/8] in 3D; operands as k_cheb_block
// takes them.
// Steps per launch of the blocked kernel (the tile's halo) and its tile width.
static constexpr int kChebBlockSteps = 5;
static constexpr int kChebTile = 16;
static_assert(kChebSteps % kChebBlockSteps == 0, "whole launches of Chebyshev steps");

static void cheb_apply(Group* G, const double* x, double* y, int j, int mpar, int guard, hipStream_t s) {
  ChebCoef cf;
  const double lo = G->dim == 3 ? 1.0 / 8.0 : 1.0 / 4.0, hi = G->dim == 3 ? 27.0 / 8.0 : 9.0 / 4.0;
  cf.theta = 0.5 * (hi + lo);
  cf.delta = 0.5 * (hi - lo);
  cf.rho[0] = cf.delta / cf.theta;
  for (int k = 1; k < kChebSteps; ++k) cf.rho[k] = 1.0 / (2.0 * cf.theta / cf.delta - cf.rho[k - 1]);
  if (G->dim == 3) {
    const int nb = (cheb3_blocks(G->maxN[0]) + 7) & ~7;  // a multiple of 8 for the XCD slabs
    for (int k = 0; k < kChebSteps; ++k)
      hipLaunchKernelGGL(k_cheb_step3, dim3(nb, 1, G->zc), dim3(kBS), 0, s, G->D, x, y, j, mpar, k, cf, guard);
    return;
  }
  const int nt = div_up(G->maxN[0], kChebTile);
  for (int L = 0; L * kChebBlockSteps < kChebSteps; ++L)
    hipLaunchKernelGGL((k_cheb_block<kChebTile, kChebBlockSteps>), dim3(nt, nt, G->zc), dim3(kBS), 0, s, G->D, x, y,
                       j, mpar, L * kChebBlockSteps, L, cf, guard);
}

template <typename T>
static void minres_iteration(Group* G, int par, int maxit, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_minres_k1, gz(G, G->max_n), dim3(kBS), 0, s, G->D, par, 0);
  hipLaunchKernelGGL(k_minres_k2<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, par, 0);
  if (G->q1) cheb_apply(G, nullptr, nullptr, 0, par, 1, s);
  schur_inv<T>(G, 1, s);
  hipLaunchKernelGGL(k_minres_k4<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, 1 - par, 1, tol, maxit, G->outsel);
}

static bool any_running(const Group* G) {
  for (int i = 0; i < G->count; ++i)
    if (G->H[i].active && G->ctrl_h[i].want_restart && !G->ctrl_h[i].stop) return true;
  return false;
}
static bool any_restart(const Group* G) {
  for (int i = 0; i < G->count; ++i)
    if (G->H[i].active && G->ctrl_h[i].want_restart) return true;
  return false;
}
// After the last restart cycle a solve whose true residual still misses the
// tolerance is a Krylov failure (counted in the statistics, IPMPDE_EKRYLOV
// from the single-step entry points), not a success.
static void mark_unfinished(Group* G) {
  for (int i = 0; i < G->count; ++i)
    if (G->H[i].active && G->ctrl_h[i].want_restart) G->ctrl_h[i].failed = 1;
}

// The graph cache key of a launch sequence for this group and these options.
static GraphKey graph_key(const Group* G, const ipmpde_options& o, int fg, int j0) {
  const int flags = (G->p2 ? 1 : 0) | (G->gen ? 2 : 0) | (G->any_small ? 4 : 0) | (G->outsel << 3) |
                    (G->q1 ? 16 : 0) | (G->heat ? 32 : 0) | (G->tile << 6) | (G->cd ? 256 : 0) |
                    (G->f3 ? 1024 : 0);
  GraphKey key{G->fp32 ? 1 : 0, o.nu_pre, o.nu_post, o.chunk, o.krylov_maxit, G->zc, G->max_n, G->max_nlev,
               G->max_cl, flags, G->coarse_lds, G->H[0].omega, o.krylov_tol};
  key.fg = fg;
  key.j0 = j0;
  key.vcycles = o.vcycles;
  return key;
}

// Launch the sequence `body(stream)` through the group's graph cache: the
// first use of a key captures it on the group's capture stream (created on
// the first capture: every stream holds one of the process's few hardware
// queues) and instantiates it; later uses launch the instantiated graph on s.
template <typename F>
static int launch_cached(Group* G, const GraphKey& key, hipStream_t s, F&& body) {
  auto it = G->graphs.find(key);
  if (it == G->graphs.end()) {
    if (G->graphs.size() >= kMaxGraphs) {
      for (auto& kv : G->graphs) (void)hipGraphExecDestroy(kv.second);
      G->graphs.clear();
    }
    hipGraph_t g;
    if (!G->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&G->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(G->cap_stream, hipStreamCaptureModeThreadLocal));
    body(G->cap_stream);
    HIP_TRY(hipStreamEndCapture(G->cap_stream, &g));
    hipGraphExec_t ge;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(IPMPDE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = G->graphs.emplace(key, ge).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, s));
  return IPMPDE_OK;
}

template <typename T>
static int run_minres_chunk(Group* G, const ipmpde_options& o, hipStream_t s) {
  auto body = [&](hipStream_t st) {
    for (int t = 0; t < o.chunk; ++t) minres_iteration<T>(G, (1 + t) & 1, o.krylov_maxit, o.krylov_tol, st);
  };
  if (!o.use_graphs) {
    body(s);
    return IPMPDE_OK;
  }
  return launch_cached(G, graph_key(G, o, 0, 0), s, body);
}

// MINRES on every active instance: a cycle from the right-hand side, then
// (for instances whose true residual missed the tolerance) cycles from the
// true residual.  Per-instance results stay in the group's ctrl array.
static constexpr int kMinresCycles = 16;

template <typename T>
static int minres_group(Group* G, const ipmpde_options& o, hipStream_t s) {
  const double tol = o.krylov_tol;
  hipLaunchKernelGGL(k_krylov_begin, gz(G, 4L * G->max_n), dim3(kBS), 0, s, G->D);
  if (G->persist) {
    // the small 2D Poisson instances run their whole solve in one workgroup
    // each; the loop below serves the others (and skips these: no pending cycle)
    hipLaunchKernelGGL(k_minres_small<T>, dim3(1, 1, G->zc), dim3(kCoarseBS), G->coarse_lds, s, G->D, tol,
                       floor_factor(), o.krylov_maxit, kMinresCycles);
    HIP_TRY(hipGetLastError());
    TRY(read_ctrl(G, s));
    if (!any_restart(G)) return IPMPDE_OK;
  }
  for (int cycle = 0; cycle < kMinresCycles; ++cycle) {
    hipLaunchKernelGGL(k_minres_init<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, cycle == 0 ? 0 : 1);
    if (G->q1) cheb_apply(G, nullptr, nullptr, 0, 0, 2, s);
    schur_inv<T>(G, 2, s);
    hipLaunchKernelGGL(k_minres_k4<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, 1, 0, tol, o.krylov_maxit, G->outsel);
    HIP_TRY(hipGetLastError());
    TRY(read_ctrl(G, s));
    int chunks = 0;
    while (any_running(G) && chunks++ < o.krylov_maxit / o.chunk + 2) {
      TRY(run_minres_chunk<T>(G, o, s));
      TRY(read_ctrl(G, s));
    }
    hipLaunchKernelGGL(k_minres_flush, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_true_residual, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_krylov_mark, dim3(1, 1, G->zc), dim3(64), 0, s, G->D, tol, floor_factor(), o.krylov_maxit, 0);
    HIP_TRY(hipGetLastError());
    TRY(read_ctrl(G, s));
    if (!any_restart(G)) return IPMPDE_OK;
  }
  mark_unfinished(G);
  return IPMPDE_OK;
}

static void mg_select(Group* G, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_select, dim3(1, 1, G->zc), dim3(64), 0, s, G->D, slot);
}

// z = P^-1 r for every instance (pt: IPMPDE_PD, IPMPDE_PT or IPMPDE_PPI);
// explicit operands, or the FGMRES slots r = V_j, z = Z_j when null.
template <typename T>
static void precond_apply(Group* G, int pt, const double* x, double* y, int j, int guard, hipStream_t s) {
  if (pt == IPMPDE_PPI) {
    // Sec. 4.3: v2 (z block), v1 = L^-1 (Mbar v2 + r_p), then
    // v3 = (L + M_r)^-1 L (L^T + M_l)^-1 ((O + Theta_y) v1 - r_y)
    hipLaunchKernelGGL(k_ppi_a<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, x, y, j, guard);
    if (G->q1)
      hipLaunchKernelGGL(k_ppi_a_q1<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, x, (const double*)y, j, guard);
    mg_select(G, 2, s);
    mg_solve<T>(G, 0, guard, 0, s);
    hipLaunchKernelGGL(k_ppi_b<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, x, y, j, G->outsel, guard);
    mg_select(G, 1, s);
    mg_solve<T>(G, 1, guard, 0, s);
    hipLaunchKernelGGL(k_ppi_c<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, G->outsel, guard);
    mg_select(G, 0, s);
    mg_solve<T>(G, 0, guard, 0, s);
    hipLaunchKernelGGL(k_store_p<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, y, j, G->outsel, guard);
    return;
  }
  hipLaunchKernelGGL(k_precond_diag<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, x, y, j, pt, guard);
  if (G->q1) cheb_apply(G, x, y, j, -1, guard, s);
  if (pt) hipLaunchKernelGGL(k_pt_rhs<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, x, (const double*)y, j, guard);
  schur_inv<T>(G, guard, s);
  hipLaunchKernelGGL(k_store_p<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, y, j, G->outsel, guard);
}

static int fg_multidot_blocks(long n4) { return std::min(nblk(n4), 256); }

template <typename T>
static void fgmres_step(Group* G, int pt, int j, double tol, int maxit, hipStream_t s) {
  const long n4 = 4L * G->max_n;
  precond_apply<T>(G, pt, nullptr, nullptr, j, 1, s);
  hipLaunchKernelGGL(k_fg_matvec, gz(G, G->max_n), dim3(kBS), 0, s, G->D, j);
  const int nbm = fg_multidot_blocks(n4);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_fg_multidot, dim3(nbm, j + 1, G->zc), dim3(kBS), 0, s, G->D, j);
    hipLaunchKernelGGL(k_fg_multidot_final, dim3(1, 1, G->zc), dim3(kBS), 0, s, G->D, j + 1, nbm, pass == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_fg_orth, gz(G, n4), dim3(kBS), 0, s, G->D, j);
  }
  hipLaunchKernelGGL(k_fg_norm_givens, dim3(nbm, 1, G->zc), dim3(kBS), 0, s, G->D, j, tol, maxit);
  hipLaunchKernelGGL(k_fg_normalize, gz(G, n4), dim3(kBS), 0, s, G->D, j);
}

template <typename T>
static int fgmres_group(Group* G, const ipmpde_options& o, hipStream_t s) {
  const long n4 = 4L * G->max_n;
  const int pt = o.precond;  // IPMPDE_PD, IPMPDE_PT or IPMPDE_PPI
  const int nbm = fg_multidot_blocks(n4);
  // Arnoldi steps between host checks: captured in one graph per range
  // (the kernels of a stopped instance return at once)
  const int step = o.use_graphs ? o.chunk : 4;
  hipLaunchKernelGGL(k_krylov_begin, gz(G, n4), dim3(kBS), 0, s, G->D);
  for (int cycle = 0; cycle < 1000; ++cycle) {
    const int src = cycle == 0 ? 0 : 1;
    hipLaunchKernelGGL(k_fg_start_norm, dim3(nbm, 1, G->zc), dim3(kBS), 0, s, G->D, src);
    hipLaunchKernelGGL(k_fg_start_scale, gz(G, n4), dim3(kBS), 0, s, G->D, src);
    TRY(read_ctrl(G, s));
    for (int j0 = 0; j0 < o.restart && any_running(G); j0 += step) {
      const int j1 = std::min(j0 + step, o.restart);
      auto body = [&](hipStream_t st) {
        for (int j = j0; j < j1; ++j) fgmres_step<T>(G, pt, j, o.krylov_tol, o.krylov_maxit, st);
      };
      if (o.use_graphs) {
        TRY(launch_cached(G, graph_key(G, o, 1 + pt, j0 * 64 + j1), s, body));
      } else {
        body(s);
      }
      HIP_TRY(hipGetLastError());
      TRY(read_ctrl(G, s));
    }
    hipLaunchKernelGGL(k_fg_solve_small, dim3(1, 1, G->zc), dim3(64), 0, s, G->D);
    hipLaunchKernelGGL(k_fg_update_x, gz(G, n4), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_true_residual, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_krylov_mark, dim3(1, 1, G->zc), dim3(64), 0, s, G->D, o.krylov_tol, floor_factor(),
                       o.krylov_maxit, 1);
    HIP_TRY(hipGetLastError());
    TRY(read_ctrl(G, s));
    if (!any_restart(G)) return IPMPDE_OK;
  }
  mark_unfinished(G);
  return IPMPDE_OK;
}

static int krylov_group(Group* G, const ipmpde_options& o, hipStream_t s) {
  if (o.krylov == IPMPDE_MINRES) return G->fp32 ? minres_group<float>(G, o, s) : minres_group<double>(G, o, s);
  return G->fp32 ? fgmres_group<float>(G, o, s) : fgmres_group<double>(G, o, s);
}

// per-instance Krylov outcome after krylov_group
static int krylov_status(const Group* G, int i) {
  const KrylovCtrl& C = G->ctrl_h[i];
  if (!(C.relres == C.relres)) return IPMPDE_EBREAKDOWN;
  return C.failed ? IPMPDE_EKRYLOV : IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// Newton setup and IPM steps (all instances)

// The coarse LDS images of the current reaction-term slot: 2D Poisson (with
// the inverse of its 7 x 7 level's operator) and convection-diffusion.
template <typename T>
static void coarse_image(Group* G, hipStream_t s) {
  if (G->p2) {
    hipLaunchKernelGGL(k_coarse_pack<T>, gz(G, G->max_cpack), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_coarse_inv7<T>, dim3(1, 1, G->zc), dim3(kBS), 0, s, G->D);
  }
  if (G->cd) {
    hipLaunchKernelGGL(k_coarse_pack_cd<T>, gz(G, G->max_cpack), dim3(kBS), 0, s, G->D);
    hipLaunchKernelGGL(k_coarse_inv7_cd<T>, dim3(1, 1, G->zc), dim3(kBS), 0, s, G->D);
  }
}

// P_Pi's extra operators: M_l (slot 1, written at level 0 by the Newton setup)
// restricted to every level and its coarse image; the coarse image of the
// zero slot (L alone); back to slot 0.
template <typename T>
static void ppi_setup(Group* G, hipStream_t s) {
  mg_select(G, 1, s);
  for (int l = 0; l + 1 < G->max_nlev; ++l)
    hipLaunchKernelGGL(k_restrict_diag<T>, gz(G, G->maxn[l + 1]), dim3(kBS), 0, s, G->D, l);
  if (G->p2 || G->cd) coarse_image<T>(G, s);
  mg_select(G, 2, s);
  if (G->p2 || G->cd) coarse_image<T>(G, s);
  mg_select(G, 0, s);
}

// Heat equation: the reaction term of every time step (written at level 0
// by the Newton setup) restricted to all levels and each step's coarse
// image, all steps in one launch per level.
template <typename T>
static void heat_setup(Group* G, hipStream_t s) {
  hipLaunchKernelGGL(k_newton_setup<T>, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  for (int i = 0; i < G->count; ++i) {
    ipmpde_problem* P = G->probs[i];
    Group* V = &P->hview;
    V->D = P->hs_d;
    V->zc = P->nt;
    for (int l = 0; l + 1 < V->max_nlev; ++l)
      hipLaunchKernelGGL(k_restrict_diag<T>, gz(V, V->maxn[l + 1]), dim3(kBS), 0, s, V->D, l);
    hipLaunchKernelGGL(k_coarse_pack<T>, gz(V, V->max_cpack), dim3(kBS), 0, s, V->D);
    hipLaunchKernelGGL(k_coarse_inv7<T>, dim3(1, 1, V->zc), dim3(kBS), 0, s, V->D);
    V->zc = 1;
  }
}

static int newton_setup_group(Group* G, const ipmpde_options& o, hipStream_t s) {
  if (G->heat && o.precond == IPMPDE_PPI)
    return fail(IPMPDE_EINVAL, "P_Pi is not available for the heat equation");
  if (G->q1 && o.precond != IPMPDE_PPI)
    for (int i = 0; i < G->count; ++i)
      if (G->probs[i]->eobs)
        return fail(IPMPDE_EINVAL, "Q1 problems observed on part of the domain take P_Pi");
  for (int i = 0; i < G->count; ++i) {
    const ipmpde_problem* P = G->probs[i];
    if (o.precond != IPMPDE_PPI && P->obs_zero && !P->has_y)
      return fail(IPMPDE_EINVAL, "unobserved nodes without state bounds make the (1,1) block singular: use P_Pi");
  }
  TRY(group_select(G, o));
  if (G->heat && G->count > 1 && !heat_one_launch(G))
    return fail(IPMPDE_EINVAL, "a batch of heat-equation problems needs every time step's hierarchy in one "
                               "workgroup (N <= 63 with FP32 or N <= 31 with FP64 V-cycles) and vcycles = 1");
  TRY(group_sync(G, s));
  if (G->heat) {
    if (G->fp32) heat_setup<float>(G, s);
    else heat_setup<double>(G, s);
  } else if (G->fp32) {
    hipLaunchKernelGGL(k_newton_setup<float>, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    for (int l = 0; l + 1 < G->max_nlev; ++l)
      hipLaunchKernelGGL(k_restrict_diag<float>, gz(G, G->maxn[l + 1]), dim3(kBS), 0, s, G->D, l);
    if (G->p2 || G->cd) coarse_image<float>(G, s);
    if (o.precond == IPMPDE_PPI) ppi_setup<float>(G, s);
  } else {
    hipLaunchKernelGGL(k_newton_setup<double>, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
    for (int l = 0; l + 1 < G->max_nlev; ++l)
      hipLaunchKernelGGL(k_restrict_diag<double>, gz(G, G->maxn[l + 1]), dim3(kBS), 0, s, G->D, l);
    if (G->p2 || G->cd) coarse_image<double>(G, s);
    if (o.precond == IPMPDE_PPI) ppi_setup<double>(G, s);
  }
  HIP_TRY(hipGetLastError());
  for (int i = 0; i < G->count; ++i) {
    G->probs[i]->setup_done = true;
    G->probs[i]->setup_fp32 = G->fp32 ? 1 : 0;
    G->probs[i]->setup_group = G;
  }
  return IPMPDE_OK;
}

static int group_step(Group* G, const ipmpde_options& o, hipStream_t s) {
  TRY(newton_setup_group(G, o, s));
  TRY(krylov_group(G, o, s));
  hipLaunchKernelGGL(k_step_lengths, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  hipLaunchKernelGGL(k_update, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  HIP_TRY(hipGetLastError());
  TRY(read_stat(G, s));
  return IPMPDE_OK;
}

// Measures of every active instance -> stat[0..2]; with `mean`, also the
// mean complementarity product -> stat[5].
static int group_measures(Group* G, hipStream_t s, bool mean = false) {
  TRY(group_sync(G, s));
  hipLaunchKernelGGL(k_measures, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  if (mean) hipLaunchKernelGGL(k_compl_mean, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  HIP_TRY(hipGetLastError());
  TRY(read_stat(G, s));
  return IPMPDE_OK;
}

// Starting point of every instance with its own mu0.
static int group_reset(Group* G, const std::vector<ipmpde_options>& po, hipStream_t s) {
  for (int i = 0; i < G->count; ++i) {
    G->H[i].active = 1;
    G->H[i].mu = po[i].mu0;
    G->H[i].alpha0 = po[i].alpha0;
    G->probs[i]->mu = po[i].mu0;
    G->probs[i]->need_init = false;
  }
  TRY(group_sync(G, s));
  hipLaunchKernelGGL(k_init_state, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

// Per-instance bookkeeping of Algorithm A.1, shared by the lockstep batch
// solve and the serving engine so that both take identical decisions.

static void ipm_begin(ipmpde_problem* P) {
  std::memset(&P->stats, 0, sizeof(P->stats));
  P->stats.status = IPMPDE_ENOTCONVERGED;
}

// After the measures of iterate k (slot i of G): record them and return the
// final status, or -1 to go on (mu is then reduced for the next step).
static int ipm_check(Group* G, int i, int k, const ipmpde_options& oi) {
  ipmpde_problem* P = G->probs[i];
  ipmpde_stats& st = P->stats;
  const double xp = G->stat_h[16 * i], xd = G->stat_h[16 * i + 1], xc = G->stat_h[16 * i + 2];
  const double w = P->rep;
  if (k < IPMPDE_MAX_HIST) {
    st.hist_mu[k] = w * P->mu;
    st.hist_xi_p[k] = w * xp;
    st.hist_xi_d[k] = w * xd;
    st.hist_xi_c[k] = w * xc;
    st.hist_len = k + 1;
  }
  st.nli = k;
  st.xi_p = w * xp; st.xi_d = w * xd; st.xi_c = w * xc; st.mu = w * P->mu;
  int finish = -1;
  if (!(xp == xp && xd == xd && xc == xc)) finish = IPMPDE_EBREAKDOWN;
  else if (oi.fixed_nli > 0 ? k >= oi.fixed_nli : (xp <= oi.eps_p && xd <= oi.eps_d && xc <= oi.eps_c))
    finish = IPMPDE_OK;
  else if (k >= oi.ipm_maxit) finish = IPMPDE_ENOTCONVERGED;
  if (finish >= 0) {
    st.status = finish;
    G->H[i].active = 0;
  } else {
    P->mu = oi.sigma * (oi.mu_rule == IPMPDE_MU_CENTRAL ? G->stat_h[16 * i + 5] : P->mu);
    G->H[i].mu = P->mu;
  }
  return finish;
}

// After Newton step k of slot i: record it; returns the final status on a
// breakdown (NaN or collapsed step), else -1.
static int ipm_after_step(Group* G, int i, int k) {
  ipmpde_stats& st = G->probs[i]->stats;
  const double aP = G->stat_h[16 * i + 3], aD = G->stat_h[16 * i + 4];
  const KrylovCtrl& C = G->ctrl_h[i];
  if (k < IPMPDE_MAX_HIST) {
    st.hist_krylov[k] = C.its_total;
    st.hist_krylov_relres[k] = C.relres;
    st.hist_alpha_p[k] = aP;
    st.hist_alpha_d[k] = aD;
  }
  st.krylov_its += C.its_total;
  const int kst = krylov_status(G, i);
  if (kst == IPMPDE_EKRYLOV) st.krylov_fail += 1;
  if (kst == IPMPDE_EBREAKDOWN || !(aP > 1e-10 && aD > 1e-10)) {
    st.status = IPMPDE_EBREAKDOWN;
    G->H[i].active = 0;
    return IPMPDE_EBREAKDOWN;
  }
  return -1;
}

// Algorithm A.1 on every instance of the group, in lockstep; each instance
// leaves the loop (and every later launch) when its own test is met.  po:
// per-instance options (IPM fields may differ; Krylov/multigrid fields must
// match).  Per-instance status goes to the problems' stats.
static int solve_group(Group* G, const std::vector<ipmpde_options>& po_in, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  std::vector<ipmpde_options> po(po_in.size());
  for (int i = 0; i < G->count; ++i) TRY(unit_form(G->probs[i], po_in[i], &po[i]));
  const ipmpde_options& o = po[0];
  for (int i = 0; i < G->count; ++i) ipm_begin(G->probs[i]);
  TRY(group_select(G, o));
  TRY(group_reset(G, po, s));
  std::vector<int> done(G->count, 0);
  bool mean = false;
  for (const ipmpde_options& oi : po) mean = mean || oi.mu_rule == IPMPDE_MU_CENTRAL;
  for (int k = 0;; ++k) {
    TRY(group_measures(G, s, mean));
    int alive = 0;
    for (int i = 0; i < G->count; ++i) {
      if (done[i]) continue;
      if (ipm_check(G, i, k, po[i]) >= 0) done[i] = 1;
      else ++alive;
    }
    if (!alive) break;
    TRY(group_step(G, o, s));
    for (int i = 0; i < G->count; ++i)
      if (!done[i] && ipm_after_step(G, i, k) >= 0) done[i] = 1;
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < G->count; ++i) G->probs[i]->stats.solve_ms = ms;
  return IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// creation

static int validate_array(const double* a, size_t n, const char* name) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return fail(IPMPDE_EINVAL, std::string(name) + " contains NaN or Inf");
  return IPMPDE_OK;
}

// f_hat = f - A_IB g: boundary neighbours' coefficients times g (host, once).
static void fold_boundary(int dim, int N, int pde, double eps, const double* g, std::vector<double>& fhat) {
  const double h = 1.0 / (N + 1);
  const int P = N + 2;
  auto gidx = [&](int a, int b, int c) { return (size_t)a + (size_t)P * ((size_t)b + (size_t)P * c); };
  const size_t n = pow_dim(N, dim);
  for (size_t idx = 0; idx < n; ++idx) {
    int i1 = idx % N, i2 = (idx / N) % N, i3 = dim == 3 ? (int)(idx / ((size_t)N * N)) : 0;
    int c[3] = {i1 + 1, i2 + 1, dim == 3 ? i3 + 1 : 0};
    double acc = 0.0;
    for (int ax = 0; ax < dim; ++ax) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int nb[3] = {c[0], c[1], c[2]};
        nb[ax] += sgn;
        if (nb[ax] >= 1 && nb[ax] <= N) continue;  // interior neighbour
        double coef;
        if (pde == IPMPDE_POISSON) {
          coef = -1.0 / (h * h);
        } else {
          const double x1 = c[0] * h, x2 = c[1] * h;
          const double w1 = 2.0 * x2 * (1.0 - x1 * x1), w2 = -2.0 * x1 * (1.0 - x2 * x2);
          const double wa = ax == 0 ? w1 : w2;
          coef = -eps / (h * h) + (sgn < 0 ? -std::max(wa, 0.0) / h : std::min(wa, 0.0) / h);
        }
        const double gv = dim == 2 ? g[gidx(nb[0], nb[1], 0)] : g[gidx(nb[0], nb[1], nb[2])];
        acc += coef * gv;
      }
    }
    fhat[idx] -= acc;
  }
}

// Q1 (divided by h^dim): f_hat = M f - L_IB g with the interior mass stencil
// applied to f and the stiffness stencil's boundary neighbours applied to g.
// By the number k of nonzero offsets of a neighbour: 2D mass (16, 4, 1) / 36
// and stiffness -1 / (3 h^2) for every neighbour; 3D mass (64, 16, 4, 1) / 216
// and stiffness (0, -1/6, -1/12) / h^2 for k = 1, 2, 3.
static void fold_q1(int dim, int N, const double* f, const double* g, std::vector<double>& fhat) {
  const double h = 1.0 / (N + 1), ih2 = 1.0 / (h * h);
  const size_t P = N + 2;
  const int N3 = dim == 3 ? N : 1, r3 = dim == 3 ? 1 : 0;
  for (int i3 = 0; i3 < N3; ++i3)
    for (int i2 = 0; i2 < N; ++i2)
      for (int i1 = 0; i1 < N; ++i1) {
        double acc = 0.0;
        for (int c = -r3; c <= r3; ++c)
          for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
              const int j1 = i1 + a, j2 = i2 + b, j3 = i3 + c;
              const int k = (a != 0) + (b != 0) + (c != 0);
              const bool inside = j1 >= 0 && j1 < N && j2 >= 0 && j2 < N && j3 >= 0 && j3 < N3;
              double m, l;  // mass weight, minus the stiffness weight
              if (dim == 2) {
                m = (k == 0 ? 16.0 : k == 1 ? 4.0 : 1.0) / 36.0;
                l = ih2 / 3.0;
              } else {
                m = (k == 0 ? 64.0 : k == 1 ? 16.0 : k == 2 ? 4.0 : 1.0) / 216.0;
                l = k == 2 ? ih2 / 6.0 : (k == 3 ? ih2 / 12.0 : 0.0);
              }
              if (inside && f) acc += m * f[j1 + (size_t)N * (j2 + (size_t)N * j3)];
              if (!inside && g) acc += l * g[(j1 + 1) + P * ((j2 + 1) + P * (size_t)(dim == 3 ? j3 + 1 : 0))];
            }
        fhat[i1 + (size_t)N * (i2 + (size_t)N * i3)] = acc;
      }
}

extern "C" const char* ipmpde_version(void) { return "libipmpde 0.2 (gfx950)"; }
extern "C" const char* ipmpde_last_error(void) { return g_err.c_str(); }

extern "C" int ipmpde_set_allocator(ipmpde_alloc_fn a, ipmpde_free_fn f, void* ctx) {
  if ((a == nullptr) != (f == nullptr)) return fail(IPMPDE_EINVAL, "allocator and free must both be set or both NULL");
  g_alloc = a;
  g_free = f;
  g_alloc_ctx = ctx;
  return IPMPDE_OK;
}

// Device bytes a problem holds while it is solved: its data, iterates and
// barrier diagonals for the handle's lifetime, plus the workspace of the
// Newton solves (Krylov vectors, multigrid levels of the chosen precision,
// FGMRES basis, reduction partials).  Mirrors the allocations one by one.
extern "C" size_t ipmpde_footprint_bytes(const ipmpde_grid* grid, const ipmpde_pde* pde, int has_y,
                                         const ipmpde_options* opts) {
  if (!grid || !pde || (grid->dim != 2 && grid->dim != 3) || !is_pow2m1(grid->n)) return 0;
  ipmpde_options o;
  if (opts) o = *opts;
  else ipmpde_default_options(&o);
  const size_t n = pow_dim(grid->n, grid->dim), n4 = 4 * n;
  auto A = [](size_t b) { return std::max<size_t>(b, 256); };
  const size_t arrays = 16 + (has_y ? 4 : 0);  // bounds, y_d, f_hat, iterates, multipliers, diagonals
  size_t bytes = arrays * A(n * 8) + A(kTicketStride * (kTicketGroups + 1) * sizeof(unsigned));
  bytes += kKrylovVecs * A(n4 * 8) + A((size_t)partials_words(nblk((long)n)) * 8);
  const size_t el = o.mg_precision == IPMPDE_FP32 ? 4 : 8;
  for (int N = grid->n;; N = (N - 1) / 2) {  // x, x2, b and the reaction-term slots
    bytes += 3 * A(pow_dim(N, grid->dim) * el) + A(kReactionSlots * pow_dim(N, grid->dim) * el);
    if (N <= 1) break;
  }
  bytes += 3 * A(n * el);  // k-cycle level-0 arrays
  bytes += A(kMaxLev * sizeof(Level));
  if (grid->dim == 2 && (pde->kind == IPMPDE_POISSON || pde->kind == IPMPDE_POISSON_Q1 ||
                         pde->kind == IPMPDE_CONVDIFF)) {  // coarse LDS images, one per reaction-term slot
    const int kind = pde->kind == IPMPDE_CONVDIFF ? kCoarseCD : kCoarseP2;
    Level lv[kMaxLev];
    int nlev = 0;
    for (int N = grid->n;; N = (N - 1) / 2) {
      lv[nlev].N = N;
      lv[nlev].n = N * N;
      ++nlev;
      if (N <= 1) break;
    }
    const int cl = pick_coarse(lv, nlev, el, 2, kind);
    size_t elems = coarse_p2_tail(lv, nlev, kind);
    for (int l = cl; l < nlev; ++l) elems += coarse_level_elems(lv[l], kind);
    bytes += A((size_t)kReactionSlots * cpack_stride((int)elems) * el);
  }
  if (o.krylov == IPMPDE_FGMRES) bytes += A((size_t)(o.restart + 1) * n4 * 8) + A((size_t)o.restart * n4 * 8);
  return bytes;
}

static void problem_free(ipmpde_problem* P) {
  if (P->self) group_release(P->self);
  P->self = nullptr;
  if (P->hs_h) (void)hipHostFree(P->hs_h);
  P->hs_h = nullptr;
  release_work(P);
  P->mem.release();
}

// Shared by the steady and the heat-equation constructors (kind, grid and
// time steps already validated): copies the data, folds boundary data (and
// for the heat equation the initial state) into f_hat.
static int problem_create_impl(int dim, int N, int kind, double eps, int nt, double tau, double alpha, double beta,
                               const double* u_a, const double* u_b, const double* y_a, const double* y_b,
                               const double* y_d, const double* f, const double* g, const double* y0,
                               ipmpde_problem** out) {
  if (!(alpha > 0 && std::isfinite(alpha))) return fail(IPMPDE_EINVAL, "alpha must be positive");
  if (!(beta >= 0 && std::isfinite(beta))) return fail(IPMPDE_EINVAL, "beta must be non-negative");
  if (!u_a || !u_b || !y_d) return fail(IPMPDE_EINVAL, "u_a, u_b and y_d are required");
  if ((y_a == nullptr) != (y_b == nullptr)) return fail(IPMPDE_EINVAL, "y_a and y_b must both be given or both NULL");
  const bool heat = kind == IPMPDE_HEAT;
  const size_t n = pow_dim(N, dim) * (size_t)nt;
  TRY(validate_array(u_a, n, "u_a"));
  TRY(validate_array(u_b, n, "u_b"));
  TRY(validate_array(y_d, n, "y_d"));
  for (size_t i = 0; i < n; ++i)
    if (!(u_a[i] < 0.0 && u_b[i] > 0.0)) return fail(IPMPDE_EINVAL, "bounds must satisfy u_a < 0 < u_b");
  if (y_a) {
    TRY(validate_array(y_a, n, "y_a"));
    TRY(validate_array(y_b, n, "y_b"));
    for (size_t i = 0; i < n; ++i)
      if (!(y_a[i] < y_b[i])) return fail(IPMPDE_EINVAL, "state bounds must satisfy y_a < y_b");
  }
  if (f) TRY(validate_array(f, n, "f"));
  if (g) TRY(validate_array(g, pow_dim(N + 2, dim), "g"));
  if (y0) TRY(validate_array(y0, pow_dim(N, dim), "y0"));

  std::vector<double> fhat(n, 0.0);
  if (f) std::copy(f, f + n, fhat.begin());
  if (heat) {
    // every time step sees the same boundary data; y0 / tau enters the first step
    const size_t n2 = pow_dim(N, dim);
    std::vector<double> step(n2, 0.0);
    if (g) fold_boundary(dim, N, IPMPDE_POISSON, 1.0, g, step);
    for (int t = 0; t < nt; ++t)
      for (size_t i = 0; i < n2; ++i) fhat[(size_t)t * n2 + i] += step[i];
    if (y0)
      for (size_t i = 0; i < n2; ++i) fhat[i] += y0[i] / tau;
  } else if (kind == IPMPDE_POISSON_Q1) {
    fold_q1(dim, N, f, g, fhat);
  } else if (g) {
    fold_boundary(dim, N, kind, kind == IPMPDE_POISSON ? 1.0 : eps, g, fhat);
  }

  ipmpde_problem* P = new ipmpde_problem();
  P->dim = dim; P->N = N; P->n = (int)n; P->pde = kind;
  P->eps = kind == IPMPDE_CONVDIFF ? eps : 1.0;
  P->nt = nt; P->tau = tau;
  P->alpha = alpha; P->beta = beta; P->has_y = y_a != nullptr;
  P->nlev = level_count(N);
  std::memset(&P->stats, 0, sizeof(P->stats));
  Inst& I = P->I;
  std::memset(&I, 0, sizeof(I));
  I.dim = dim; I.N = N; I.n = (int)n; I.pde = P->pde; I.has_y = P->has_y ? 1 : 0;
  I.h = 1.0 / (N + 1); I.eps = P->eps; I.alpha = alpha; I.beta = beta;
  I.nt = nt; I.tau = tau;
  I.active = 1;
  I.mu = 1.0;
  I.alpha0 = 0.995;
  auto cleanup = [&](int rc) { problem_free(P); delete P; return rc; };
  int rc = IPMPDE_OK;
  double* dev[32];
  int nd = 0;
  AllocList& M = P->mem;
  auto A = [&](double** p) -> int { int r = M.alloc_t(p, n); if (r == IPMPDE_OK) dev[nd++] = *p; return r; };
  double *ua, *ub, *ya = nullptr, *yb = nullptr, *yd, *fh;
  if ((rc = A(&ua)) || (rc = A(&ub)) || (rc = A(&yd)) || (rc = A(&fh))) return cleanup(rc);
  if (P->has_y && ((rc = A(&ya)) || (rc = A(&yb)))) return cleanup(rc);
  if ((rc = A(&I.y)) || (rc = A(&I.w)) || (rc = A(&I.v)) || (rc = A(&I.p)) || (rc = A(&I.lwa)) ||
      (rc = A(&I.lwb)) || (rc = A(&I.lva)) || (rc = A(&I.lvb)) || (rc = A(&I.ty)) || (rc = A(&I.tw)) ||
      (rc = A(&I.tv)) || (rc = A(&I.mh)))
    return cleanup(rc);
  if (P->has_y && ((rc = A(&I.lya)) || (rc = A(&I.lyb)))) return cleanup(rc);
  I.ua = ua; I.ub = ub; I.ya = ya; I.yb = yb; I.yd = yd; I.fhat = fh;
  if ((rc = M.alloc_t(&I.counter, kTicketStride * (kTicketGroups + 1)))) return cleanup(rc);
  auto hip_fail = [&](hipError_t e, const char* what) {
    return cleanup(fail(IPMPDE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)));
  };
  hipError_t e;
  if ((e = hipMemset(I.counter, 0, kTicketStride * (kTicketGroups + 1) * sizeof(unsigned))) != hipSuccess)
    return hip_fail(e, "hipMemset");
  for (int k = 0; k < nd; ++k)
    if ((e = hipMemset(dev[k], 0, n * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMemset");
  if ((e = hipMemcpy(ua, u_a, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(ub, u_b, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(yd, y_d, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(fh, fhat.data(), n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if (P->has_y) {
    if ((e = hipMemcpy(ya, y_a, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(yb, y_b, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  if (heat) {
    if ((rc = M.alloc_t(&P->hs_d, (size_t)nt))) return cleanup(rc);
    if ((e = hipHostMalloc((void**)&P->hs_h, sizeof(Inst) * nt, hipHostMallocDefault)) != hipSuccess)
      return hip_fail(e, "hipHostMalloc");
    std::memset((void*)P->hs_h, 0, sizeof(Inst) * nt);
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "init");
  *out = P;
  return IPMPDE_OK;
}

extern "C" int ipmpde_problem_create(const ipmpde_grid* grid, const ipmpde_pde* pde, double alpha, double beta,
                                     const double* u_a, const double* u_b, const double* y_a, const double* y_b,
                                     const double* y_d, const double* f, const double* g, ipmpde_problem** out) {
  if (!out) return fail(IPMPDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !pde) return fail(IPMPDE_EINVAL, "grid and pde are required");
  if (grid->dim != 2 && grid->dim != 3) return fail(IPMPDE_EINVAL, "dim must be 2 or 3");
  if (!is_pow2m1(grid->n)) return fail(IPMPDE_EINVAL, "n must be 2^k - 1 with k >= 2");
  if (grid->n > (grid->dim == 2 ? 8191 : 511)) return fail(IPMPDE_EINVAL, "grid too large");
  if (pde->kind == IPMPDE_HEAT) return fail(IPMPDE_EINVAL, "heat-equation problems are made by ipmpde_heat_create");
  if (pde->kind != IPMPDE_POISSON && pde->kind != IPMPDE_CONVDIFF && pde->kind != IPMPDE_POISSON_Q1)
    return fail(IPMPDE_EINVAL, "unknown pde kind");
  if (pde->kind == IPMPDE_CONVDIFF && grid->dim != 2) return fail(IPMPDE_EINVAL, "convection-diffusion is 2D only");
  if (pde->kind == IPMPDE_CONVDIFF && !(pde->eps > 0 && std::isfinite(pde->eps)))
    return fail(IPMPDE_EINVAL, "eps must be positive");
  return problem_create_impl(grid->dim, grid->n, pde->kind, pde->eps, 1, 0.0, alpha, beta, u_a, u_b, y_a, y_b, y_d,
                             f, g, nullptr, out);
}

extern "C" int ipmpde_heat_create(const ipmpde_grid* grid, int nt, double tau, double alpha, double beta,
                                  const double* u_a, const double* u_b, const double* y_a, const double* y_b,
                                  const double* y_d, const double* f, const double* g, const double* y0,
                                  ipmpde_problem** out) {
  if (!out) return fail(IPMPDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid) return fail(IPMPDE_EINVAL, "grid is required");
  if (grid->dim != 2) return fail(IPMPDE_EINVAL, "the heat equation is posed on a 2D grid");
  if (!is_pow2m1(grid->n)) return fail(IPMPDE_EINVAL, "n must be 2^k - 1 with k >= 2");
  if (grid->n > 2047) return fail(IPMPDE_EINVAL, "grid too large");
  if (nt < 1 || nt > 65535) return fail(IPMPDE_EINVAL, "nt must be in [1, 65535]");
  if (!(tau > 0 && std::isfinite(tau))) return fail(IPMPDE_EINVAL, "tau must be positive");
  if ((double)grid->n * grid->n * nt > 1.0e8) return fail(IPMPDE_EINVAL, "too many space-time nodes");
  return problem_create_impl(2, grid->n, IPMPDE_HEAT, 1.0, nt, tau, alpha, beta, u_a, u_b, y_a, y_b, y_d, f, g, y0,
                             out);
}

extern "C" void ipmpde_problem_destroy(ipmpde_problem* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  problem_free(P);
  delete P;
}

// ---------------------------------------------------------------------------
// C API: solve, step, query

static hipStream_t S(ipmpde_stream s) { return (hipStream_t)s; }

// The group of one behind the single-problem entry points, created on first
// use; a problem that has not been solved or reset yet is put at the
// starting point first (default options).
static int ensure_self(ipmpde_problem* P, hipStream_t s) {
  if (P->in_engine) return fail(IPMPDE_EINVAL, "problem is queued or running in an engine");
  if (!P->self) TRY(group_create({P}, 1, P->dim, &P->self));
  if (P->need_init) {
    ipmpde_options o;
    ipmpde_default_options(&o);
    TRY(group_select(P->self, o));
    TRY(group_reset(P->self, {o}, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return IPMPDE_OK;
}

static int status_error(int st) {
  if (st == IPMPDE_ENOTCONVERGED) return fail(st, "IPM iteration limit reached");
  if (st == IPMPDE_EBREAKDOWN) return fail(st, "breakdown: NaN in the iterates or a collapsed step length");
  return st;
}

extern "C" int ipmpde_solve(ipmpde_problem* P, const ipmpde_options* opts, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  ipmpde_options o;
  TRY(resolve_opts(opts, &o));
  TRY(ensure_self(P, S(stream)));
  TRY(solve_group(P->self, {o}, S(stream)));
  return status_error(P->stats.status);
}

extern "C" int ipmpde_reset(ipmpde_problem* P, const ipmpde_options* opts, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  ipmpde_options oi, o;
  TRY(resolve_opts(opts, &oi));
  TRY(unit_form(P, oi, &o));
  TRY(ensure_self(P, S(stream)));
  TRY(group_select(P->self, o));
  return group_reset(P->self, {o}, S(stream));
}

// One Newton setup + Krylov solve of the single-problem group at barrier mu_new.
static int single_newton(ipmpde_problem* P, const ipmpde_options& o, double mu_new, hipStream_t s, int* its,
                         double* relres) {
  TRY(ensure_self(P, s));
  Group* G = P->self;
  G->H[0].active = 1;
  G->H[0].mu = mu_new;
  G->H[0].alpha0 = o.alpha0;
  TRY(newton_setup_group(G, o, s));
  TRY(krylov_group(G, o, s));
  if (its) *its = G->ctrl_h[0].its_total;
  if (relres) *relres = G->ctrl_h[0].relres;
  return krylov_status(G, 0);
}

extern "C" int ipmpde_ipm_step(ipmpde_problem* P, const ipmpde_options* opts, double mu_new, ipmpde_stream stream,
                               double* alpha_p, double* alpha_d, int* krylov_its, double* relres) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options oi, o;
  TRY(resolve_opts(opts, &oi));
  TRY(unit_form(P, oi, &o));
  mu_new /= P->rep;
  hipStream_t s = S(stream);
  int its = 0;
  double rel = 0;
  const int krc = single_newton(P, o, mu_new, s, &its, &rel);
  if (krc != IPMPDE_OK && krc != IPMPDE_EKRYLOV) return fail(krc, "Newton solve broke down");
  Group* G = P->self;
  hipLaunchKernelGGL(k_step_lengths, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  hipLaunchKernelGGL(k_update, gz(G, G->max_n), dim3(kBS), 0, s, G->D);
  HIP_TRY(hipGetLastError());
  TRY(read_stat(G, s));
  P->mu = mu_new;
  if (alpha_p) *alpha_p = G->stat_h[3];
  if (alpha_d) *alpha_d = G->stat_h[4];
  if (krylov_its) *krylov_its = its;
  if (relres) *relres = rel;
  if (krc == IPMPDE_EKRYLOV) return fail(krc, "Krylov tolerance not reached");
  return IPMPDE_OK;
}

extern "C" int ipmpde_newton_setup(ipmpde_problem* P, const ipmpde_options* opts, double mu_new, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options oi, o;
  TRY(resolve_opts(opts, &oi));
  TRY(unit_form(P, oi, &o));
  mu_new /= P->rep;
  TRY(ensure_self(P, S(stream)));
  Group* G = P->self;
  G->H[0].active = 1;
  G->H[0].mu = mu_new;
  TRY(newton_setup_group(G, o, S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  return IPMPDE_OK;
}

extern "C" int ipmpde_newton_direction(ipmpde_problem* P, const ipmpde_options* opts, double mu_new,
                                       ipmpde_stream stream, int* krylov_its, double* relres) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options oi, o;
  TRY(resolve_opts(opts, &oi));
  TRY(unit_form(P, oi, &o));
  const int rc = single_newton(P, o, mu_new / P->rep, S(stream), krylov_its, relres);
  if (rc == IPMPDE_EKRYLOV) return fail(rc, "Krylov tolerance not reached");
  if (rc != IPMPDE_OK) return fail(rc, "Newton solve broke down");
  return IPMPDE_OK;
}

extern "C" int ipmpde_measures(ipmpde_problem* P, ipmpde_stream stream, double* xp, double* xd, double* xc) {
  if (!P || !xp || !xd || !xc) return fail(IPMPDE_EINVAL, "NULL argument");
  TRY(ensure_self(P, S(stream)));
  Group* G = P->self;
  G->H[0].active = 1;
  TRY(group_measures(G, S(stream)));
  *xp = P->rep * G->stat_h[0];
  *xd = P->rep * G->stat_h[1];
  *xc = P->rep * G->stat_h[2];
  return IPMPDE_OK;
}

extern "C" int ipmpde_get_stats(const ipmpde_problem* P, ipmpde_stats* out) {
  if (!P || !out) return fail(IPMPDE_EINVAL, "NULL argument");
  *out = P->stats;
  return IPMPDE_OK;
}

static const double* field_ptr(const ipmpde_problem* P, int field, int* kind) {
  const Inst& I = P->I;
  const int n = P->n;
  *kind = 0;
  switch (field) {
    case IPMPDE_FIELD_Y: return I.y;
    case IPMPDE_FIELD_P: return I.p;
    case IPMPDE_FIELD_W: return I.w;
    case IPMPDE_FIELD_V: return I.v;
    case IPMPDE_FIELD_LAM_YA: return I.lya;
    case IPMPDE_FIELD_LAM_YB: return I.lyb;
    case IPMPDE_FIELD_LAM_WA: return I.lwa;
    case IPMPDE_FIELD_LAM_WB: return I.lwb;
    case IPMPDE_FIELD_LAM_VA: return I.lva;
    case IPMPDE_FIELD_LAM_VB: return I.lvb;
    case IPMPDE_FIELD_DY: return I.X;
    case IPMPDE_FIELD_DW: return I.X + n;
    case IPMPDE_FIELD_DV: return I.X + 2 * n;
    case IPMPDE_FIELD_DP: return I.X + 3 * n;
    case IPMPDE_FIELD_THETA_Y: return I.ty;
    case IPMPDE_FIELD_THETA_W: return I.tw;
    case IPMPDE_FIELD_THETA_V: return I.tv;
    case IPMPDE_FIELD_FHAT: return I.fhat;
    case IPMPDE_FIELD_U: *kind = 1; return nullptr;
    default: *kind = -1; return nullptr;
  }
}

extern "C" int ipmpde_set_observation(ipmpde_problem* P, const double* weights, size_t count) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (P->in_engine) return fail(IPMPDE_EINVAL, "problem is queued or running in an engine");
  if (P->pde == IPMPDE_POISSON_Q1) {
    // one weight per element ((N+1)^dim, numbered by the lower corner, x1
    // fastest): the tracking mass is assembled from the observed elements
    if (!weights) {
      P->I.eobs = P->eobs = nullptr;
      return IPMPDE_OK;
    }
    const size_t ne = pow_dim(P->N + 1, P->dim);
    if (count != ne) return fail(IPMPDE_EINVAL, "count must equal the number of elements, (N+1)^dim");
    for (size_t i = 0; i < count; ++i)
      if (!(weights[i] >= 0.0 && std::isfinite(weights[i]))) return fail(IPMPDE_EINVAL, "weights must be finite and >= 0");
    if (!P->eobs) TRY(P->mem.alloc_t(&P->eobs, count));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(P->eobs, weights, count * sizeof(double), hipMemcpyHostToDevice));
    P->I.eobs = P->eobs;
    return IPMPDE_OK;
  }
  if (!weights) {
    P->I.obs = P->obs = nullptr;
    P->obs_zero = false;
    return IPMPDE_OK;
  }
  if (count != (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal the number of nodes");
  bool zero = false;
  for (size_t i = 0; i < count; ++i) {
    if (!(weights[i] >= 0.0 && std::isfinite(weights[i]))) return fail(IPMPDE_EINVAL, "weights must be finite and >= 0");
    zero = zero || weights[i] == 0.0;
  }
  if (!P->obs) TRY(P->mem.alloc_t(&P->obs, count));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(P->obs, weights, count * sizeof(double), hipMemcpyHostToDevice));
  P->I.obs = P->obs;
  P->obs_zero = zero;
  return IPMPDE_OK;
}

// Fields reported in HD units under IPMPDE_MASS_HD: the bound multipliers and
// the barrier diagonals Theta (w times their unit-form values).
static bool hd_scaled(int field) {
  return (field >= IPMPDE_FIELD_LAM_YA && field <= IPMPDE_FIELD_LAM_VB) ||
         (field >= IPMPDE_FIELD_THETA_Y && field <= IPMPDE_FIELD_THETA_V);
}

extern "C" int ipmpde_query(const ipmpde_problem* P, int field, double* out, size_t count) {
  if (!P || !out) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal the number of nodes");
  int kind;
  const double* src = field_ptr(P, field, &kind);
  if (kind < 0) return fail(IPMPDE_EINVAL, "unknown field");
  if (P->in_engine) return fail(IPMPDE_EINVAL, "problem is queued or running in an engine");
  if (P->need_init) TRY(ensure_self((ipmpde_problem*)P, nullptr));
  src = field_ptr(P, field, &kind);
  if (field >= IPMPDE_FIELD_DY && field <= IPMPDE_FIELD_DP && !src)
    return fail(IPMPDE_EINVAL, "no Newton direction (workspace released)");
  HIP_TRY(hipDeviceSynchronize());
  if (kind == 1) {
    std::vector<double> v(count);
    HIP_TRY(hipMemcpy(out, P->I.w, count * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(v.data(), P->I.v, count * 8, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < count; ++i) out[i] -= v[i];
    return IPMPDE_OK;
  }
  if (!src) return fail(IPMPDE_EINVAL, "field not present (no state bounds)");
  HIP_TRY(hipMemcpy(out, src, count * 8, hipMemcpyDeviceToHost));
  if (P->rep != 1.0 && hd_scaled(field))
    for (size_t i = 0; i < count; ++i) out[i] *= P->rep;
  return IPMPDE_OK;
}

extern "C" int ipmpde_set_field(ipmpde_problem* P, int field, const double* in, size_t count) {
  if (!P || !in) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal the number of nodes");
  if (!(field == IPMPDE_FIELD_Y || field == IPMPDE_FIELD_P || field == IPMPDE_FIELD_W || field == IPMPDE_FIELD_V ||
        (field >= IPMPDE_FIELD_LAM_YA && field <= IPMPDE_FIELD_LAM_VB)))
    return fail(IPMPDE_EINVAL, "field is not an iterate");
  TRY(validate_array(in, count, "field"));
  TRY(ensure_self(P, nullptr));
  int kind;
  double* dst = (double*)field_ptr(P, field, &kind);
  if (!dst) return fail(IPMPDE_EINVAL, "field not present (no state bounds)");
  HIP_TRY(hipDeviceSynchronize());
  if (P->rep != 1.0 && hd_scaled(field)) {
    std::vector<double> v(in, in + count);
    for (double& x : v) x /= P->rep;
    HIP_TRY(hipMemcpy(dst, v.data(), count * 8, hipMemcpyHostToDevice));
    return IPMPDE_OK;
  }
  HIP_TRY(hipMemcpy(dst, in, count * 8, hipMemcpyHostToDevice));
  return IPMPDE_OK;
}

extern "C" int ipmpde_query_rhs(const ipmpde_problem* P, double* out, size_t count) {
  if (!P || !out) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != 4 * (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal 4 n");
  if (!P->I.rhs) return fail(IPMPDE_EINVAL, "no Newton right-hand side (workspace not allocated)");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, P->I.rhs, count * 8, hipMemcpyDeviceToHost));
  return IPMPDE_OK;
}

extern "C" int ipmpde_apply_operator(const ipmpde_problem* P, int transpose, const double* x, double* y,
                                     ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  TRY(ensure_self((ipmpde_problem*)P, S(stream)));
  Group* G = P->self;
  G->H[0].active = 1;
  TRY(group_sync(G, S(stream)));
  hipLaunchKernelGGL(k_apply_op, gz(G, P->n), dim3(kBS), 0, S(stream), G->D, x, y, transpose);
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

extern "C" int ipmpde_apply_saddle(ipmpde_problem* P, const double* x, double* y, ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  if (!P->setup_done || !P->self || P->setup_group != P->self) return fail(IPMPDE_EINVAL, "no Newton setup yet");
  Group* G = P->self;
  hipLaunchKernelGGL(k_saddle, gz(G, P->n), dim3(kBS), 0, S(stream), G->D, x, y);
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

extern "C" int ipmpde_apply_precond(ipmpde_problem* P, const ipmpde_options* opts, const double* x, double* y,
                                    ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  ipmpde_options o;
  TRY(resolve_opts(opts, &o));
  if (!P->setup_done || !P->self || P->setup_group != P->self || P->setup_fp32 != (o.mg_precision == IPMPDE_FP32))
    return fail(IPMPDE_EINVAL, "no Newton setup for this multigrid precision");
  Group* G = P->self;
  TRY(group_select(G, o));
  TRY(group_sync(G, S(stream)));
  const int pt = o.precond;  // IPMPDE_PD, IPMPDE_PT or IPMPDE_PPI
  if (G->fp32) precond_apply<float>(G, pt, x, y, 0, 0, S(stream));
  else precond_apply<double>(G, pt, x, y, 0, 0, S(stream));
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// batches

// A batch: one group over all instances, and for solves split into lanes
// (options.lanes > 1) one group per lane over its share of the instances,
// built on first use of a lane count.  Each lane runs on a stream of the
// batch's own (default priority), which also serves as its group's capture
// stream: a process has only a few hardware queues, and two lanes whose
// streams share one run one after the other.
struct ipmpde_batch {
  Group* G = nullptr;
  std::vector<Group*> lane_G;
  std::vector<std::vector<int>> lane_idx;  // instances of each lane (ascending)
  std::vector<hipStream_t> lane_s;
  std::vector<hipEvent_t> lane_ev;         // lane k's end
  hipEvent_t start_ev = nullptr;           // the caller's stream at the start of a solve
};

static void batch_release_lanes(ipmpde_batch* B) {
  for (Group* g : B->lane_G) group_release(g);
  for (hipStream_t s : B->lane_s)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : B->lane_ev)
    if (e) (void)hipEventDestroy(e);
  if (B->start_ev) (void)hipEventDestroy(B->start_ev);
  B->start_ev = nullptr;
  B->lane_G.clear();
  B->lane_idx.clear();
  B->lane_s.clear();
  B->lane_ev.clear();
}

// Split the batch's instances into L lanes of about equal work: the largest
// instances (by node count, times the steps of a heat problem) first, each to
// the lane with the least work so far.
static int batch_make_lanes(ipmpde_batch* B, int L) {
  if ((int)B->lane_G.size() == L) return IPMPDE_OK;
  batch_release_lanes(B);
  const Group* G = B->G;
  std::vector<int> order(G->count);
  for (int i = 0; i < G->count; ++i) order[i] = i;
  auto work = [&](int i) { return (double)G->probs[i]->n * std::max(1, G->probs[i]->nt); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<double> load(L, 0.0);
  B->lane_idx.assign(L, {});
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    B->lane_idx[k].push_back(i);
    load[k] += work(i);
  }
  B->lane_G.assign(L, nullptr);
  B->lane_s.assign(L, nullptr);
  B->lane_ev.assign(L, nullptr);
  hipError_t e = hipEventCreateWithFlags(&B->start_ev, hipEventDisableTiming);
  // the streams first, one after the other, so that they take distinct hardware queues where there are enough
  for (int k = 0; k < L && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&B->lane_s[k], hipStreamNonBlocking);
  for (int k = 0; k < L && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&B->lane_ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_release_lanes(B);
    return fail(IPMPDE_EDEVICE, std::string("lane setup: ") + hipGetErrorString(e));
  }
  for (int k = 0; k < L; ++k) {
    std::sort(B->lane_idx[k].begin(), B->lane_idx[k].end());
    std::vector<ipmpde_problem*> v;
    for (int i : B->lane_idx[k]) v.push_back(G->probs[i]);
    const int rc = group_create(v, (int)v.size(), G->dim, &B->lane_G[k]);
    if (rc != IPMPDE_OK) {
      batch_release_lanes(B);
      return rc;
    }
    B->lane_G[k]->cap_stream = B->lane_s[k];
    B->lane_G[k]->own_cap = false;
  }
  return IPMPDE_OK;
}

// Solve the batch split into L > 1 lanes, each lane's group on its own stream
// from a host thread of its own (lane 0 from the calling thread), between an
// event on the caller's stream and the caller's stream waiting for every
// lane.  The workspaces are allocated here first, so every allocation (the
// registered allocator's included) happens on the calling thread.
static int batch_solve_lanes(ipmpde_batch* B, const std::vector<ipmpde_options>& po, int L, hipStream_t s) {
  TRY(batch_make_lanes(B, L));
  std::vector<std::vector<ipmpde_options>> lpo(L);
  for (int k = 0; k < L; ++k) {
    for (int i : B->lane_idx[k]) lpo[k].push_back(po[i]);
    ipmpde_options u;
    TRY(unit_form(B->lane_G[k]->probs[0], lpo[k][0], &u));
    TRY(group_select(B->lane_G[k], u));
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipEventRecord(B->start_ev, s));
  for (int k = 0; k < L; ++k) HIP_TRY(hipStreamWaitEvent(B->lane_s[k], B->start_ev, 0));
  std::vector<int> rc(L, IPMPDE_OK);
  std::vector<std::string> msg(L);
  auto run = [&](int k) {
    if (k > 0) {
      const hipError_t e = hipSetDevice(dev);
      if (e != hipSuccess) {
        rc[k] = IPMPDE_EDEVICE;
        msg[k] = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return;
      }
    }
    rc[k] = solve_group(B->lane_G[k], lpo[k], B->lane_s[k]);
    if (rc[k] != IPMPDE_OK) msg[k] = g_err;
  };
  std::vector<std::thread> th;
  try {
    for (int k = 1; k < L; ++k) th.emplace_back(run, k);
  } catch (const std::exception& ex) {
    for (int k = (int)th.size() + 1; k < L; ++k) {
      rc[k] = IPMPDE_EDEVICE;
      msg[k] = std::string("cannot start a lane thread: ") + ex.what();
    }
  }
  run(0);
  for (auto& t : th) t.join();
  for (int k = 0; k < L; ++k) {
    HIP_TRY(hipEventRecord(B->lane_ev[k], B->lane_s[k]));
    HIP_TRY(hipStreamWaitEvent(s, B->lane_ev[k], 0));
  }
  for (int k = 0; k < L; ++k)
    if (rc[k] != IPMPDE_OK) return fail(rc[k], msg[k]);
  return IPMPDE_OK;
}

extern "C" int ipmpde_batch_create(ipmpde_problem* const* probs, int count, ipmpde_batch** out) {
  if (!out) return fail(IPMPDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || count < 1 || count > 65535) return fail(IPMPDE_EINVAL, "count must be in [1, 65535]");
  std::vector<ipmpde_problem*> v(probs, probs + count);
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(IPMPDE_EINVAL, "NULL problem in batch");
    if (v[i]->dim != v[0]->dim) return fail(IPMPDE_EINVAL, "all problems of a batch must have the same dimension");
    if ((v[i]->pde == IPMPDE_HEAT) != (v[0]->pde == IPMPDE_HEAT))
      return fail(IPMPDE_EINVAL, "a batch holds only heat-equation problems or none");
    if ((v[i]->pde == IPMPDE_POISSON_Q1) != (v[0]->pde == IPMPDE_POISSON_Q1))
      return fail(IPMPDE_EINVAL, "a batch holds only Q1 problems or none");
    for (int j = 0; j < i; ++j)
      if (v[j] == v[i]) return fail(IPMPDE_EINVAL, "a problem appears twice in the batch");
  }
  for (int i = 0; i < count; ++i)
    if (v[i]->in_engine) return fail(IPMPDE_EINVAL, "a problem of the batch is queued or running in an engine");
  ipmpde_batch* B = new ipmpde_batch();
  const int rc = group_create(v, count, v[0]->dim, &B->G);
  if (rc != IPMPDE_OK) { delete B; return rc; }
  *out = B;
  return IPMPDE_OK;
}

extern "C" void ipmpde_batch_destroy(ipmpde_batch* B) {
  if (!B) return;
  (void)hipDeviceSynchronize();
  batch_release_lanes(B);
  group_release(B->G);
  delete B;
}

extern "C" int ipmpde_batch_solve(ipmpde_batch* B, const ipmpde_options* opts, int per_problem, ipmpde_stream stream) {
  if (!B) return fail(IPMPDE_EINVAL, "batch is NULL");
  Group* G = B->G;
  std::vector<ipmpde_options> po(G->count);
  for (int i = 0; i < G->count; ++i) TRY(resolve_opts(opts ? (per_problem ? &opts[i] : opts) : nullptr, &po[i]));
  for (int i = 1; i < G->count; ++i) {
    const ipmpde_options &a = po[0], &b = po[i];
    if (a.krylov != b.krylov || a.precond != b.precond || a.restart != b.restart || a.krylov_tol != b.krylov_tol ||
        a.krylov_maxit != b.krylov_maxit || a.nu_pre != b.nu_pre || a.nu_post != b.nu_post || a.omega != b.omega ||
        a.mg_precision != b.mg_precision || a.chunk != b.chunk || a.use_graphs != b.use_graphs || a.vcycles != b.vcycles ||
        a.mg_tile != b.mg_tile || std::max(a.lanes, 1) != std::max(b.lanes, 1))
      return fail(IPMPDE_EINVAL, "Krylov, multigrid and lane options must agree across a batch");
  }
  const int L = std::min(std::max(po[0].lanes, 1), G->count);
  if (L > 1) return batch_solve_lanes(B, po, L, S(stream));
  return solve_group(G, po, S(stream));
}

#include "autotune.hip"
#include "engine.hip"
#include "noalloc.hip"
#include "timing.hip"
