// libipmpde: host driver and C ABI.
//
// One translation unit: the kernel files are included here so that every
// launch site sees its kernel.  The interior point loop (Appendix,
// Algorithm A.1) runs on the host; every vector operation of it runs in the
// kernels on the caller's stream.  The only device-to-host traffic is a few
// scalars per IPM iteration (measures, step lengths) and per Krylov chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ipmpde.h"
#include "common.h"
#include "kernels_ipm.hip"
#include "kernels_krylov.hip"
#include "kernels_mg.hip"
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

#define TRY(expr)                 \
  do {                            \
    int rc_ = (expr);             \
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

// ---------------------------------------------------------------------------
// problem

struct GraphKey {
  int mg_fp32, nu_pre, nu_post, chunk, maxit, parity, krylov, precond, restart;
  double omega;
  bool operator<(const GraphKey& o) const {
    return std::tie(mg_fp32, nu_pre, nu_post, chunk, maxit, parity, krylov, precond, restart, omega) <
           std::tie(o.mg_fp32, o.nu_pre, o.nu_post, o.chunk, o.maxit, o.parity, o.krylov, o.precond, o.restart,
                    o.omega);
  }
};

struct ipmpde_problem {
  Inst I;
  int dim = 0, N = 0, n = 0, pde = 0;
  double eps = 1.0, alpha = 0.0, beta = 0.0;
  bool has_y = false;
  std::vector<Alloc> allocs;
  // Newton system and Krylov workspace (4n each)
  double* rhs = nullptr;
  double* X = nullptr;
  double* V[2] = {nullptr, nullptr};
  double* Z[2] = {nullptr, nullptr};
  double* W[2] = {nullptr, nullptr};
  double* Q = nullptr;
  double* R = nullptr;
  double* KW[2] = {nullptr, nullptr};  // K w for the two most recent MINRES directions
  double* Rt = nullptr;                // tracked MINRES residual
  // FGMRES basis (allocated on first use)
  double* fV = nullptr;
  double* fZ = nullptr;
  int f_restart = 0;
  // multigrid storage per precision
  int nlev = 0;
  Level lv32[kMaxLev];
  Level lv64[kMaxLev];
  Level* lvd32 = nullptr;  // device copies of the level tables
  Level* lvd64 = nullptr;
  bool have32 = false, have64 = false;
  int coarse32 = 0, coarse64 = 0;
  // host mirrors (pinned)
  KrylovCtrl* ctrl_h = nullptr;
  double* stat_h = nullptr;
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  ipmpde_stats stats;
  double mu = 1.0;
  bool setup_done = false;
  int setup_fp32 = -1;
  double setup_mu = 0.0;
};

static int dalloc(ipmpde_problem* P, void** out, size_t bytes) {
  void* p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (g_alloc) {
    p = g_alloc(bytes, g_alloc_ctx);
    if (!p) return fail(IPMPDE_ENOMEM, "allocator callback returned NULL");
    P->allocs.push_back({p, g_free, g_alloc_ctx});
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(IPMPDE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    P->allocs.push_back({p, nullptr, nullptr});
  }
  *out = p;
  return IPMPDE_OK;
}

template <typename T>
static int dalloc_t(ipmpde_problem* P, T** out, size_t count) {
  return dalloc(P, (void**)out, count * sizeof(T));
}

static void free_all(ipmpde_problem* P) {
  for (auto& kv : P->graphs) hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  for (auto& a : P->allocs) {
    if (a.fr) a.fr(a.p, a.ctx);
    else hipFree(a.p);
  }
  P->allocs.clear();
  if (P->ctrl_h) hipHostFree(P->ctrl_h);
  if (P->stat_h) hipHostFree(P->stat_h);
  if (P->cap_stream) hipStreamDestroy(P->cap_stream);
  P->ctrl_h = nullptr;
  P->stat_h = nullptr;
  P->cap_stream = nullptr;
}

static bool is_pow2m1(int N) { return N >= 3 && ((N + 1) & N) == 0; }

static int level_count(int N) {
  int c = 1;
  while (N > 1) { N = (N - 1) / 2; ++c; }
  return c;
}

static size_t pow_dim(int N, int dim) { return dim == 2 ? (size_t)N * N : (size_t)N * N * N; }

// LDS budget of the single-workgroup coarse kernel (gfx950 has 160 KB of
// LDS per CU), and the largest grid it takes; finer levels run as
// grid-wide kernels.
static constexpr size_t kCoarseLds = 150 * 1024;

// p2: the Poisson 2D coarse kernel (padded layout), else the generic one.
static size_t coarse_level_elems(const Level& L, bool p2) {
  return p2 ? (size_t)coarse_p2_elems(L.N) : 4 * (size_t)L.n;
}

static int pick_coarse(const Level* lv, int nlev, size_t elem, int dim, bool p2) {
  const int nmax = dim == 2 ? 63 : 15;
  int cl = nlev - 1;
  size_t need = 0;
  for (int l = nlev - 1; l >= 0; --l) {
    need += coarse_level_elems(lv[l], p2) * elem;
    if (need > kCoarseLds || lv[l].N > nmax) break;
    cl = l;
  }
  return cl;
}

static size_t coarse_lds_bytes(const Level* lv, int nlev, int cl, size_t elem, bool p2) {
  size_t need = 0;
  for (int l = cl; l < nlev; ++l) need += coarse_level_elems(lv[l], p2) * elem;
  return need;
}

// Allow the coarse kernel more than the default 64 KB of dynamic LDS.
static int set_coarse_lds_limit() {
  static bool done = false;
  if (done) return IPMPDE_OK;
  HIP_TRY(hipFuncSetAttribute((const void*)k_mg_coarse<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kCoarseLds));
  HIP_TRY(hipFuncSetAttribute((const void*)k_mg_coarse<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kCoarseLds));
  HIP_TRY(hipFuncSetAttribute((const void*)k_mg_coarse_p2<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kCoarseLds));
  HIP_TRY(hipFuncSetAttribute((const void*)k_mg_coarse_p2<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kCoarseLds));
  done = true;
  return IPMPDE_OK;
}

static int ensure_mg(ipmpde_problem* P, bool fp32) {
  TRY(set_coarse_lds_limit());
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
    TRY(dalloc(P, &lv[l].x, nb));
    TRY(dalloc(P, &lv[l].x2, nb));
    TRY(dalloc(P, &lv[l].b, nb));
    TRY(dalloc(P, &lv[l].mh, nb));
    HIP_TRY(hipMemset(lv[l].x, 0, nb));
    HIP_TRY(hipMemset(lv[l].x2, 0, nb));
    HIP_TRY(hipMemset(lv[l].b, 0, nb));
    HIP_TRY(hipMemset(lv[l].mh, 0, nb));
    N = (N - 1) / 2;
  }
  (fp32 ? P->coarse32 : P->coarse64) = pick_coarse(lv, P->nlev, el, P->dim, P->dim == 2 && P->pde == IPMPDE_POISSON);
  Level*& lvd = fp32 ? P->lvd32 : P->lvd64;
  TRY(dalloc(P, (void**)&lvd, sizeof(Level) * kMaxLev));
  HIP_TRY(hipMemcpy(lvd, lv, sizeof(Level) * kMaxLev, hipMemcpyHostToDevice));
  have = true;
  return IPMPDE_OK;
}

static void select_mg(ipmpde_problem* P, const ipmpde_options& o) {
  const bool fp32 = o.mg_precision == IPMPDE_FP32;
  Level* lv = fp32 ? P->lv32 : P->lv64;
  for (int l = 0; l < P->nlev; ++l) P->I.lv[l] = lv[l];
  P->I.nlev = P->nlev;
  P->I.coarse_lev = fp32 ? P->coarse32 : P->coarse64;
  P->I.lvd = fp32 ? P->lvd32 : P->lvd64;
  P->I.mg_fp32 = fp32 ? 1 : 0;
  P->I.nu_pre = o.nu_pre;
  P->I.nu_post = o.nu_post;
  P->I.vcycles = o.vcycles;
  P->I.omega = o.omega > 0 ? o.omega : (P->dim == 2 ? 0.8 : 6.0 / 7.0);
}

static int nblk(long n) { return div_up(n, kBS); }

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
  return IPMPDE_OK;
}

static int check_options(const ipmpde_problem* P, const ipmpde_options& o) {
  if (!(o.sigma > 0 && o.sigma < 1)) return fail(IPMPDE_EINVAL, "sigma must lie in (0,1)");
  if (!(o.alpha0 > 0 && o.alpha0 < 1)) return fail(IPMPDE_EINVAL, "alpha0 must lie in (0,1)");
  if (!(o.eps_p > 0 && o.eps_d > 0 && o.eps_c > 0)) return fail(IPMPDE_EINVAL, "tolerances must be positive");
  if (!(o.mu0 > 0)) return fail(IPMPDE_EINVAL, "mu0 must be positive");
  if (o.ipm_maxit < 1 || o.ipm_maxit > IPMPDE_MAX_HIST - 1) return fail(IPMPDE_EINVAL, "ipm_maxit out of range");
  if (o.fixed_nli < 0 || o.fixed_nli > IPMPDE_MAX_HIST - 1) return fail(IPMPDE_EINVAL, "fixed_nli out of range");
  if (o.krylov != IPMPDE_MINRES && o.krylov != IPMPDE_FGMRES) return fail(IPMPDE_EINVAL, "unknown krylov");
  if (o.precond != IPMPDE_PD && o.precond != IPMPDE_PT) return fail(IPMPDE_EINVAL, "unknown precond");
  if (o.precond == IPMPDE_PT && o.krylov != IPMPDE_FGMRES)
    return fail(IPMPDE_EINVAL, "the block-triangular preconditioner needs FGMRES");
  if (o.restart < 1 || o.restart > 60) return fail(IPMPDE_EINVAL, "restart must be in [1,60]");
  if (!(o.krylov_tol > 0 && o.krylov_tol < 1)) return fail(IPMPDE_EINVAL, "krylov_tol must be in (0,1)");
  if (o.krylov_maxit < 1) return fail(IPMPDE_EINVAL, "krylov_maxit must be >= 1");
  if (o.vcycles != 1) return fail(IPMPDE_EINVAL, "vcycles must be 1");
  if (o.nu_pre < 1 || o.nu_pre > 6 || o.nu_post < 1 || o.nu_post > 6) return fail(IPMPDE_EINVAL, "nu out of [1,6]");
  if (o.krylov == IPMPDE_MINRES && o.nu_pre != o.nu_post)
    return fail(IPMPDE_EINVAL, "MINRES needs nu_pre == nu_post (symmetric preconditioner)");
  if (!(o.omega >= 0 && o.omega < 1.5)) return fail(IPMPDE_EINVAL, "omega out of range");
  if (o.mg_precision != IPMPDE_FP32 && o.mg_precision != IPMPDE_FP64) return fail(IPMPDE_EINVAL, "bad mg_precision");
  if (o.chunk < 2 || o.chunk > 64 || (o.chunk & 1)) return fail(IPMPDE_EINVAL, "chunk must be even in [2,64]");
  (void)P;
  return IPMPDE_OK;
}

static int resolve_opts(const ipmpde_options* in, ipmpde_options* out) {
  if (in) *out = *in;
  else ipmpde_default_options(out);
  return IPMPDE_OK;
}

// ---------------------------------------------------------------------------
// multigrid launch sequence

template <typename T>
static void launch_coarse(ipmpde_problem* P, int transpose, int guard, hipStream_t s) {
  const Inst& I = P->I;
  const bool p2 = P->dim == 2 && P->pde == IPMPDE_POISSON;
  const size_t lds = coarse_lds_bytes(I.lv, I.nlev, I.coarse_lev, sizeof(T), p2);
  if (p2) hipLaunchKernelGGL(k_mg_coarse_p2<T>, dim3(1), dim3(kCoarseBS), lds, s, I, guard);
  else hipLaunchKernelGGL(k_mg_coarse<T>, dim3(1), dim3(kCoarseBS), lds, s, I, transpose, guard);
}

template <typename T>
static void mg_vcycle_generic(ipmpde_problem* P, int transpose, int guard, hipStream_t s, T** out) {
  const Inst& I = P->I;
  const int cl = I.coarse_lev;
  T* cur[kMaxLev];
  for (int l = 0; l < cl; ++l) {
    const Level& L = I.lv[l];
    T* a = (T*)L.x;
    T* c = (T*)L.x2;
    for (int sw = 0; sw < I.nu_pre; ++sw) {
      hipLaunchKernelGGL(k_mg_jacobi<T>, dim3(nblk(L.n)), dim3(kBS), 0, s, I, l, a, c, sw == 0 ? 1 : 0, transpose, guard);
      std::swap(a, c);
    }
    cur[l] = a;
    hipLaunchKernelGGL(k_mg_restrict<T>, dim3(nblk(I.lv[l + 1].n)), dim3(kBS), 0, s, I, l, a, transpose, guard);
  }
  launch_coarse<T>(P, transpose, guard, s);
  cur[cl] = (T*)I.lv[cl].x;
  for (int l = cl - 1; l >= 0; --l) {
    const Level& L = I.lv[l];
    T* a = cur[l];
    T* c = (a == (T*)L.x) ? (T*)L.x2 : (T*)L.x;
    hipLaunchKernelGGL(k_mg_prolong<T>, dim3(nblk(L.n)), dim3(kBS), 0, s, I, l, a, cur[l + 1], guard);
    for (int sw = 0; sw < I.nu_post; ++sw) {
      hipLaunchKernelGGL(k_mg_jacobi<T>, dim3(nblk(L.n)), dim3(kBS), 0, s, I, l, a, c, 0, transpose, guard);
      std::swap(a, c);
    }
    cur[l] = a;
  }
  *out = cur[0];
}

template <typename T>
static void launch_down2d(int nu, dim3 g, size_t lds, hipStream_t s, const Inst& I, int l, const T* bsrc,
                          const double* ty, T* xout, int tr, int guard) {
  switch (nu) {
#define D_(NU) case NU: hipLaunchKernelGGL((k_mg_down2d<T, NU>), g, dim3(kBS), lds, s, I, l, bsrc, ty, xout, tr, guard); break;
    D_(1) D_(2) D_(3) D_(4) D_(5) D_(6)
#undef D_
  }
}
template <typename T>
static void launch_up2d(int nu, dim3 g, size_t lds, hipStream_t s, const Inst& I, int l, const T* xpre, const T* xc,
                        T* xout, int tr, int guard) {
  switch (nu) {
#define U_(NU) case NU: hipLaunchKernelGGL((k_mg_up2d<T, NU>), g, dim3(kBS), lds, s, I, l, xpre, xc, xout, tr, guard); break;
    U_(1) U_(2) U_(3) U_(4) U_(5) U_(6)
#undef U_
  }
}

// 2D V-cycle with the fused level kernels: per level one descent launch
// (smoothing + residual + restriction) and one ascent launch (prolongation +
// smoothing).  scaled_src != nullptr: the level-0 right-hand side is
// (1 + Theta_y) scaled_src.  Output: level 0's x2.
template <typename T>
static void mg_vcycle_2d(ipmpde_problem* P, int transpose, int guard, const T* scaled_src, hipStream_t s, T** out) {
  const Inst& I = P->I;
  const int cl = I.coarse_lev;
  const size_t ldd = 4 * (size_t)down_width(I.nu_pre) * down_width(I.nu_pre) * sizeof(T);
  const size_t ldu = 4 * (size_t)up_width(I.nu_post) * up_width(I.nu_post) * sizeof(T);
  for (int l = 0; l < cl; ++l) {
    const Level& L = I.lv[l];
    const int nt = div_up(I.lv[l + 1].N, kTC);
    const T* bsrc = (l == 0 && scaled_src) ? scaled_src : (const T*)L.b;
    const double* ty = (l == 0 && scaled_src) ? I.ty : nullptr;
    launch_down2d<T>(I.nu_pre, dim3(nt, nt), ldd, s, I, l, bsrc, ty, (T*)L.x, transpose, guard);
  }
  launch_coarse<T>(P, transpose, guard, s);
  for (int l = cl - 1; l >= 0; --l) {
    const Level& L = I.lv[l];
    const int nt = div_up(L.N, kTF);
    const T* xc = (l + 1 == cl) ? (const T*)I.lv[cl].x : (const T*)I.lv[l + 1].x2;
    launch_up2d<T>(I.nu_post, dim3(nt, nt), ldu, s, I, l, (const T*)L.x, xc, (T*)L.x2, transpose, guard);
  }
  *out = cl == 0 ? (T*)I.lv[0].x : (T*)I.lv[0].x2;
}

template <typename T>
static void mg_vcycle(ipmpde_problem* P, int transpose, int guard, hipStream_t s, T** out) {
  if (P->dim == 2) mg_vcycle_2d<T>(P, transpose, guard, nullptr, s, out);
  else mg_vcycle_generic<T>(P, transpose, guard, s, out);
}

// S_hat^-1 applied to lv[0].b (Sec. 4.2): V-cycle on A + M_hat, scale by
// 1 + Theta_y, V-cycle on (A + M_hat)^T.  Returns the level-0 output array.
template <typename T>
static T* schur_inv(ipmpde_problem* P, int guard, hipStream_t s) {
  T* x1;
  T* x2;
  if (P->dim == 2 && P->I.coarse_lev > 0) {
    mg_vcycle_2d<T>(P, 0, guard, nullptr, s, &x1);
    mg_vcycle_2d<T>(P, 1, guard, x1, s, &x2);
    return x2;
  }
  mg_vcycle<T>(P, 0, guard, s, &x1);
  hipLaunchKernelGGL(k_mg_scale_ty<T>, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, (const T*)x1, guard);
  mg_vcycle<T>(P, 1, guard, s, &x2);
  return x2;
}

// ---------------------------------------------------------------------------
// MINRES

template <typename T>
static void minres_iteration(ipmpde_problem* P, int par, int maxit, hipStream_t s) {
  const Inst& I = P->I;
  const int nb = nblk(P->n);
  double* Zc = P->Z[par];
  double* Zo = P->Z[1 - par];
  double* Vc = P->V[par];
  double* Vo = P->V[1 - par];
  hipLaunchKernelGGL(k_minres_k1, dim3(nb), dim3(kBS), 0, s, I, Zc, Zo, P->W[1 - par], P->W[par], P->X, P->Q,
                     P->KW[1 - par], P->KW[par], P->Rt, 0);
  hipLaunchKernelGGL(k_minres_k2<T>, dim3(nb), dim3(kBS), 0, s, I, P->Q, Vc, Vo, Zo);
  T* xs = schur_inv<T>(P, 1, s);
  hipLaunchKernelGGL(k_minres_k4<T>, dim3(nb), dim3(kBS), 0, s, I, (const T*)xs, Vo, Zo, 1, 0.0, maxit);
}

template <typename T>
static void minres_start(ipmpde_problem* P, const double* src, double rtarget, int maxit, hipStream_t s) {
  const Inst& I = P->I;
  const int nb = nblk(P->n);
  hipLaunchKernelGGL(k_minres_init<T>, dim3(nb), dim3(kBS), 0, s, I, src, P->V[1], P->V[0], P->Z[1], P->W[0], P->W[1],
                     P->KW[0], P->KW[1], P->Rt);
  T* xs = schur_inv<T>(P, 0, s);
  hipLaunchKernelGGL(k_minres_k4<T>, dim3(nb), dim3(kBS), 0, s, I, (const T*)xs, P->V[1], P->Z[1], 0, rtarget, maxit);
}

// Clear the stop flag (used before timing the iteration kernels in isolation).
__global__ void k_ctrl_continue(KrylovCtrl* C, double unused) {
  (void)unused;
  C->stop = 0;
  C->pending = 0;
}

static int read_ctrl(ipmpde_problem* P, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(P->ctrl_h, P->I.ctrl, offsetof(KrylovCtrl, hcol), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IPMPDE_OK;
}

template <typename T>
static int run_minres_chunk(ipmpde_problem* P, const ipmpde_options& o, int par, int maxit, hipStream_t s) {
  if (!o.use_graphs) {
    for (int t = 0; t < o.chunk; ++t) minres_iteration<T>(P, (par + t) & 1, maxit, s);
    return IPMPDE_OK;
  }
  GraphKey key{P->I.mg_fp32, o.nu_pre, o.nu_post, o.chunk, maxit, par, IPMPDE_MINRES, IPMPDE_PD, 0, P->I.omega};
  auto it = P->graphs.find(key);
  if (it == P->graphs.end()) {
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < o.chunk; ++t) minres_iteration<T>(P, (par + t) & 1, maxit, P->cap_stream);
    HIP_TRY(hipStreamEndCapture(P->cap_stream, &g));
    hipGraphExec_t ge;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return fail(IPMPDE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = P->graphs.emplace(key, ge).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, s));
  return IPMPDE_OK;
}

// Attainable accuracy: a relative residual below c eps |(|K||x| + |b|)| / |b|
// cannot be resolved by evaluating b - K x in FP64; the Krylov solves accept
// it as converged when the requested tolerance lies below that floor.
static double floor_factor() { return 16.0 * 2.220446049250313e-16; }

// Solve K X = rhs to |rhs - K X| <= tol |rhs|.  MINRES stops on its tracked
// residual; the true residual is then checked, and a drift of the recurrence
// (rare) restarts MINRES from the true residual.  Returns IPMPDE_OK or
// IPMPDE_EKRYLOV; *its receives the iterations, *relres the true relative residual.
template <typename T>
static int minres_solve(ipmpde_problem* P, const ipmpde_options& o, hipStream_t s, int* its, double* relres) {
  const int n4 = 4 * P->n;
  HIP_TRY(hipMemsetAsync(P->X, 0, n4 * sizeof(double), s));
  TRY(read_ctrl(P, s));
  const double bnorm = P->ctrl_h->bnorm;
  *its = 0;
  *relres = 0.0;
  if (!(bnorm > 0.0)) {
    if (bnorm != bnorm) return fail(IPMPDE_EBREAKDOWN, "NaN in the Newton right-hand side");
    return IPMPDE_OK;
  }
  const double tol = o.krylov_tol;
  const double* src = P->rhs;
  int total = 0;
  for (int cycle = 0; cycle < 16; ++cycle) {
    const int left = o.krylov_maxit - total;
    minres_start<T>(P, src, tol * bnorm, left, s);
    TRY(read_ctrl(P, s));
    while (!P->ctrl_h->stop && P->ctrl_h->iter < left) {
      TRY(run_minres_chunk<T>(P, o, 1, left, s));
      TRY(read_ctrl(P, s));
    }
    const int it = P->ctrl_h->iter;
    // the pending update exists when the stop came from K4 (limit, breakdown)
    hipLaunchKernelGGL(k_minres_flush, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, P->Z[it & 1], P->W[it & 1],
                       P->W[(it + 1) & 1], P->X);
    hipLaunchKernelGGL(k_true_residual, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, P->X, P->rhs, P->R);
    TRY(read_ctrl(P, s));
    total += it;
    const double rel = P->ctrl_h->rnorm / bnorm;
    *its = total;
    *relres = rel;
    if (rel <= std::max(tol, floor_factor() * P->ctrl_h->rfloor / bnorm)) return IPMPDE_OK;
    if (!(rel == rel)) return fail(IPMPDE_EBREAKDOWN, "NaN in the Krylov iterate");
    if (P->ctrl_h->breakdown) return fail(IPMPDE_EKRYLOV, "MINRES breakdown (preconditioner not positive definite)");
    if (total >= o.krylov_maxit) return fail(IPMPDE_EKRYLOV, "Krylov iteration limit reached");
    src = P->R;
  }
  return fail(IPMPDE_EKRYLOV, "Krylov solve did not converge within 16 restarts");
}

// ---------------------------------------------------------------------------
// Newton setup and IPM step

template <typename T>
static int newton_setup_t(ipmpde_problem* P, double mu, hipStream_t s) {
  const Inst& I = P->I;
  hipLaunchKernelGGL(k_newton_setup<T>, dim3(nblk(P->n)), dim3(kBS), 0, s, I, mu, P->rhs, (T*)I.lv[0].mh);
  for (int l = 0; l + 1 < I.nlev; ++l)
    hipLaunchKernelGGL(k_restrict_diag<T>, dim3(nblk(I.lv[l + 1].n)), dim3(kBS), 0, s, (const T*)I.lv[l].mh,
                       (T*)I.lv[l + 1].mh, I.lv[l].N, I.lv[l + 1].N, P->dim);
  return IPMPDE_OK;
}

static int newton_setup(ipmpde_problem* P, const ipmpde_options& o, double mu, hipStream_t s) {
  TRY(ensure_mg(P, o.mg_precision == IPMPDE_FP32));
  select_mg(P, o);
  if (o.mg_precision == IPMPDE_FP32) TRY(newton_setup_t<float>(P, mu, s));
  else TRY(newton_setup_t<double>(P, mu, s));
  HIP_TRY(hipGetLastError());
  P->setup_done = true;
  P->setup_fp32 = o.mg_precision == IPMPDE_FP32;
  P->setup_mu = mu;
  return IPMPDE_OK;
}

static int ensure_fgmres(ipmpde_problem* P, int restart);
template <typename T>
static int fgmres_solve(ipmpde_problem* P, const ipmpde_options& o, hipStream_t s, int* its, double* relres);

static int krylov_solve(ipmpde_problem* P, const ipmpde_options& o, hipStream_t s, int* its, double* relres) {
  const bool f32 = o.mg_precision == IPMPDE_FP32;
  if (o.krylov == IPMPDE_MINRES) return f32 ? minres_solve<float>(P, o, s, its, relres) : minres_solve<double>(P, o, s, its, relres);
  TRY(ensure_fgmres(P, o.restart));
  return f32 ? fgmres_solve<float>(P, o, s, its, relres) : fgmres_solve<double>(P, o, s, its, relres);
}

static int read_stat(ipmpde_problem* P, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(P->stat_h, P->I.stat, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IPMPDE_OK;
}

static int measures(ipmpde_problem* P, hipStream_t s, double* xp, double* xd, double* xc) {
  hipLaunchKernelGGL(k_measures, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I);
  HIP_TRY(hipGetLastError());
  TRY(read_stat(P, s));
  *xp = P->stat_h[0];
  *xd = P->stat_h[1];
  *xc = P->stat_h[2];
  return IPMPDE_OK;
}

// One pass of the loop body of Algorithm A.1 at barrier mu_new.
static int ipm_step_impl(ipmpde_problem* P, const ipmpde_options& o, double mu_new, hipStream_t s, double* aP,
                         double* aD, int* its, double* relres) {
  TRY(newton_setup(P, o, mu_new, s));
  int krc = krylov_solve(P, o, s, its, relres);
  if (krc != IPMPDE_OK && krc != IPMPDE_EKRYLOV) return krc;
  hipLaunchKernelGGL(k_step_lengths, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, P->X, mu_new, o.alpha0);
  hipLaunchKernelGGL(k_update, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, P->X, mu_new);
  HIP_TRY(hipGetLastError());
  TRY(read_stat(P, s));
  *aP = P->stat_h[3];
  *aD = P->stat_h[4];
  P->mu = mu_new;
  return krc;
}

static void reset_state(ipmpde_problem* P, double mu0, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, mu0);
  P->mu = mu0;
}

static int solve_impl(ipmpde_problem* P, const ipmpde_options& o, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  ipmpde_stats& st = P->stats;
  std::memset(&st, 0, sizeof(st));
  reset_state(P, o.mu0, s);
  HIP_TRY(hipGetLastError());
  int status = IPMPDE_ENOTCONVERGED;
  double aP = 0, aD = 0;
  for (int k = 0;; ++k) {
    double xp, xd, xc;
    TRY(measures(P, s, &xp, &xd, &xc));
    st.hist_mu[k] = P->mu;
    st.hist_xi_p[k] = xp;
    st.hist_xi_d[k] = xd;
    st.hist_xi_c[k] = xc;
    st.hist_len = k + 1;
    st.nli = k;
    st.xi_p = xp; st.xi_d = xd; st.xi_c = xc; st.mu = P->mu;
    if (!(xp == xp && xd == xd && xc == xc)) { status = fail(IPMPDE_EBREAKDOWN, "NaN in the IPM iterates"); break; }
    if (o.fixed_nli > 0) {
      if (k >= o.fixed_nli) { status = IPMPDE_OK; break; }
    } else if (xp <= o.eps_p && xd <= o.eps_d && xc <= o.eps_c) {
      status = IPMPDE_OK;
      break;
    }
    if (k >= o.ipm_maxit) { status = fail(IPMPDE_ENOTCONVERGED, "IPM iteration limit reached"); break; }
    int its = 0;
    double rel = 0;
    int rc = ipm_step_impl(P, o, o.sigma * P->mu, s, &aP, &aD, &its, &rel);
    st.hist_krylov[k] = its;
    st.hist_krylov_relres[k] = rel;
    st.hist_alpha_p[k] = aP;
    st.hist_alpha_d[k] = aD;
    st.krylov_its += its;
    if (rc == IPMPDE_EKRYLOV) st.krylov_fail += 1;
    else if (rc != IPMPDE_OK) { status = rc; break; }
    if (!(aP > 1e-10 && aD > 1e-10)) { status = fail(IPMPDE_EBREAKDOWN, "step length collapsed"); break; }
  }
  st.status = status;
  st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
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
    // 1-based full-grid coordinates
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

extern "C" const char* ipmpde_version(void) { return "libipmpde 0.1 (gfx950)"; }
extern "C" const char* ipmpde_last_error(void) { return g_err.c_str(); }

extern "C" int ipmpde_set_allocator(ipmpde_alloc_fn a, ipmpde_free_fn f, void* ctx) {
  if ((a == nullptr) != (f == nullptr)) return fail(IPMPDE_EINVAL, "allocator and free must both be set or both NULL");
  g_alloc = a;
  g_free = f;
  g_alloc_ctx = ctx;
  return IPMPDE_OK;
}

extern "C" size_t ipmpde_footprint_bytes(const ipmpde_grid* grid, const ipmpde_pde* pde, int has_y,
                                         const ipmpde_options* opts) {
  if (!grid || !pde) return 0;
  ipmpde_options o;
  resolve_opts(opts, &o);
  const size_t n = pow_dim(grid->n, grid->dim);
  size_t fields = 6 + 8 + 4 + (has_y ? 4 : 0);  // data, iterates, diagonals
  size_t words = fields * n + 4 * n * 11;        // Newton rhs, X, V, Z, W, Q, R
  if (o.krylov == IPMPDE_FGMRES) words += 4 * n * (2 * (size_t)o.restart + 1);
  const size_t el = o.mg_precision == IPMPDE_FP32 ? 4 : 8;
  const double lvl = grid->dim == 2 ? 4.0 / 3.0 : 8.0 / 7.0;
  return words * 8 + (size_t)(4 * el * n * lvl) + (1 << 20);
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
  if (pde->kind != IPMPDE_POISSON && pde->kind != IPMPDE_CONVDIFF) return fail(IPMPDE_EINVAL, "unknown pde kind");
  if (pde->kind == IPMPDE_CONVDIFF && grid->dim != 2) return fail(IPMPDE_EINVAL, "convection-diffusion is 2D only");
  if (pde->kind == IPMPDE_CONVDIFF && !(pde->eps > 0 && std::isfinite(pde->eps)))
    return fail(IPMPDE_EINVAL, "eps must be positive");
  if (!(alpha > 0 && std::isfinite(alpha))) return fail(IPMPDE_EINVAL, "alpha must be positive");
  if (!(beta >= 0 && std::isfinite(beta))) return fail(IPMPDE_EINVAL, "beta must be non-negative");
  if (!u_a || !u_b || !y_d) return fail(IPMPDE_EINVAL, "u_a, u_b and y_d are required");
  if ((y_a == nullptr) != (y_b == nullptr)) return fail(IPMPDE_EINVAL, "y_a and y_b must both be given or both NULL");
  const int dim = grid->dim, N = grid->n;
  const size_t n = pow_dim(N, dim);
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

  std::vector<double> fhat(n, 0.0);
  if (f) std::copy(f, f + n, fhat.begin());
  if (g) fold_boundary(dim, N, pde->kind, pde->kind == IPMPDE_POISSON ? 1.0 : pde->eps, g, fhat);

  ipmpde_problem* P = new ipmpde_problem();
  P->dim = dim; P->N = N; P->n = (int)n; P->pde = pde->kind;
  P->eps = pde->kind == IPMPDE_POISSON ? 1.0 : pde->eps;
  P->alpha = alpha; P->beta = beta; P->has_y = y_a != nullptr;
  P->nlev = level_count(N);
  std::memset(&P->stats, 0, sizeof(P->stats));
  Inst& I = P->I;
  std::memset(&I, 0, sizeof(I));
  I.dim = dim; I.N = N; I.n = (int)n; I.pde = P->pde; I.has_y = P->has_y ? 1 : 0;
  I.h = 1.0 / (N + 1); I.eps = P->eps; I.alpha = alpha; I.beta = beta;
  auto cleanup = [&](int rc) { free_all(P); delete P; return rc; };
  int rc = IPMPDE_OK;
  double* dev[32];
  int nd = 0;
  auto A = [&](double** p) -> int { int r = dalloc_t(P, p, n); if (r == IPMPDE_OK) dev[nd++] = *p; return r; };
  double *ua, *ub, *ya = nullptr, *yb = nullptr, *yd, *fh;
  if ((rc = A(&ua)) || (rc = A(&ub)) || (rc = A(&yd)) || (rc = A(&fh))) return cleanup(rc);
  if (P->has_y && ((rc = A(&ya)) || (rc = A(&yb)))) return cleanup(rc);
  if ((rc = A(&I.y)) || (rc = A(&I.w)) || (rc = A(&I.v)) || (rc = A(&I.p)) || (rc = A(&I.lwa)) ||
      (rc = A(&I.lwb)) || (rc = A(&I.lva)) || (rc = A(&I.lvb)) || (rc = A(&I.ty)) || (rc = A(&I.tw)) ||
      (rc = A(&I.tv)) || (rc = A(&I.mh)))
    return cleanup(rc);
  if (P->has_y && ((rc = A(&I.lya)) || (rc = A(&I.lyb)))) return cleanup(rc);
  I.ua = ua; I.ub = ub; I.ya = ya; I.yb = yb; I.yd = yd; I.fhat = fh;
  const size_t n4 = 4 * n;
  if ((rc = dalloc_t(P, &P->rhs, n4)) || (rc = dalloc_t(P, &P->X, n4)) || (rc = dalloc_t(P, &P->V[0], n4)) ||
      (rc = dalloc_t(P, &P->V[1], n4)) || (rc = dalloc_t(P, &P->Z[0], n4)) || (rc = dalloc_t(P, &P->Z[1], n4)) ||
      (rc = dalloc_t(P, &P->W[0], n4)) || (rc = dalloc_t(P, &P->W[1], n4)) || (rc = dalloc_t(P, &P->Q, n4)) ||
      (rc = dalloc_t(P, &P->R, n4)) || (rc = dalloc_t(P, &P->KW[0], n4)) || (rc = dalloc_t(P, &P->KW[1], n4)) ||
      (rc = dalloc_t(P, &P->Rt, n4)))
    return cleanup(rc);
  const size_t nparts = std::max<size_t>(4 * (size_t)nblk((long)n), 64 * kBS) + 64;
  if ((rc = dalloc_t(P, &I.partials, nparts)) || (rc = dalloc_t(P, &I.counter, kTicketStride * (kTicketGroups + 1))) ||
      (rc = dalloc(P, (void**)&I.ctrl, sizeof(KrylovCtrl))) || (rc = dalloc_t(P, &I.stat, 16)))
    return cleanup(rc);
  auto hip_fail = [&](hipError_t e, const char* what) {
    return cleanup(fail(IPMPDE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)));
  };
  hipError_t e;
  if ((e = hipMemset(I.counter, 0, kTicketStride * (kTicketGroups + 1) * sizeof(unsigned))) != hipSuccess) return hip_fail(e, "hipMemset");
  if ((e = hipMemset(I.ctrl, 0, sizeof(KrylovCtrl))) != hipSuccess) return hip_fail(e, "hipMemset");
  if ((e = hipMemset(I.stat, 0, 16 * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMemset");
  for (int k = 0; k < nd; ++k)
    if ((e = hipMemset(dev[k], 0, n * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMemset");
  if ((e = hipMemset(P->X, 0, n4 * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMemset");
  if ((e = hipMemcpy(ua, u_a, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(ub, u_b, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(yd, y_d, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if ((e = hipMemcpy(fh, fhat.data(), n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  if (P->has_y) {
    if ((e = hipMemcpy(ya, y_a, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(yb, y_b, n * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  if ((e = hipHostMalloc((void**)&P->ctrl_h, sizeof(KrylovCtrl), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "hipHostMalloc");
  if ((e = hipHostMalloc((void**)&P->stat_h, 16 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "hipHostMalloc");
  if ((e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "hipStreamCreate");
  ipmpde_options o;
  ipmpde_default_options(&o);
  if ((rc = ensure_mg(P, true)) != IPMPDE_OK) return cleanup(rc);
  select_mg(P, o);
  reset_state(P, o.mu0, nullptr);
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "init");
  *out = P;
  return IPMPDE_OK;
}

extern "C" void ipmpde_problem_destroy(ipmpde_problem* P) {
  if (!P) return;
  hipDeviceSynchronize();
  free_all(P);
  delete P;
}

// ---------------------------------------------------------------------------
// C API: solve, step, query

static hipStream_t S(ipmpde_stream s) { return (hipStream_t)s; }

extern "C" int ipmpde_solve(ipmpde_problem* P, const ipmpde_options* opts, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  return solve_impl(P, o, S(stream));
}

extern "C" int ipmpde_reset(ipmpde_problem* P, const ipmpde_options* opts, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  reset_state(P, o.mu0, S(stream));
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

extern "C" int ipmpde_ipm_step(ipmpde_problem* P, const ipmpde_options* opts, double mu_new, ipmpde_stream stream,
                               double* alpha_p, double* alpha_d, int* krylov_its, double* relres) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  double aP = 0, aD = 0, rel = 0;
  int its = 0;
  int rc = ipm_step_impl(P, o, mu_new, S(stream), &aP, &aD, &its, &rel);
  if (alpha_p) *alpha_p = aP;
  if (alpha_d) *alpha_d = aD;
  if (krylov_its) *krylov_its = its;
  if (relres) *relres = rel;
  return rc;
}

extern "C" int ipmpde_newton_setup(ipmpde_problem* P, const ipmpde_options* opts, double mu_new, ipmpde_stream stream) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  TRY(newton_setup(P, o, mu_new, S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  return IPMPDE_OK;
}

extern "C" int ipmpde_newton_direction(ipmpde_problem* P, const ipmpde_options* opts, double mu_new,
                                       ipmpde_stream stream, int* krylov_its, double* relres) {
  if (!P) return fail(IPMPDE_EINVAL, "problem is NULL");
  if (!(mu_new > 0)) return fail(IPMPDE_EINVAL, "mu_new must be positive");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  TRY(newton_setup(P, o, mu_new, S(stream)));
  int its = 0;
  double rel = 0;
  int rc = krylov_solve(P, o, S(stream), &its, &rel);
  if (krylov_its) *krylov_its = its;
  if (relres) *relres = rel;
  return rc;
}

extern "C" int ipmpde_measures(ipmpde_problem* P, ipmpde_stream stream, double* xp, double* xd, double* xc) {
  if (!P || !xp || !xd || !xc) return fail(IPMPDE_EINVAL, "NULL argument");
  return measures(P, S(stream), xp, xd, xc);
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
    case IPMPDE_FIELD_DY: return P->X;
    case IPMPDE_FIELD_DW: return P->X + n;
    case IPMPDE_FIELD_DV: return P->X + 2 * n;
    case IPMPDE_FIELD_DP: return P->X + 3 * n;
    case IPMPDE_FIELD_THETA_Y: return I.ty;
    case IPMPDE_FIELD_THETA_W: return I.tw;
    case IPMPDE_FIELD_THETA_V: return I.tv;
    case IPMPDE_FIELD_FHAT: return I.fhat;
    case IPMPDE_FIELD_U: *kind = 1; return nullptr;
    default: *kind = -1; return nullptr;
  }
}

extern "C" int ipmpde_query(const ipmpde_problem* P, int field, double* out, size_t count) {
  if (!P || !out) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal the number of nodes");
  int kind;
  const double* src = field_ptr(P, field, &kind);
  if (kind < 0) return fail(IPMPDE_EINVAL, "unknown field");
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
  return IPMPDE_OK;
}

extern "C" int ipmpde_set_field(ipmpde_problem* P, int field, const double* in, size_t count) {
  if (!P || !in) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal the number of nodes");
  if (!(field == IPMPDE_FIELD_Y || field == IPMPDE_FIELD_P || field == IPMPDE_FIELD_W || field == IPMPDE_FIELD_V ||
        (field >= IPMPDE_FIELD_LAM_YA && field <= IPMPDE_FIELD_LAM_VB)))
    return fail(IPMPDE_EINVAL, "field is not an iterate");
  TRY(validate_array(in, count, "field"));
  int kind;
  double* dst = (double*)field_ptr(P, field, &kind);
  if (!dst) return fail(IPMPDE_EINVAL, "field not present (no state bounds)");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(dst, in, count * 8, hipMemcpyHostToDevice));
  return IPMPDE_OK;
}

extern "C" int ipmpde_query_rhs(const ipmpde_problem* P, double* out, size_t count) {
  if (!P || !out) return fail(IPMPDE_EINVAL, "NULL argument");
  if (count != 4 * (size_t)P->n) return fail(IPMPDE_EINVAL, "count must equal 4 n");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, P->rhs, count * 8, hipMemcpyDeviceToHost));
  return IPMPDE_OK;
}

extern "C" int ipmpde_apply_operator(const ipmpde_problem* P, int transpose, const double* x, double* y,
                                     ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_apply_op, dim3(nblk(P->n)), dim3(kBS), 0, S(stream), P->I, x, y, transpose);
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

extern "C" int ipmpde_apply_saddle(ipmpde_problem* P, const double* x, double* y, ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  if (!P->setup_done) return fail(IPMPDE_EINVAL, "no Newton setup yet");
  hipLaunchKernelGGL(k_saddle, dim3(nblk(P->n)), dim3(kBS), 0, S(stream), P->I, x, y);
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

template <typename T>
static void precond_apply_t(ipmpde_problem* P, int pt, const double* x, double* y, int guard, hipStream_t s) {
  hipLaunchKernelGGL(k_precond_diag<T>, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, x, y, pt, guard);
  if (pt) hipLaunchKernelGGL(k_pt_rhs<T>, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, x, (const double*)y, guard);
  T* xs = schur_inv<T>(P, guard, s);
  hipLaunchKernelGGL(k_store_p<T>, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, (const T*)xs, y, guard);
}

extern "C" int ipmpde_apply_precond(ipmpde_problem* P, const ipmpde_options* opts, const double* x, double* y,
                                    ipmpde_stream stream) {
  if (!P || !x || !y) return fail(IPMPDE_EINVAL, "NULL argument");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  if (!P->setup_done || P->setup_fp32 != (o.mg_precision == IPMPDE_FP32))
    return fail(IPMPDE_EINVAL, "no Newton setup for this multigrid precision");
  select_mg(P, o);
  const int pt = o.precond == IPMPDE_PT;
  if (o.mg_precision == IPMPDE_FP32) precond_apply_t<float>(P, pt, x, y, 0, S(stream));
  else precond_apply_t<double>(P, pt, x, y, 0, S(stream));
  HIP_TRY(hipGetLastError());
  return IPMPDE_OK;
}

#include "fgmres_host.hip"
#include "timing.hip"
