// Internal definitions shared by the HIP kernels and the host driver of
// libipmpde.  Everything here is gfx950-only HIP C++.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ipm {

constexpr int kMaxLev = 16;
// Levels of the widest single-workgroup coarse hierarchy (63, 31, 15, 7, 3, 1).
constexpr int kCoarseLevels = 6;
// Width of the 2D Poisson coarse level solved exactly (by its stored inverse).
constexpr int kCoarseInvN = 7;
// Arrays of n per level in the convection-diffusion coarse image.
constexpr int kCoarseCDArrays = 9;
constexpr int kBS = 256;        // threads per block of the elementwise and stencil kernels
constexpr int kCoarseBS = 1024;  // threads of the single-workgroup coarse-grid kernel
constexpr int kTicketGroups = 8;   // sub-counters of the grid reduction ticket
constexpr int kTicketStride = 64;  // unsigned words between sub-counters (one 256-byte line)

// One multigrid level.  Arrays hold T = float or double (the V-cycle precision).
struct Level {
  int N;      // interior points per axis
  int n;      // N^dim
  double h;   // mesh width 1/(N+1)
  float invN; // 1/N, for index arithmetic
  void* x;    // iterate
  void* x2;   // second iterate buffer (Jacobi ping-pong)
  void* b;    // right-hand side
  void* mh;   // diagonal reaction term of the operator being solved with (M_hat restricted to this level)
  void* mhb;  // base of the level's reaction-term slots (n each): 0 M_hat (P_Pi: Sigma), 1 O + Theta_y, 2 zero
};

// Scalars of one Krylov solve, in device memory.
struct KrylovCtrl {
  // MINRES recurrence (Paige-Saunders with a symmetric positive definite preconditioner)
  double gamma_prev, gamma, delta;
  double c_prev, c, s_prev, s;
  double eta, eta0;
  double a1, a2, a3, coef_x, gamma_w;  // coefficients of the pending direction/solution update
  double coef_x_def;   // coefficient of the direction whose solution update was deferred (odd iterations)
  double est;          // |eta| / eta0: relative preconditioned residual estimate
  double trigger;      // estimate at which the host checks the true residual
  double dot_tmp;      // partial result of a split reduction (diagonal blocks)
  double bnorm;        // |b|_2 of the right-hand side
  double rnorm;        // |b - K x|_2 from the last true-residual check
  double rtarget;      // stop when the tracked residual norm falls to this value
  double rtrack;       // tracked residual norm |r_j|_2 (recurrence)
  double rs2, rc;      // r_j = rs2 r_{j-1} + rc v_{j+1} (applied with the next Lanczos step)
  double rfloor;       // |(|K||x| + |b|)|_2 from the last true-residual check (rounding floor scale)
  int iter;            // iterations completed
  int stop;            // 0 running, 1 stopped (converged estimate, breakdown)
  int pending;         // a direction/solution update is pending
  int breakdown;       // 1: preconditioner indefinite or NaN
  int rpend;           // a residual update (rs2, rc) is pending
  int j;               // FGMRES: Arnoldi steps completed in this cycle
  int want_restart;    // 1: the last cycle missed the tolerance; start another from the true residual
  int its_total;       // Krylov iterations over all cycles of this solve
  int failed;          // 1: iteration limit or breakdown
  double relres;       // true relative residual after the last cycle
  // FGMRES (not copied back to the host: everything above hcol is)
  double hcol[64];     // current Hessenberg column
  double g[64];        // rotated residual vector
  double cs[64], sn[64];
  double H[64 * 64];   // Hessenberg (column-major, restart+1 rows)
  double y[64];        // least-squares solution
  double hpass[64];    // coefficients of the current Gram-Schmidt pass
};

// Everything a kernel needs to know about one problem instance.  Kernels
// receive a device array of these and serve instance blockIdx.z, so one
// launch can advance many (unevenly sized) instances; a single problem is a
// batch of one.
struct Inst {
  int dim, N, n, pde;  // pde: 0 Poisson, 1 convection-diffusion, 2 heat (n = N^2 nt space-time nodes),
                       // 3 Poisson with Q1 finite elements (2D)
  int nt;              // heat: time steps (1 otherwise)
  double tau;          // heat: time step
  int has_y;
  int active;          // 0: every kernel skips this instance
  double h, eps, alpha, beta;
  double mu;           // barrier parameter of the current Newton system
  double alpha0;       // fraction-to-boundary factor
  // data (FP64, n values)
  const double* ua;
  const double* ub;
  const double* ya;
  const double* yb;
  const double* yd;
  const double* fhat;
  // iterates
  double *y, *w, *v, *p, *lya, *lyb, *lwa, *lwb, *lva, *lvb;
  // barrier diagonals and preconditioner data
  double *ty, *tw, *tv, *mh;
  // Newton system and Krylov workspace (4n each)
  double *rhs, *X, *Q, *R, *Rt;
  double *V[2], *Z[2], *W[2];
  double *fV, *fZ;      // FGMRES basis (restart + 1 and restart vectors), or null
  int nparts;           // capacity of `partials` in doubles
  // reductions
  double* partials;     // per-block partial results
  unsigned* counter;    // ticket for the last-block pattern (must be 0 between kernels)
  KrylovCtrl* ctrl;
  double* stat;         // small scalar results (measures, step lengths)
  // multigrid
  int nlev;             // number of levels (finest 0)
  int coarse_lev;       // first level handled by the single-workgroup kernel
  int coarse_p2;        // 1: the coarse levels run in the padded 2D Poisson kernel
  void* cpack;          // Poisson 2D: the coarse levels' LDS image (zero iterates, d, 1/d), built per Newton setup
  void* cpackb;         // base of the coarse LDS images of the three reaction-term slots
  int cpack_slot;       // elements between two slots' images
  const double* obs;    // observation weights O (nullptr: the whole domain, O = I)
  const double* eobs;   // Q1: observed-element weights, (N+1)^dim by lower corner (nullptr: all)
  int ppi;              // 1: the partial-observation preconditioner P_Pi (three multigrid operators)
  void* kc_b0;          // k-cycle solves (vcycles > 1): the solve's level-0 right-hand side
  void* kc_s[2];        // and its accumulated iterate (ping-pong)
  int cpack_elems;      // its length in elements of the multigrid type
  int mg_fp32;          // 1: levels hold float
  int nu_pre, nu_post, vcycles;
  double omega;
  Level lv[kMaxLev];
  // copies for the 2D Poisson coarse kernel, so its loads need not wait for
  // coarse_lev: lv[coarse_lev].b, .x and .N, and 1/h^2 of coarse level q
  // (h = 1/(N_q + 1)), computed once on the host
  const void* cb;
  void* cx;
  int cN0;
  double cih2[kCoarseLevels];
  const Level* lvd;     // the same level table in device memory (for loops over levels)
  const Inst* hsteps;   // heat equation: the nt per-time-step multigrid descriptors (device)
};

// ---------------------------------------------------------------------------
// stencils

// Convection-diffusion wind of Sec. 5.2 at x = (x1, x2).
__device__ __forceinline__ void wind(double x1, double x2, double& w1, double& w2) {
  w1 = 2.0 * x2 * (1.0 - x1 * x1);
  w2 = -2.0 * x1 * (1.0 - x2 * x2);
}

// Diagonal entry of the operator at node (i1, i2) (0-based) on a grid of width h.
__device__ __forceinline__ double op_diag(int dim, int pde, double h, double eps, int i1, int i2) {
  if (pde == 0) return 2.0 * dim / (h * h);
  if (pde == 3) return 8.0 / (3.0 * h * h);
  double w1, w2;
  wind((i1 + 1) * h, (i2 + 1) * h, w1, w2);
  return 4.0 * eps / (h * h) + (fabs(w1) + fabs(w2)) / h;
}

// (A x)_i or (A^T x)_i at the node with storage index idx and grid
// coordinates (i1, i2, i3) (0-based); sy, sz are the storage strides of the
// second and third axis.  Off-grid neighbours are 0 (homogeneous Dirichlet;
// inhomogeneous data is folded into f_hat on the host).
template <typename T, bool ABS = false>
__device__ __forceinline__ T ldv(const T* __restrict__ x, int k) {
  return ABS ? (T)fabs(x[k]) : x[k];
}

// ABS = true evaluates A|x| (used for rounding-error bounds).
template <typename T, bool ABS = false>
__device__ __forceinline__ T apply_op_s(const T* __restrict__ x, int idx, int i1, int i2, int i3, int N, int sy, int sz,
                                        int dim, int pde, double h, double eps, bool transpose) {
#define X_(k) ldv<T, ABS>(x, (k))
  if (pde == 0) {
    const T ih2 = (T)(1.0 / (h * h));
    T nb = 0;
    if (i1 > 0) nb += X_(idx - 1);
    if (i1 < N - 1) nb += X_(idx + 1);
    if (i2 > 0) nb += X_(idx - sy);
    if (i2 < N - 1) nb += X_(idx + sy);
    if (dim == 3) {
      if (i3 > 0) nb += X_(idx - sz);
      if (i3 < N - 1) nb += X_(idx + sz);
    }
    return ih2 * ((T)(2 * dim) * X_(idx) - nb);
  }
  if (pde == 3 && dim == 3) {
    // trilinear Q1 stiffness divided by h^3: (8/3 x - 1/6 (the 12 edge
    // neighbours) - 1/12 (the 8 corner neighbours)) / h^2; the 6 face
    // neighbours carry 0.  Symmetric.
    T e = 0, c = 0;
#pragma unroll
    for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
      for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
        for (int o1 = -1; o1 <= 1; ++o1) {
          const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
          if (k < 2) continue;
          if ((unsigned)(i1 + o1) >= (unsigned)N || (unsigned)(i2 + o2) >= (unsigned)N ||
              (unsigned)(i3 + o3) >= (unsigned)N)
            continue;
          const T v = X_(idx + o1 + o2 * sy + o3 * sz);
          if (k == 2) e += v;
          else c += v;
        }
    return (T)(1.0 / (h * h)) * ((T)(8.0 / 3.0) * X_(idx) - (T)(1.0 / 6.0) * e - (T)(1.0 / 12.0) * c);
  }
  if (pde == 3) {
    // Q1 stiffness divided by h^2 (2D): (8 x - the eight neighbours) / (3 h^2), symmetric
    const T ih2 = (T)(1.0 / (3.0 * h * h));
    const bool l = i1 > 0, r = i1 < N - 1, d = i2 > 0, u = i2 < N - 1;
    T nb = 0;
    if (l) nb += X_(idx - 1);
    if (r) nb += X_(idx + 1);
    if (d) {
      nb += X_(idx - sy);
      if (l) nb += X_(idx - sy - 1);
      if (r) nb += X_(idx - sy + 1);
    }
    if (u) {
      nb += X_(idx + sy);
      if (l) nb += X_(idx + sy - 1);
      if (r) nb += X_(idx + sy + 1);
    }
    return ih2 * ((T)8 * X_(idx) - nb);
  }
  // 2D upwind convection-diffusion
  const double ed = eps / (h * h), ih = 1.0 / h;
  double w1, w2;
  const double x1 = (i1 + 1) * h, x2 = (i2 + 1) * h;
  wind(x1, x2, w1, w2);
  double r = (4.0 * ed + (fabs(w1) + fabs(w2)) * ih) * (double)X_(idx);
  if (!transpose) {
    if (i1 > 0) r += (-ed - fmax(w1, 0.0) * ih) * (double)X_(idx - 1);
    if (i1 < N - 1) r += (-ed + fmin(w1, 0.0) * ih) * (double)X_(idx + 1);
    if (i2 > 0) r += (-ed - fmax(w2, 0.0) * ih) * (double)X_(idx - sy);
    if (i2 < N - 1) r += (-ed + fmin(w2, 0.0) * ih) * (double)X_(idx + sy);
  } else {
    // column i of A: the neighbour j's coefficient for node i, with the wind at j
    double a1, a2;
    if (i1 < N - 1) { wind(x1 + h, x2, a1, a2); r += (-ed - fmax(a1, 0.0) * ih) * (double)X_(idx + 1); }
    if (i1 > 0)     { wind(x1 - h, x2, a1, a2); r += (-ed + fmin(a1, 0.0) * ih) * (double)X_(idx - 1); }
    if (i2 < N - 1) { wind(x1, x2 + h, a1, a2); r += (-ed - fmax(a2, 0.0) * ih) * (double)X_(idx + sy); }
    if (i2 > 0)     { wind(x1, x2 - h, a1, a2); r += (-ed + fmin(a2, 0.0) * ih) * (double)X_(idx - sy); }
  }
#undef X_
  return (T)r;
}

template <typename T>
__device__ __forceinline__ T apply_op(const T* __restrict__ x, int idx, int i1, int i2, int i3, int N, int dim,
                                      int pde, double h, double eps, bool transpose) {
  return apply_op_s<T>(x, idx, i1, i2, i3, N, N, N * N, dim, pde, h, eps, transpose);
}

// i = q N + r for 0 <= i < 2^22 via a float reciprocal and one correction.
__device__ __forceinline__ void fast_divmod(int i, int N, int& q, int& r) {
  q = (int)((float)i * __builtin_amdgcn_rcpf((float)N));
  r = i - q * N;
  if (r < 0) { q -= 1; r += N; }
  else if (r >= N) { q += 1; r -= N; }
}

__device__ __forceinline__ void node_coords_small(int idx, int N, int dim, int& i1, int& i2, int& i3) {
  int t;
  fast_divmod(idx, N, t, i1);
  if (dim == 2) { i2 = t; i3 = 0; }
  else fast_divmod(t, N, i3, i2);
}

__device__ __forceinline__ void node_coords(int idx, int N, int dim, int& i1, int& i2, int& i3) {
  i1 = idx % N;
  int t = idx / N;
  if (dim == 2) { i2 = t; i3 = 0; }
  else { i2 = t % N; i3 = t / N; }
}

// Coordinates of node idx of an instance's state vector: for the heat
// equation (time steps stacked after the N^2 nodes of each step) i3 is the
// time step.
__device__ __forceinline__ void inst_coords(int pde, int idx, int N, int dim, int& i1, int& i2, int& i3) {
  node_coords(idx, N, pde == 2 ? 3 : dim, i1, i2, i3);
}

// (A x)_idx or (A^T x)_idx of the instance's state operator.  Heat equation
// (Sec. 4.4, divided by tau with M = I): blocks I/tau + A_h on the diagonal,
// -I/tau on the block subdiagonal, so A couples step i3 to step i3 - 1 and
// A^T to step i3 + 1.
template <typename T>
__device__ __forceinline__ T inst_op(const Inst& I, const T* __restrict__ x, int idx, int i1, int i2, int i3,
                                     bool transpose) {
  if (I.pde != 2) return apply_op<T>(x, idx, i1, i2, i3, I.N, I.dim, I.pde, I.h, I.eps, transpose);
  const double it = 1.0 / I.tau;
  const int nn = I.N * I.N;
  double r = (double)apply_op_s<T>(x, idx, i1, i2, 0, I.N, I.N, nn, 2, 0, I.h, 0.0, false) + it * (double)x[idx];
  if (!transpose) {
    if (i3 > 0) r -= it * (double)x[idx - nn];
  } else {
    if (i3 < I.nt - 1) r -= it * (double)x[idx + nn];
  }
  return (T)r;
}

// Q1 mass matrix divided by h^2 (2D): (16 x + 4 (edge neighbours) + corner
// neighbours) / 36, so that rows sum to 1 away from the boundary.  Its
// diagonal, the D_M of the preconditioners, is 4/9.  ABS: with |x|.
constexpr double kQ1MassDiag = 16.0 / 36.0;
// The trilinear mass divided by h^3 (3D): (64 x + 16 (face) + 4 (edge) +
// (corner neighbours)) / 216; its diagonal is 8/27.
constexpr double kQ1MassDiag3 = 64.0 / 216.0;
__device__ __forceinline__ double q1_mass_diag(int dim) { return dim == 3 ? kQ1MassDiag3 : kQ1MassDiag; }

template <typename T, bool ABS = false>
__device__ __forceinline__ T q1_mass3(const T* __restrict__ x, int idx, int i1, int i2, int i3, int N) {
  const int sy = N, sz = N * N;
  T f = 0, e = 0, c = 0;
#pragma unroll
  for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
    for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
        if (k == 0) continue;
        if ((unsigned)(i1 + o1) >= (unsigned)N || (unsigned)(i2 + o2) >= (unsigned)N ||
            (unsigned)(i3 + o3) >= (unsigned)N)
          continue;
        const T v = ldv<T, ABS>(x, idx + o1 + o2 * sy + o3 * sz);
        if (k == 1) f += v;
        else if (k == 2) e += v;
        else c += v;
      }
  return ((T)64 * ldv<T, ABS>(x, idx) + (T)16 * f + (T)4 * e + c) * (T)(1.0 / 216.0);
}

template <typename T, bool ABS = false>
__device__ __forceinline__ T q1_mass2(const T* __restrict__ x, int idx, int i1, int i2, int N) {
#define X_(k) ldv<T, ABS>(x, (k))
  const bool l = i1 > 0, r = i1 < N - 1, d = i2 > 0, u = i2 < N - 1;
  T e = 0, c = 0;
  if (l) e += X_(idx - 1);
  if (r) e += X_(idx + 1);
  if (d) {
    e += X_(idx - N);
    if (l) c += X_(idx - N - 1);
    if (r) c += X_(idx - N + 1);
  }
  if (u) {
    e += X_(idx + N);
    if (l) c += X_(idx + N - 1);
    if (r) c += X_(idx + N + 1);
  }
#undef X_
  return ((T)16 * ldv<T, ABS>(x, idx) + (T)4 * e + c) * (T)(1.0 / 36.0);
}

// The Q1 mass (divided by the lumped mass h^dim) applied at node idx.
template <typename T, bool ABS = false>
__device__ __forceinline__ T q1_mass(const T* __restrict__ x, int idx, int i1, int i2, int i3, int N, int dim) {
  return dim == 3 ? q1_mass3<T, ABS>(x, idx, i1, i2, i3, N) : q1_mass2<T, ABS>(x, idx, i1, i2, N);
}

// Q1 mass of the observed elements (partial observation, Sec. 4.3) at node
// idx, divided by h^dim: over the 2^dim elements around the node (lower
// corners (i1 + a, i2 + b[, i3 + c]) on the (N+2)^dim grid), the element's
// weight times its mass row, (4, 2, 1) / 36 in 2D and (8, 4, 2, 1) / 216 in
// 3D by the number of coordinates in which the other node differs.
template <typename T, bool ABS = false>
__device__ __forceinline__ T q1_mass_obs(const T* __restrict__ x, int idx, int i1, int i2, int i3, int N, int dim,
                                         const double* __restrict__ ew) {
  const int E = N + 1;
  const int nc = dim == 3 ? 2 : 1;
  T acc = 0;
  for (int c = 0; c < nc; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double we = ew[(i1 + a) + E * ((i2 + b) + (dim == 3 ? E * (i3 + c) : 0))];
        if (we == 0.0) continue;
        T sum = 0;
        for (int s3 = 0; s3 < nc; ++s3)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int s1 = 0; s1 < 2; ++s1) {
              const int o1 = a - 1 + s1, o2 = b - 1 + s2, o3 = dim == 3 ? c - 1 + s3 : 0;
              if ((unsigned)(i1 + o1) >= (unsigned)N || (unsigned)(i2 + o2) >= (unsigned)N ||
                  (dim == 3 && (unsigned)(i3 + o3) >= (unsigned)N))
                continue;
              const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
              const T wk = dim == 3 ? (T)(8 >> k) : (T)(k == 0 ? 4 : (k == 1 ? 2 : 1));
              sum += wk * ldv<T, ABS>(x, idx + o1 + N * (o2 + N * o3));
            }
        acc += (T)we * sum;
      }
  return acc * (T)(dim == 3 ? 1.0 / 216.0 : 1.0 / 36.0);
}

// Diagonal of that mass at node (i1, i2, i3): 4/36 (2D) or 8/216 (3D) times
// the sum of the weights of the elements around the node.
__device__ __forceinline__ double q1_obs_diag(int i1, int i2, int i3, int N, int dim, const double* __restrict__ ew) {
  const int E = N + 1;
  double sw = 0.0;
  for (int c = 0; c < (dim == 3 ? 2 : 1); ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) sw += ew[(i1 + a) + E * ((i2 + b) + (dim == 3 ? E * (i3 + c) : 0))];
  return sw * (dim == 3 ? 8.0 / 216.0 : 4.0 / 36.0);
}

// Tracking mass of a Q1 instance: the observed elements' mass, or the whole mass.
template <typename T, bool ABS = false>
__device__ __forceinline__ T q1_mass_track(const Inst& I, const T* __restrict__ x, int idx, int i1, int i2, int i3) {
  return I.eobs ? q1_mass_obs<T, ABS>(x, idx, i1, i2, i3, I.N, I.dim, I.eobs)
                : q1_mass<T, ABS>(x, idx, i1, i2, i3, I.N, I.dim);
}

// (|A| |x|)_idx (or with |A^T|) for rounding-error bounds.  Every
// off-diagonal entry of the operators is <= 0, so |A||x| = 2 diag |x| - A|x|.
__device__ __forceinline__ double inst_op_abs(const Inst& I, const double* __restrict__ x, int idx, int i1, int i2,
                                              int i3, bool transpose) {
  if (I.pde != 2) {
    const double d = op_diag(I.dim, I.pde, I.h, I.eps, i1, i2);
    return 2.0 * d * fabs(x[idx]) -
           apply_op_s<double, true>(x, idx, i1, i2, i3, I.N, I.N, I.N * I.N, I.dim, I.pde, I.h, I.eps, transpose);
  }
  const double it = 1.0 / I.tau, d = 4.0 / (I.h * I.h);
  const int nn = I.N * I.N;
  double r = 2.0 * d * fabs(x[idx]) - apply_op_s<double, true>(x, idx, i1, i2, 0, I.N, I.N, nn, 2, 0, I.h, 0.0, false);
  r += it * fabs(x[idx]);
  if (!transpose) {
    if (i3 > 0) r += it * fabs(x[idx - nn]);
  } else {
    if (i3 < I.nt - 1) r += it * fabs(x[idx + nn]);
  }
  return r;
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed-order trees, no floating-point atomics)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
// max/min that propagate NaN (so that a broken iterate shows in the measures)
__device__ __forceinline__ double nmax(double a, double b) { return (a != a) ? a : (a > b ? a : b); }
__device__ __forceinline__ double nmin(double a, double b) { return (a != a) ? a : (a < b ? a : b); }
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nmax(v, __shfl_down(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nmin(v, __shfl_down(v, o, 64));
  return v;
}

enum RedOp { kSum = 0, kMax = 1, kMin = 2 };

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
  if (OP == kSum) return a + b;
  if (OP == kMax) return nmax(a, b);
  return nmin(a, b);
}
template <int OP>
__device__ __forceinline__ double red_wave(double v) {
  if (OP == kSum) return wave_sum(v);
  if (OP == kMax) return wave_max(v);
  return wave_min(v);
}
template <int OP>
__device__ __forceinline__ double red_identity() {
  if (OP == kSum) return 0.0;
  if (OP == kMax) return -INFINITY;
  return INFINITY;
}

// Block-wide reduction of K values per thread; result valid in thread 0.
template <int OP, int K, int BS>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* smem /* K * BS/64 */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NW = BS / 64;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = red_wave<OP>(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) smem[k * NW + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = smem[k * NW];
      for (int w = 1; w < NW; ++w) a = red_op<OP>(a, smem[k * NW + w]);
      v[k] = a;
    }
  }
  __syncthreads();
}

// Grid-wide deterministic reduction with the last-block pattern.  Each block
// stores K partials; the block that arrives last combines all partials in
// index order and returns true (thread 0 then holds the results in v).
//
// Cross-block visibility without cache-wide maintenance: the partials are
// written and read with agent-scope relaxed atomic accesses (coherent across
// the XCDs' L2s), and each block waits for its stores to complete before it
// takes its ticket.  An agent-scope fence here would write back and
// invalidate the whole L2 once per block.
template <int OP, int K, int BS>
__device__ __forceinline__ bool grid_reduce(double (&v)[K], double* __restrict__ partials, unsigned* counter,
                                            int nblocks, int bid, double* smem) {
  block_reduce<OP, K, BS>(v, smem);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      __hip_atomic_store(&partials[k * nblocks + bid], v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    // two-level ticket: blocks are spread over kTicketGroups counters (one
    // cache line each) so that no single address takes every block's atomic
    const int g = bid % kTicketGroups;
    const int gsize = (nblocks - g + kTicketGroups - 1) / kTicketGroups;
    const int ngroups = nblocks < kTicketGroups ? nblocks : kTicketGroups;
    unsigned* cg = counter + kTicketStride * (1 + g);
    int last = 0;
    const unsigned t1 = __hip_atomic_fetch_add(cg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t1 == (unsigned)(gsize - 1)) {
      __hip_atomic_store(cg, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
      const unsigned t0 = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = (t0 == (unsigned)(ngroups - 1));
    }
    is_last = last;
  }
  __syncthreads();
  if (!is_last) return false;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc[k] = red_identity<OP>();
    for (int b = threadIdx.x; b < nblocks; b += BS)
      acc[k] = red_op<OP>(acc[k], __hip_atomic_load(&partials[k * nblocks + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  block_reduce<OP, K, BS>(acc, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = acc[k];
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Level-0 output array of the V-cycle: level 0's x when the whole hierarchy
// runs in the single-workgroup kernel, else x (outsel = 0) or x2 (outsel = 1).
template <typename T>
__device__ __forceinline__ const T* mg_out(const Inst& I, int outsel) {
  return (const T*)((I.coarse_lev == 0 || !outsel) ? I.lv[0].x : I.lv[0].x2);
}


// Observation weight of node i (the (1,1) block is O + Theta_y).
__device__ __forceinline__ double obs_w(const Inst& I, int i) { return I.obs ? I.obs[i] : 1.0; }

// Node of this thread in a stencil kernel.  The workgroups of a launch are
// dispatched round-robin over the 8 XCDs, each with its own L2; the hardware
// block index is remapped so that XCD x sweeps the x-th contiguous eighth of
// the instance's blocks, which keeps the stencil's rows above and below a
// block mostly in the same L2 instead of fetching them again.  The instance's
// block count is rounded up to a multiple of 8, as every launch grid is
// (nodes >= n mean "no node").  The map depends only on n, so an instance
// computes the same partial sums alone and in a batch.
__device__ __forceinline__ int xcd_node(int n) {
  const int nb = ((n + kBS - 1) / kBS + 7) & ~7;
  const int b = blockIdx.x;
  if (b >= nb) return n;
  return ((b & 7) * (nb >> 3) + (b >> 3)) * kBS + threadIdx.x;
}

// Descriptor fields loaded together.  A kernel starts with cold caches, and
// each load the compiler places behind a branch on an earlier one (active?
// this level? stopped?) adds a memory round trip before the first byte of
// data is requested: five of them cost several microseconds, more than the
// work of a small launch.  IPM_LOAD_TOGETHER(gate, a, b, ...) makes the
// uniform values a, b, ... inputs of one empty asm statement that also
// rewrites gate, so every load producing them is issued before it and waited
// for once, and the branches that test gate come after.  Up to 28 values.
#define IPM_S_(a) "s"(a)
#define IPM_SN_1(a) IPM_S_(a)
#define IPM_SN_2(a, ...) IPM_S_(a), IPM_SN_1(__VA_ARGS__)
#define IPM_SN_3(a, ...) IPM_S_(a), IPM_SN_2(__VA_ARGS__)
#define IPM_SN_4(a, ...) IPM_S_(a), IPM_SN_3(__VA_ARGS__)
#define IPM_SN_5(a, ...) IPM_S_(a), IPM_SN_4(__VA_ARGS__)
#define IPM_SN_6(a, ...) IPM_S_(a), IPM_SN_5(__VA_ARGS__)
#define IPM_SN_7(a, ...) IPM_S_(a), IPM_SN_6(__VA_ARGS__)
#define IPM_SN_8(a, ...) IPM_S_(a), IPM_SN_7(__VA_ARGS__)
#define IPM_SN_9(a, ...) IPM_S_(a), IPM_SN_8(__VA_ARGS__)
#define IPM_SN_10(a, ...) IPM_S_(a), IPM_SN_9(__VA_ARGS__)
#define IPM_SN_11(a, ...) IPM_S_(a), IPM_SN_10(__VA_ARGS__)
#define IPM_SN_12(a, ...) IPM_S_(a), IPM_SN_11(__VA_ARGS__)
#define IPM_SN_13(a, ...) IPM_S_(a), IPM_SN_12(__VA_ARGS__)
#define IPM_SN_14(a, ...) IPM_S_(a), IPM_SN_13(__VA_ARGS__)
#define IPM_SN_15(a, ...) IPM_S_(a), IPM_SN_14(__VA_ARGS__)
#define IPM_SN_16(a, ...) IPM_S_(a), IPM_SN_15(__VA_ARGS__)
#define IPM_SN_17(a, ...) IPM_S_(a), IPM_SN_16(__VA_ARGS__)
#define IPM_SN_18(a, ...) IPM_S_(a), IPM_SN_17(__VA_ARGS__)
#define IPM_SN_19(a, ...) IPM_S_(a), IPM_SN_18(__VA_ARGS__)
#define IPM_SN_20(a, ...) IPM_S_(a), IPM_SN_19(__VA_ARGS__)
#define IPM_SN_21(a, ...) IPM_S_(a), IPM_SN_20(__VA_ARGS__)
#define IPM_SN_22(a, ...) IPM_S_(a), IPM_SN_21(__VA_ARGS__)
#define IPM_SN_23(a, ...) IPM_S_(a), IPM_SN_22(__VA_ARGS__)
#define IPM_SN_24(a, ...) IPM_S_(a), IPM_SN_23(__VA_ARGS__)
#define IPM_SN_25(a, ...) IPM_S_(a), IPM_SN_24(__VA_ARGS__)
#define IPM_SN_26(a, ...) IPM_S_(a), IPM_SN_25(__VA_ARGS__)
#define IPM_SN_27(a, ...) IPM_S_(a), IPM_SN_26(__VA_ARGS__)
#define IPM_SN_28(a, ...) IPM_S_(a), IPM_SN_27(__VA_ARGS__)
#define IPM_NARGS_(_1, _2, _3, _4, _5, _6, _7, _8, _9, _10, _11, _12, _13, _14, _15, _16, _17, _18, _19, _20, _21, \
                   _22, _23, _24, _25, _26, _27, _28, N, ...)                                                      \
  N
#define IPM_NARGS(...)                                                                                            \
  IPM_NARGS_(__VA_ARGS__, 28, 27, 26, 25, 24, 23, 22, 21, 20, 19, 18, 17, 16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, \
             4, 3, 2, 1, 0)
#define IPM_CAT_(a, b) a##b
#define IPM_CAT(a, b) IPM_CAT_(a, b)
#define IPM_LOAD_TOGETHER(gate, ...) \
  asm volatile("" : "+s"(gate) : IPM_CAT(IPM_SN_, IPM_NARGS(__VA_ARGS__))(__VA_ARGS__))

// Start of every kernel: the instance of this block, skipped when inactive.
#define INST_BEGIN                         \
  const Inst& I = Dp[blockIdx.z];          \
  if (!I.active) return;

}  // namespace ipm
