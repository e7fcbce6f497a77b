// Geometric multigrid for the Schur-complement approximation of Sec. 4.2:
// S_hat^-1 = (A + M_hat)^-T (I + Theta_y) (A + M_hat)^-1, each inverse
// replaced by V-cycles (the paper uses algebraic multigrid; this is the
// geometric counterpart on the nested grids N_l = (N_{l-1} - 1) / 2).
//
// Components: damped Jacobi smoothing on A_l + diag(M_hat_l), residual with
// full-weighting restriction, bilinear/trilinear prolongation, and one
// workgroup that runs every level from `coarse_lev` down to the single-node
// grid inside LDS.  With equal pre/post sweep counts, R = 2^-d P^T and the
// transposed stencil on the transposed solve, the V-cycle for (A+M_hat)^T is
// the exact adjoint of the one for A + M_hat, so the composed Schur block is
// symmetric positive definite as MINRES requires.
#include "common.h"

namespace ipm {

// ---------------------------------------------------------------- per-node pieces

// Jacobi update at node i of level (N, h): x_out = x_in + omega (b - (A + mh) x_in) / d,
// or omega b / d from a zero iterate.
template <typename T>
__device__ __forceinline__ T jacobi_node(const T* __restrict__ xin, const T* __restrict__ b, const T* __restrict__ mh,
                                         int i, int N, int dim, int pde, double h, double eps, double omega,
                                         bool first, bool transpose) {
  int i1, i2, i3;
  node_coords(i, N, dim, i1, i2, i3);
  const T m = mh[i];
  const T d = (T)op_diag(dim, pde, h, eps, i1, i2) + m;
  if (first) return (T)omega * b[i] / d;
  const T xi = xin[i];
  const T Ax = apply_op<T>(xin, i, i1, i2, i3, N, dim, pde, h, eps, transpose) + m * xi;
  return xi + (T)omega * (b[i] - Ax) / d;
}

// Residual b - (A + mh) x at fine node (i1, i2, i3).
template <typename T>
__device__ __forceinline__ T resid_node(const T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ mh,
                                        int i1, int i2, int i3, int N, int dim, int pde, double h, double eps,
                                        bool transpose) {
  const int i = i1 + N * (i2 + N * i3);
  return b[i] - (apply_op<T>(x, i, i1, i2, i3, N, dim, pde, h, eps, transpose) + mh[i] * x[i]);
}

// Full-weighting restriction of the residual onto coarse node ic.
template <typename T>
__device__ __forceinline__ T restrict_resid_node(const T* __restrict__ x, const T* __restrict__ b,
                                                 const T* __restrict__ mh, int ic, int Nf, int Nc, int dim, int pde,
                                                 double hf, double eps, bool transpose) {
  int j1, j2, j3;
  node_coords(ic, Nc, dim, j1, j2, j3);
  const int f1 = 2 * j1 + 1, f2 = 2 * j2 + 1, f3 = 2 * j3 + 1;
  const T wt[3] = {(T)0.25, (T)0.5, (T)0.25};
  T acc = 0;
  if (dim == 2) {
    for (int bb = -1; bb <= 1; ++bb)
      for (int a = -1; a <= 1; ++a)
        acc += wt[a + 1] * wt[bb + 1] * resid_node<T>(x, b, mh, f1 + a, f2 + bb, 0, Nf, dim, pde, hf, eps, transpose);
  } else {
    for (int c = -1; c <= 1; ++c)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a)
          acc += wt[a + 1] * wt[bb + 1] * wt[c + 1] *
                 resid_node<T>(x, b, mh, f1 + a, f2 + bb, f3 + c, Nf, dim, pde, hf, eps, transpose);
  }
  return acc;
}

// Bilinear/trilinear interpolation of the coarse correction at fine node i.
template <typename T>
__device__ __forceinline__ T prolong_node(const T* __restrict__ xc, int i, int Nf, int Nc, int dim) {
  int i1, i2, i3;
  node_coords(i, Nf, dim, i1, i2, i3);
  // per axis: fine 1-based index F; even -> coarse F/2 (weight 1); odd -> (F-1)/2, (F+1)/2 (1/2 each);
  // coarse 1-based indices 0 and Nc+1 are boundary (zero).
  int lo[3], hi[3];
  const int F[3] = {i1 + 1, i2 + 1, i3 + 1};
  for (int a = 0; a < 3; ++a) {
    if (F[a] & 1) { lo[a] = (F[a] - 1) >> 1; hi[a] = (F[a] + 1) >> 1; }
    else { lo[a] = hi[a] = F[a] >> 1; }
  }
  T acc = 0;
  const int nax = dim;
  const int c3lo = nax == 3 ? 0 : 0, c3hi = nax == 3 ? 1 : 0;
  for (int c = c3lo; c <= c3hi; ++c) {
    const int k3 = c == 0 ? lo[2] : hi[2];
    if (nax == 3 && (k3 < 1 || k3 > Nc)) continue;
    if (nax == 3 && c == 1 && hi[2] == lo[2]) continue;
    for (int bb = 0; bb <= 1; ++bb) {
      const int k2 = bb == 0 ? lo[1] : hi[1];
      if (k2 < 1 || k2 > Nc) continue;
      if (bb == 1 && hi[1] == lo[1]) continue;
      for (int a = 0; a <= 1; ++a) {
        const int k1 = a == 0 ? lo[0] : hi[0];
        if (k1 < 1 || k1 > Nc) continue;
        if (a == 1 && hi[0] == lo[0]) continue;
        T wgt = (lo[0] == hi[0] ? (T)1 : (T)0.5) * (lo[1] == hi[1] ? (T)1 : (T)0.5);
        if (nax == 3) wgt *= (lo[2] == hi[2] ? (T)1 : (T)0.5);
        const int kc = (k1 - 1) + Nc * ((k2 - 1) + (nax == 3 ? Nc * (k3 - 1) : 0));
        acc += wgt * xc[kc];
      }
    }
  }
  return acc;
}

// ---------------------------------------------------------------- grid-wide kernels

template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_jacobi(Inst I, int l, const T* __restrict__ xin, T* __restrict__ xout,
                                                   int first, int transpose, int guard) {
  if (guard && I.ctrl->stop) return;
  const Level& L = I.lv[l];
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= L.n) return;
  xout[i] = jacobi_node<T>(xin, (const T*)L.b, (const T*)L.mh, i, L.N, I.dim, I.pde, L.h, I.eps, I.omega,
                           first != 0, transpose != 0);
}

template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_restrict(Inst I, int l, const T* __restrict__ x, int transpose, int guard) {
  if (guard && I.ctrl->stop) return;
  const Level& F = I.lv[l];
  const Level& C = I.lv[l + 1];
  const int ic = blockIdx.x * kBS + threadIdx.x;
  if (ic >= C.n) return;
  ((T*)C.b)[ic] = restrict_resid_node<T>(x, (const T*)F.b, (const T*)F.mh, ic, F.N, C.N, I.dim, I.pde, F.h, I.eps,
                                         transpose != 0);
}

template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_prolong(Inst I, int l, T* __restrict__ x, const T* __restrict__ xc, int guard) {
  if (guard && I.ctrl->stop) return;
  const Level& F = I.lv[l];
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= F.n) return;
  x[i] += prolong_node<T>(xc, i, F.N, I.lv[l + 1].N, I.dim);
}

// All levels l >= coarse_lev in one workgroup: V-cycle from b at coarse_lev
// (global) to x at coarse_lev (global), every level's x, x2 and b in LDS.
// Offsets are recomputed from the level sizes (no per-level pointer tables,
// which would live in scratch memory); bit l of `alt` records whether level
// l's iterate currently sits in x2.
template <typename T>
__device__ __forceinline__ T* lds_level(T* lds, const Level* __restrict__ LV, int cl, int l, int which) {
  int off = 0;
  for (int m = cl; m < l; ++m) off += 3 * LV[m].n;
  return lds + off + which * LV[l].n;
}

template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_mg_coarse(Inst I, int transpose, int guard) {
  if (guard && I.ctrl->stop) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = (T*)lds_raw;
  const int cl = I.coarse_lev, L = I.nlev;
  const Level* __restrict__ LV = I.lvd;
  const bool tr = transpose != 0;
  const int tid = threadIdx.x;
  unsigned alt = 0;
  {
    const T* bg = (const T*)LV[cl].b;
    T* B = lds_level(lds, LV, cl, cl, 2);
    for (int i = tid; i < LV[cl].n; i += kCoarseBS) B[i] = bg[i];
  }
  __syncthreads();
  // descend
  for (int l = cl; l < L - 1; ++l) {
    const Level& Lv = LV[l];
    const T* mh = (const T*)Lv.mh;
    T* a = lds_level(lds, LV, cl, l, 0);
    T* c = lds_level(lds, LV, cl, l, 1);
    const T* B = lds_level(lds, LV, cl, l, 2);
    for (int s = 0; s < I.nu_pre; ++s) {
      for (int i = tid; i < Lv.n; i += kCoarseBS)
        c[i] = jacobi_node<T>(a, B, mh, i, Lv.N, I.dim, I.pde, Lv.h, I.eps, I.omega, s == 0, tr);
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
    const Level& Cv = LV[l + 1];
    T* Bc = lds_level(lds, LV, cl, l + 1, 2);
    for (int ic = tid; ic < Cv.n; ic += kCoarseBS)
      Bc[ic] = restrict_resid_node<T>(a, B, mh, ic, Lv.N, Cv.N, I.dim, I.pde, Lv.h, I.eps, tr);
    __syncthreads();
  }
  // coarsest grid (a single node): exact solve
  {
    const Level& Lv = LV[L - 1];
    const T* mh = (const T*)Lv.mh;
    T* X = lds_level(lds, LV, cl, L - 1, 0);
    const T* B = lds_level(lds, LV, cl, L - 1, 2);
    for (int i = tid; i < Lv.n; i += kCoarseBS) {
      int i1, i2, i3;
      node_coords(i, Lv.N, I.dim, i1, i2, i3);
      X[i] = B[i] / ((T)op_diag(I.dim, I.pde, Lv.h, I.eps, i1, i2) + mh[i]);
    }
    __syncthreads();
  }
  // ascend
  for (int l = L - 2; l >= cl; --l) {
    const Level& Lv = LV[l];
    const T* mh = (const T*)Lv.mh;
    const int ca = (alt >> l) & 1u;
    T* a = lds_level(lds, LV, cl, l, ca);
    T* c = lds_level(lds, LV, cl, l, 1 - ca);
    const T* B = lds_level(lds, LV, cl, l, 2);
    const T* xc = lds_level(lds, LV, cl, l + 1, (alt >> (l + 1)) & 1u);
    const int Nc = LV[l + 1].N;
    for (int i = tid; i < Lv.n; i += kCoarseBS) a[i] += prolong_node<T>(xc, i, Lv.N, Nc, I.dim);
    __syncthreads();
    for (int s = 0; s < I.nu_post; ++s) {
      for (int i = tid; i < Lv.n; i += kCoarseBS)
        c[i] = jacobi_node<T>(a, B, mh, i, Lv.N, I.dim, I.pde, Lv.h, I.eps, I.omega, false, tr);
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
  }
  T* xg = (T*)LV[cl].x;
  const T* xs = lds_level(lds, LV, cl, cl, (alt >> cl) & 1u);
  for (int i = tid; i < LV[cl].n; i += kCoarseBS) xg[i] = xs[i];
}

// b_0 = (1 + Theta_y) x between the two solves of S_hat^-1.
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_scale_ty(Inst I, const T* __restrict__ x, int guard) {
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  ((T*)I.lv[0].b)[i] = (T)(1.0 + I.ty[i]) * x[i];
}

#define IPM_MG_INST(T)                                                            \
  template __global__ void k_mg_jacobi<T>(Inst, int, const T*, T*, int, int, int); \
  template __global__ void k_mg_restrict<T>(Inst, int, const T*, int, int);        \
  template __global__ void k_mg_prolong<T>(Inst, int, T*, const T*, int);          \
  template __global__ void k_mg_coarse<T>(Inst, int, int);                         \
  template __global__ void k_mg_scale_ty<T>(Inst, const T*, int);
IPM_MG_INST(float)
IPM_MG_INST(double)
#undef IPM_MG_INST

}  // namespace ipm
