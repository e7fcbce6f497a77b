// Fused V-cycle level kernels for 3D Poisson with the 7-point stencil, the
// multigrid of S_hat^-1 (Sec. 4.2) for the 3D finite-difference problems:
// one descent launch (nu damped-Jacobi sweeps, residual, full-weighting
// restriction) and one ascent launch (trilinear prolongation, nu sweeps) per
// level, each workgroup on a cube of nodes staged in LDS with a halo of nu
// nodes, which it smooths redundantly instead of exchanging.
//
// Per node the descent stages d = 6/h^2 + m of A + M_hat (m = the level's
// M_hat entry), the ascent w = omega / d, so a sweep is
//   x <- (1 - omega) x + w (b + (sum of the six neighbours) / h^2)
// and the residual is b + (sum of the neighbours) / h^2 - d x.  Nodes of the
// LDS cube outside the grid hold b = d = w = x = 0: the homogeneous Dirichlet
// condition with no tests in the sweeps.  The cube size is a template
// parameter (the launch takes 4^3 coarse nodes per descent cube and 8^3 fine
// nodes per ascent cube, where they fit the LDS); it changes no node's
// arithmetic.
#include "common.h"

namespace ipm {

// Threads per workgroup of the cube kernels (8 waves: a cube's phases are
// latency bound, so more threads per cube shorten them).
constexpr int kP3BS = 512;

__host__ __device__ constexpr int p3_down_width(int nu, int tc) { return 2 * tc + 1 + 2 * nu; }
__host__ __device__ constexpr int p3_up_width(int nu, int tf) { return tf + 2 * nu; }
__host__ __device__ constexpr int p3_up_coarse_width(int nu, int tf) { return p3_up_width(nu, tf) / 2 + 2; }
template <typename T, int NU, int TC>
constexpr size_t p3_down_lds() {
  return 4 * sizeof(T) * (size_t)p3_down_width(NU, TC) * p3_down_width(NU, TC) * p3_down_width(NU, TC);
}
template <typename T, int NU, int TF>
constexpr size_t p3_up_lds() {
  constexpr size_t w = p3_up_width(NU, TF), wc = p3_up_coarse_width(NU, TF);
  return sizeof(T) * (4 * w * w * w + wc * wc * wc);
}

// Cube (tx, ty, tz) of this workgroup from the launch's nx x nx x nx cubes
// (grid x = nx, grid y = nx * nx).  The cubes are dispatched round-robin
// over the 8 XCDs; when their count is a multiple of 8, XCD x takes the x-th
// contiguous eighth (a slab of cube layers), so the halo planes a cube shares
// with its neighbours are mostly in the same L2.  The order changes no
// node's arithmetic.
__device__ __forceinline__ void xcd_cube(int nx, int& tx, int& ty, int& tz) {
  const int nt = nx * nx * nx;
  int t = blockIdx.x + nx * blockIdx.y;
  if ((nt & 7) == 0) t = (t & 7) * (nt >> 3) + (t >> 3);
  tz = t / (nx * nx);
  t -= tz * nx * nx;
  ty = t / nx;
  tx = t - ty * nx;
}

// Sum of the six neighbours of LDS node li in a cube of width W.
template <typename T, int W>
__device__ __forceinline__ T p3_nb(const T* __restrict__ a, int li) {
  return ((a[li - 1] + a[li + 1]) + (a[li - W] + a[li + W])) + (a[li - W * W] + a[li + W * W]);
}

// Descent at level l for a cube of TC^3 coarse nodes: NU sweeps from a zero
// iterate (the first is x = w b), the smoothed iterate of the cube's own
// (2TC)^3 fine nodes into level l's x, the residual and its full-weighting
// restriction into level l + 1's b.  scaled (level 0 only): the right-hand
// side is (O + Theta_y) times level 0's x2 (the first solve's output); it is
// also stored as level 0's b for the ascent.
template <typename T, int NU, int TC>
__global__ void __launch_bounds__(kP3BS) k_mg_down_p3(const Inst* __restrict__ Dp, int l, int scaled, int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int dim = I.dim, pde = I.pde, cl = I.coarse_lev;
  const KrylovCtrl* ctrl = I.ctrl;
  const int N = I.lv[l].N, Nc = I.lv[l + 1].N;
  const double h = I.lv[l].h, omega = I.omega;
  const T* __restrict__ bsrc = (const T*)(scaled ? I.lv[l].x2 : I.lv[l].b);
  const T* __restrict__ mh = (const T*)I.lv[l].mh;
  T* __restrict__ xfine = (T*)I.lv[l].x;
  T* __restrict__ bfine = (T*)I.lv[l].b;
  T* __restrict__ bcoarse = (T*)I.lv[l + 1].b;
  const double* __restrict__ tyv = scaled ? I.ty : nullptr;
  const double* __restrict__ obs = I.obs;
  const int gx = gridDim.x;
  IPM_LOAD_TOGETHER(go, dim, pde, cl, ctrl, N, Nc, h, omega, bsrc, mh, xfine, bfine, bcoarse, tyv, obs, gx);
  if (!go || dim != 3 || pde != 0 || l >= cl) return;
  int tx, ty, tz;
  xcd_cube(gx, tx, ty, tz);
  const int J1 = tx * TC, J2 = ty * TC, J3 = tz * TC;
  // a cube owns fine nodes 2 J ... 2 J + 2 TC - 1 (the last fine node, 2 Nc, has no coarse node of its own)
  if (J1 > Nc || J2 > Nc || J3 > Nc) return;
  constexpr int W = p3_down_width(NU, TC), WW = W * W;
  __shared__ T bs[W * WW], ds[W * WW], xa[W * WW], xb[W * WW];
  const int o1 = 2 * J1 - NU, o2 = 2 * J2 - NU, o3 = 2 * J3 - NU;  // fine coordinates of LDS (0, 0, 0)
  const T ih2 = (T)(1.0 / (h * h)), dg = (T)6 * ih2;
  const T om = (T)omega, om1 = (T)1 - om;
  const int tid = threadIdx.x;
  // the stop flag is requested with the cube's data and tested before the
  // first global store (the staging writes LDS only)
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  for (int k = tid; k < W * WW; k += kP3BS) {
    const int q3 = k / WW, q2 = (k - q3 * WW) / W, q1 = k - q3 * WW - q2 * W;
    const int g1 = o1 + q1, g2 = o2 + q2, g3 = o3 + q3;
    T bv = 0, dv = 0, wv = 0;
    if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N && (unsigned)g3 < (unsigned)N) {
      const int gi = g1 + N * (g2 + N * g3);
      bv = bsrc[gi];
      if (tyv) bv = (T)((obs ? obs[gi] : 1.0) + tyv[gi]) * bv;
      dv = dg + mh[gi];
      wv = omega_over<T>(om, dv);
    }
    bs[k] = bv;
    ds[k] = dv;
    xa[k] = wv * bv;
  }
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  __syncthreads();
  if (tyv) {
    for (int k = tid; k < 8 * TC * TC * TC; k += kP3BS) {
      const int r3 = k / (4 * TC * TC), r2 = (k / (2 * TC)) % (2 * TC), r1 = k % (2 * TC);
      const int g1 = 2 * J1 + r1, g2 = 2 * J2 + r2, g3 = 2 * J3 + r3;
      if (g1 < N && g2 < N && g3 < N) bfine[g1 + N * (g2 + N * g3)] = bs[(NU + r1) + W * (NU + r2) + WW * (NU + r3)];
    }
  }
  T* a = xa;
  T* c = xb;
#pragma unroll
  for (int s = 1; s < NU; ++s) {
    const int w = W - 2 * s;  // the cube shrinks by one node per side per sweep
    for (int k = tid; k < w * w * w; k += kP3BS) {
      const int r3 = k / (w * w), r2 = (k - r3 * w * w) / w, r1 = k - r3 * w * w - r2 * w;
      const int li = (r1 + s) + W * (r2 + s) + WW * (r3 + s);
      const T d = ds[li];
      const T wv = d > (T)0 ? omega_over<T>(om, d) : (T)0;
      c[li] = om1 * a[li] + wv * (bs[li] + ih2 * p3_nb<T, W>(a, li));
    }
    __syncthreads();
    T* t = a; a = c; c = t;
  }
  for (int k = tid; k < 8 * TC * TC * TC; k += kP3BS) {
    const int r3 = k / (4 * TC * TC), r2 = (k / (2 * TC)) % (2 * TC), r1 = k % (2 * TC);
    const int g1 = 2 * J1 + r1, g2 = 2 * J2 + r2, g3 = 2 * J3 + r3;
    if (g1 < N && g2 < N && g3 < N) xfine[g1 + N * (g2 + N * g3)] = a[(NU + r1) + W * (NU + r2) + WW * (NU + r3)];
  }
  {
    constexpr int w = 2 * TC + 1;
    for (int k = tid; k < w * w * w; k += kP3BS) {
      const int r3 = k / (w * w), r2 = (k - r3 * w * w) / w, r1 = k - r3 * w * w - r2 * w;
      const int li = (r1 + NU) + W * (r2 + NU) + WW * (r3 + NU);
      c[li] = bs[li] + ih2 * p3_nb<T, W>(a, li) - ds[li] * a[li];
    }
  }
  __syncthreads();
  const T wt[3] = {(T)0.25, (T)0.5, (T)0.25};
  for (int k = tid; k < TC * TC * TC; k += kP3BS) {
    const int j3 = k / (TC * TC), j2 = (k / TC) % TC, j1 = k % TC;
    const int c1 = J1 + j1, c2 = J2 + j2, c3 = J3 + j3;
    if (c1 < Nc && c2 < Nc && c3 < Nc) {
      const int li = (NU + 2 * j1 + 1) + W * (NU + 2 * j2 + 1) + WW * (NU + 2 * j3 + 1);  // fine node 2c + 1
      T acc = 0;
#pragma unroll
      for (int e3 = -1; e3 <= 1; ++e3)
#pragma unroll
        for (int e2 = -1; e2 <= 1; ++e2)
#pragma unroll
          for (int e1 = -1; e1 <= 1; ++e1)
            acc += wt[e1 + 1] * wt[e2 + 1] * wt[e3 + 1] * c[li + e1 + W * e2 + WW * e3];
      bcoarse[c1 + Nc * (c2 + Nc * c3)] = acc;
    }
  }
}

// Ascent at level l for a cube of TF^3 fine nodes: x = x_pre + P x_c
// (trilinear prolongation from a coarse patch staged in LDS), then NU
// sweeps; writes the cube's own nodes to level l's x2.
template <typename T, int NU, int TF>
__global__ void __launch_bounds__(kP3BS) k_mg_up_p3(const Inst* __restrict__ Dp, int l, int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int dim = I.dim, pde = I.pde, cl = I.coarse_lev;
  const KrylovCtrl* ctrl = I.ctrl;
  const int N = I.lv[l].N, Nc = I.lv[l + 1].N;
  const double h = I.lv[l].h, omega = I.omega;
  const void* xc1 = I.lv[l + 1].x;
  const void* xc2 = I.lv[l + 1].x2;
  const T* __restrict__ xpre = (const T*)I.lv[l].x;
  const T* __restrict__ b = (const T*)I.lv[l].b;
  const T* __restrict__ mh = (const T*)I.lv[l].mh;
  T* __restrict__ xout = (T*)I.lv[l].x2;
  const int gx = gridDim.x;
  IPM_LOAD_TOGETHER(go, dim, pde, cl, ctrl, N, Nc, h, omega, xc1, xc2, xpre, b, mh, xout, gx);
  if (!go || dim != 3 || pde != 0 || l >= cl) return;
  // the coarse iterate: the coarse kernel's output at the coarsest fused level
  const T* __restrict__ xc = (const T*)(l + 1 == cl ? xc1 : xc2);
  int tx, ty, tz;
  xcd_cube(gx, tx, ty, tz);
  if (tx * TF >= N || ty * TF >= N || tz * TF >= N) return;
  constexpr int W = p3_up_width(NU, TF), WW = W * W;
  constexpr int WC = p3_up_coarse_width(NU, TF);
  __shared__ T bs[W * WW], ws[W * WW], xa[W * WW], xb[W * WW], cs[WC * WC * WC];
  const int o1 = tx * TF - NU, o2 = ty * TF - NU, o3 = tz * TF - NU;
  // coarse 1-based index of the patch's first entry per axis: the lower
  // coarse neighbour of the region's first fine node (fine 1-based o + 1)
  const int cb1 = (o1 + 1) >> 1, cb2 = (o2 + 1) >> 1, cb3 = (o3 + 1) >> 1;
  const T ih2 = (T)(1.0 / (h * h)), dg = (T)6 * ih2;
  const T om = (T)omega, om1 = (T)1 - om;
  const int tid = threadIdx.x;
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  for (int k = tid; k < WC * WC * WC; k += kP3BS) {
    const int p3 = k / (WC * WC), p2 = (k / WC) % WC, p1 = k % WC;
    const int c1 = cb1 + p1 - 1, c2 = cb2 + p2 - 1, c3 = cb3 + p3 - 1;  // 0-based coarse node
    cs[k] = ((unsigned)c1 < (unsigned)Nc && (unsigned)c2 < (unsigned)Nc && (unsigned)c3 < (unsigned)Nc)
                ? xc[c1 + Nc * (c2 + Nc * c3)]
                : (T)0;
  }
  for (int k = tid; k < W * WW; k += kP3BS) {
    const int q3 = k / WW, q2 = (k - q3 * WW) / W, q1 = k - q3 * WW - q2 * W;
    const int g1 = o1 + q1, g2 = o2 + q2, g3 = o3 + q3;
    T bv = 0, wv = 0, xv = 0;
    if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N && (unsigned)g3 < (unsigned)N) {
      const int gi = g1 + N * (g2 + N * g3);
      bv = b[gi];
      wv = omega_over<T>(om, dg + mh[gi]);
      xv = xpre[gi];
    }
    bs[k] = bv;
    ws[k] = wv;
    xa[k] = xv;
  }
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  __syncthreads();
  for (int k = tid; k < W * WW; k += kP3BS) {
    const int q3 = k / WW, q2 = (k - q3 * WW) / W, q1 = k - q3 * WW - q2 * W;
    const int g1 = o1 + q1, g2 = o2 + q2, g3 = o3 + q3;
    if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N && (unsigned)g3 < (unsigned)N) {
      // per axis: fine 1-based F even -> coarse F/2 (weight 1); odd -> (F-1)/2 and (F+1)/2 (1/2 each);
      // the patch holds zeros at the boundary's coarse indices 0 and Nc + 1
      const int F1 = g1 + 1, F2 = g2 + 1, F3 = g3 + 1;
      const int lo1 = (F1 >> 1) - cb1, lo2 = (F2 >> 1) - cb2, lo3 = (F3 >> 1) - cb3;
      const int d1 = F1 & 1, d2 = (F2 & 1) * WC, d3 = (F3 & 1) * WC * WC;
      const int pi = lo1 + WC * (lo2 + WC * lo3);
      const T w1 = (F1 & 1) ? (T)0.5 : (T)1, w2 = (F2 & 1) ? (T)0.5 : (T)1, w3 = (F3 & 1) ? (T)0.5 : (T)1;
      // the terms of a non-odd axis repeat the same coarse node with weight 0 (offset 0 and 1 coincide)
      const T e1 = (F1 & 1) ? (T)1 : (T)0, e2 = (F2 & 1) ? (T)1 : (T)0, e3 = (F3 & 1) ? (T)1 : (T)0;
      const T v = w1 * w2 * w3 *
                  (((cs[pi] + e1 * cs[pi + d1]) + e2 * (cs[pi + d2] + e1 * cs[pi + d1 + d2])) +
                   e3 * ((cs[pi + d3] + e1 * cs[pi + d1 + d3]) + e2 * (cs[pi + d2 + d3] + e1 * cs[pi + d1 + d2 + d3])));
      xa[k] += v;
    }
  }
  __syncthreads();
  T* a = xa;
  T* c = xb;
#pragma unroll
  for (int s = 1; s <= NU; ++s) {
    const int w = W - 2 * s;
    for (int k = tid; k < w * w * w; k += kP3BS) {
      const int r3 = k / (w * w), r2 = (k - r3 * w * w) / w, r1 = k - r3 * w * w - r2 * w;
      const int li = (r1 + s) + W * (r2 + s) + WW * (r3 + s);
      c[li] = om1 * a[li] + ws[li] * (bs[li] + ih2 * p3_nb<T, W>(a, li));
    }
    __syncthreads();
    T* t = a; a = c; c = t;
  }
  for (int k = tid; k < TF * TF * TF; k += kP3BS) {
    const int r3 = k / (TF * TF), r2 = (k / TF) % TF, r1 = k % TF;
    const int g1 = tx * TF + r1, g2 = ty * TF + r2, g3 = tz * TF + r3;
    if (g1 < N && g2 < N && g3 < N) xout[g1 + N * (g2 + N * g3)] = a[(NU + r1) + W * (NU + r2) + WW * (NU + r3)];
  }
}

}  // namespace ipm
