// Fused V-cycle level kernels for 2D Poisson (constant 5-point stencil, ST =
// 5, or the Q1 nine-point stiffness divided by h^2, ST = 9), the multigrid of
// S_hat^-1 (Sec. 4.2) for the Poisson problems.
//
// Per node the kernels stage in LDS the diagonal d = 4/h^2 + m (ST = 5) or
// 8/(3 h^2) + m (ST = 9) of A + M_hat (m = the level's M_hat entry; the
// descent, which also needs d for the residual) or w = omega / d (the
// ascent), so a damped-Jacobi sweep is
//   x <- (1 - omega) x + w (b + s (sum of the neighbours)),
// s = 1/h^2 over the four neighbours or 1/(3 h^2) over the eight, and the
// residual is b + s (sum of the neighbours) - d x.  Nodes of the
// LDS region outside the grid hold b = d = w = x = 0, which keeps the
// homogeneous Dirichlet condition with no tests in the sweeps.  The tile size
// is a template parameter (a launch choice); it changes no node's arithmetic,
// only how much halo is recomputed.
#include "common.h"

namespace ipm {

__host__ __device__ constexpr int p2_down_width(int nu, int tc) { return 2 * tc + 1 + 2 * nu; }
__host__ __device__ constexpr int p2_up_width(int nu, int tf) { return tf + 2 * nu; }
__host__ __device__ constexpr int p2_up_coarse_width(int nu, int tf) { return p2_up_width(nu, tf) / 2 + 2; }
template <typename T, int NU, int TC>
constexpr size_t p2_down_lds() { return 4 * sizeof(T) * p2_down_width(NU, TC) * p2_down_width(NU, TC); }
template <typename T, int NU, int TF>
constexpr size_t p2_up_lds() {
  return sizeof(T) * (4 * p2_up_width(NU, TF) * p2_up_width(NU, TF) +
                      p2_up_coarse_width(NU, TF) * p2_up_coarse_width(NU, TF));
}
constexpr size_t kStaticLdsMax = 65536;

// Tiles of this workgroup: a run of tpw consecutive tiles (row-major over the
// nt x nt tiles of the level) starting at tile w tpw, w the workgroup index.
// The workgroups of a launch are dispatched round-robin over the 8 XCDs;
// when their count is a multiple of 8, XCD x takes the x-th contiguous eighth
// of them (a band of tile rows), so the halo rows a tile shares with the
// tiles above and below are mostly in the same L2, and consecutive tiles of a
// run share their halo columns.  While a tile is smoothed in LDS the next
// tile's data are already on their way into registers.  The order of the
// tiles changes no node's arithmetic.
__device__ __forceinline__ void tile_run(int nwg, int tpw, int ntiles, int& t0, int& t1) {
  int w = blockIdx.x;
  if ((nwg & 7) == 0) w = (w & 7) * (nwg >> 3) + (w >> 3);
  t0 = w * tpw;
  t1 = t0 + tpw < ntiles ? t0 + tpw : ntiles;
}

// Neighbour sum of LDS node li (row pitch W) scaled by s, for stencil ST.
template <typename T, int ST>
__device__ __forceinline__ T p2l_nb(const T* __restrict__ a, int li, int W, T s) {
  if constexpr (ST == 5) {
    return s * ((a[li - 1] + a[li + 1]) + (a[li - W] + a[li + W]));
  } else {
    return s * (((a[li - 1] + a[li + 1]) + (a[li - W] + a[li + W])) +
                ((a[li - W - 1] + a[li - W + 1]) + (a[li + W - 1] + a[li + W + 1])));
  }
}
// The stencil's diagonal and neighbour scale at mesh width h.
template <typename T, int ST>
__device__ __forceinline__ T p2l_diag(double h) { return ST == 5 ? (T)4 * (T)(1.0 / (h * h)) : (T)(8.0 / (3.0 * h * h)); }
template <typename T, int ST>
__device__ __forceinline__ T p2l_scale(double h) { return ST == 5 ? (T)(1.0 / (h * h)) : (T)(1.0 / (3.0 * h * h)); }

// omega / d in the multigrid type (a hardware reciprocal in FP32).
template <typename T>
__device__ __forceinline__ T omega_over(T om, T d) { return om / d; }
template <>
__device__ __forceinline__ float omega_over<float>(float om, float d) { return om * __builtin_amdgcn_rcpf(d); }

// Descent at level l for a tile of TC x TC coarse nodes: NU sweeps from a
// zero iterate (the first is x = w b), the smoothed iterate of the tile's own
// 2TC x 2TC fine nodes, the residual and its full-weighting restriction.
// scaled (level 0 only): the right-hand side is (1 + Theta_y) times level 0's
// x2 (the first solve's output); it is also stored as level 0's b for the
// ascent.
template <typename T, int NU, int TC, int ST = 5, int BS = kBS>
__global__ void __launch_bounds__(BS) k_mg_down_p2(const Inst* __restrict__ Dp, int l, int scaled, int guard, int nt,
                                                    int tpw) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int kind = I.coarse_p2, cl = I.coarse_lev;
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
  IPM_LOAD_TOGETHER(go, kind, cl, ctrl, N, Nc, h, omega, bsrc, mh, xfine, bfine, bcoarse, tyv, obs, gx);
  if (!go || kind != (ST == 5 ? 1 : 2) || l >= cl) return;
  int t0, t1;
  tile_run(gx, tpw, nt * nt, t0, t1);
  if (t0 >= t1) return;
  constexpr int W = p2_down_width(NU, TC);
  constexpr int R = (W * W + BS - 1) / BS;  // staged nodes per thread
  __shared__ T bs[W * W], ds[W * W], xa[W * W], xb[W * W];
  const T ih2 = p2l_scale<T, ST>(h), dg = p2l_diag<T, ST>(h);
  const T om = (T)omega, om1 = (T)1 - om;
  const int tid = threadIdx.x;
  // the stop flag is requested with the first tile's data and tested before
  // the first global store (the staging writes LDS only)
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  // the tile's right-hand side (and Theta_y, O when scaled) and M_hat in registers
  T rb[R], rm[R];
  double rt[R], ro[R];
  auto fetch = [&](int t) {
    const int o1 = 2 * (t % nt) * TC - NU, o2 = 2 * (t / nt) * TC - NU;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = tid + r * BS;
      const int q2 = k / W, q1 = k - q2 * W;
      const int g1 = o1 + q1, g2 = o2 + q2;
      if (k < W * W && (unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
        const int gi = g1 + N * g2;
        rb[r] = bsrc[gi];
        rm[r] = mh[gi];
        if (tyv) {
          rt[r] = tyv[gi];
          ro[r] = obs ? obs[gi] : 1.0;
        }
      }
    }
  };
  fetch(t0);
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  for (int t = t0; t < t1; ++t) {
    const int J1 = (t % nt) * TC, J2 = (t / nt) * TC;
    const bool live = J1 < Nc && J2 < Nc;  // uniform: the tile lies in this instance's grid
    if (live) {
      const int o1 = 2 * J1 - NU, o2 = 2 * J2 - NU;  // fine coordinates of LDS (0, 0)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = tid + r * BS;
        if (k < W * W) {
          const int q2 = k / W, q1 = k - q2 * W;
          const int g1 = o1 + q1, g2 = o2 + q2;
          T bv = 0, dv = 0, wv = 0;
          if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
            bv = rb[r];
            if (tyv) bv = (T)(ro[r] + rt[r]) * bv;
            dv = dg + rm[r];
            wv = omega_over<T>(om, dv);
          }
          bs[k] = bv;
          ds[k] = dv;
          xa[k] = wv * bv;
        }
      }
    }
    __syncthreads();
    if (t + 1 < t1) fetch(t + 1);
    if (live) {
      if (tyv) {
        for (int k = tid; k < 4 * TC * TC; k += BS) {
          const int r2 = k / (2 * TC), r1 = k - r2 * (2 * TC);
          const int g1 = 2 * J1 + r1, g2 = 2 * J2 + r2;
          if (g1 < N && g2 < N) bfine[g1 + N * g2] = bs[(NU + r1) + W * (NU + r2)];
        }
      }
      T* a = xa;
      T* c = xb;
#pragma unroll
      for (int s = 1; s < NU; ++s) {
        const int w = W - 2 * s;  // the region shrinks by one node per sweep
        for (int k = tid; k < w * w; k += BS) {
          const int r2 = k / w, r1 = k - r2 * w;
          const int li = (r1 + s) + W * (r2 + s);
          const T d = ds[li];
          const T wv = d > (T)0 ? omega_over<T>(om, d) : (T)0;
          c[li] = om1 * a[li] + wv * (bs[li] + p2l_nb<T, ST>(a, li, W, ih2));
        }
        __syncthreads();
        T* tmp = a; a = c; c = tmp;
      }
      for (int k = tid; k < 4 * TC * TC; k += BS) {
        const int r2 = k / (2 * TC), r1 = k - r2 * (2 * TC);
        const int g1 = 2 * J1 + r1, g2 = 2 * J2 + r2;
        if (g1 < N && g2 < N) xfine[g1 + N * g2] = a[(NU + r1) + W * (NU + r2)];
      }
      {
        constexpr int w = 2 * TC + 1;
        for (int k = tid; k < w * w; k += BS) {
          const int r2 = k / w, r1 = k - r2 * w;
          const int li = (r1 + NU) + W * (r2 + NU);
          c[li] = bs[li] + p2l_nb<T, ST>(a, li, W, ih2) - ds[li] * a[li];
        }
      }
      __syncthreads();
      for (int k = tid; k < TC * TC; k += BS) {
        const int j2 = k / TC, j1 = k - j2 * TC;
        const int c1 = J1 + j1, c2 = J2 + j2;
        if (c1 < Nc && c2 < Nc) {
          const int li = (NU + 2 * j1 + 1) + W * (NU + 2 * j2 + 1);  // fine node 2c + 1
          const T v = (T)0.25 * c[li] + (T)0.125 * ((c[li - 1] + c[li + 1]) + (c[li - W] + c[li + W])) +
                      (T)0.0625 * ((c[li - 1 - W] + c[li + 1 - W]) + (c[li - 1 + W] + c[li + 1 + W]));
          bcoarse[c1 + Nc * c2] = v;
        }
      }
    }
    __syncthreads();  // the next tile's staging overwrites the LDS
  }
}

// Ascent at level l for a tile of TF x TF fine nodes: x = x_pre + P x_c
// (bilinear prolongation from a coarse patch staged in LDS), then NU sweeps;
// writes the tile's own nodes to level l's x2.
template <typename T, int NU, int TF, int ST = 5, int BS = kBS>
__global__ void __launch_bounds__(BS) k_mg_up_p2(const Inst* __restrict__ Dp, int l, int guard, int nt, int tpw) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int kind = I.coarse_p2, cl = I.coarse_lev;
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
  IPM_LOAD_TOGETHER(go, kind, cl, ctrl, N, Nc, h, omega, xc1, xc2, xpre, b, mh, xout, gx);
  if (!go || kind != (ST == 5 ? 1 : 2) || l >= cl) return;
  // the coarse iterate: the coarse kernel's output at the coarsest fused level
  const T* __restrict__ xc = (const T*)(l + 1 == cl ? xc1 : xc2);
  int t0, t1;
  tile_run(gx, tpw, nt * nt, t0, t1);
  if (t0 >= t1) return;
  constexpr int W = p2_up_width(NU, TF);
  constexpr int WC = p2_up_coarse_width(NU, TF);
  constexpr int R = (W * W + BS - 1) / BS, RC = (WC * WC + BS - 1) / BS;  // staged nodes per thread
  __shared__ T bs[W * W], ws[W * W], xa[W * W], xb[W * W], cs[WC * WC];
  const T ih2 = p2l_scale<T, ST>(h), dg = p2l_diag<T, ST>(h);
  const T om = (T)omega, om1 = (T)1 - om;
  const int tid = threadIdx.x;
  // the stop flag is requested with the first tile's data and tested before
  // the first global store (the staging writes LDS only)
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  // the tile's coarse patch, right-hand side, M_hat and pre-smoothed iterate in registers
  T rc[RC], rb[R], rm[R], rx[R];
  auto fetch = [&](int t) {
    const int o1 = (t % nt) * TF - NU, o2 = (t / nt) * TF - NU;
    // coarse 1-based index of the patch's first column/row: the lower coarse
    // neighbour of the region's first fine node (fine 1-based index o + 1)
    const int cb1 = (o1 + 1) >> 1, cb2 = (o2 + 1) >> 1;
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int k = tid + r * BS;
      const int p2 = k / WC, p1 = k - p2 * WC;
      const int c1 = cb1 + p1 - 1, c2 = cb2 + p2 - 1;  // 0-based coarse node
      rc[r] = (k < WC * WC && (unsigned)c1 < (unsigned)Nc && (unsigned)c2 < (unsigned)Nc) ? xc[c1 + Nc * c2] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = tid + r * BS;
      const int q2 = k / W, q1 = k - q2 * W;
      const int g1 = o1 + q1, g2 = o2 + q2;
      if (k < W * W && (unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
        const int gi = g1 + N * g2;
        rb[r] = b[gi];
        rm[r] = mh[gi];
        rx[r] = xpre[gi];
      }
    }
  };
  fetch(t0);
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  for (int t = t0; t < t1; ++t) {
    const int tx = t % nt, ty = t / nt;
    const bool live = tx * TF < N && ty * TF < N;  // uniform: the tile lies in this instance's grid
    const int o1 = tx * TF - NU, o2 = ty * TF - NU;
    const int cb1 = (o1 + 1) >> 1, cb2 = (o2 + 1) >> 1;
    if (live) {
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const int k = tid + r * BS;
        if (k < WC * WC) cs[k] = rc[r];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = tid + r * BS;
        if (k < W * W) {
          const int q2 = k / W, q1 = k - q2 * W;
          const int g1 = o1 + q1, g2 = o2 + q2;
          T bv = 0, wv = 0, xv = 0;
          if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
            bv = rb[r];
            wv = omega_over<T>(om, dg + rm[r]);
            xv = rx[r];
          }
          bs[k] = bv;
          ws[k] = wv;
          xa[k] = xv;
        }
      }
    }
    __syncthreads();
    if (t + 1 < t1) fetch(t + 1);
    if (live) {
      for (int k = tid; k < W * W; k += BS) {
        const int q2 = k / W, q1 = k - q2 * W;
        const int g1 = o1 + q1, g2 = o2 + q2;
        if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
          // fine 1-based F: even -> coarse F/2; odd -> (F-1)/2 and (F+1)/2, 1/2 each
          const int F1 = g1 + 1, F2 = g2 + 1;
          const int pi = ((F1 >> 1) - cb1) + WC * ((F2 >> 1) - cb2);
          T v;
          if (F1 & 1) {
            v = (F2 & 1) ? (T)0.25 * ((cs[pi] + cs[pi + 1]) + (cs[pi + WC] + cs[pi + WC + 1]))
                         : (T)0.5 * (cs[pi] + cs[pi + 1]);
          } else {
            v = (F2 & 1) ? (T)0.5 * (cs[pi] + cs[pi + WC]) : cs[pi];
          }
          xa[k] += v;
        }
      }
      __syncthreads();
      T* a = xa;
      T* c = xb;
#pragma unroll
      for (int s = 1; s <= NU; ++s) {
        const int w = W - 2 * s;
        for (int k = tid; k < w * w; k += BS) {
          const int r2 = k / w, r1 = k - r2 * w;
          const int li = (r1 + s) + W * (r2 + s);
          c[li] = om1 * a[li] + ws[li] * (bs[li] + p2l_nb<T, ST>(a, li, W, ih2));
        }
        __syncthreads();
        T* tmp = a; a = c; c = tmp;
      }
      for (int k = tid; k < TF * TF; k += BS) {
        const int r2 = k / TF, r1 = k - r2 * TF;
        const int g1 = tx * TF + r1, g2 = ty * TF + r2;
        if (g1 < N && g2 < N) xout[g1 + N * g2] = a[(NU + r1) + W * (NU + r2)];
      }
    }
    __syncthreads();  // the next tile's staging overwrites the LDS
  }
}

}  // namespace ipm
