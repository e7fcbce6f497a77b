// Krylov kernels for the Newton saddle-point system of eq. (NewtonSystem)
// with M = I, unknowns [dy; dw; dv; dp] stored as four consecutive blocks of
// n doubles:
//
//   K = [ I+Th_y    0        0       A^T ]
//       [ 0       a+Th_w    -a       -I  ]
//       [ 0        -a      a+Th_v     I  ]
//       [ A        -I        I        0  ]
//
// Preconditioned MINRES (Sec. 4: the Krylov method used with P_D) runs with
// all scalars on the device.  One iteration is
//   K1  pending direction/solution update of the previous iteration, then
//       q = K z_j / gamma_j and delta_j = <q, z_j / gamma_j>
//   K2  Lanczos step v_{j+1} = q - (delta_j/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1},
//       exact (1,1)-block inverse of P_D on the y, w, v blocks and their part
//       of <v_{j+1}, z_{j+1}>; the p block is handed to the multigrid.  It
//       also advances the unpreconditioned residual of the previous iterate,
//       r_{j-1} = s^2 r_{j-2} + (phi c / gamma_j) v_j (the residual in the
//       Lanczos basis is phi times the last column of the transposed QR
//       rotations; the identity needs only the computed three-term relation,
//       so it holds with an inexact FP32 preconditioner), and stops the solve
//       once |r|_2 <= tol |b|_2
//   MG  z_{j+1,p} = S_hat^-1 v_{j+1,p}
//   K4  rest of <v_{j+1}, z_{j+1}>, gamma_{j+1}, the Givens rotation and the
//       coefficients of the next update, all in the last block.
// Every kernel serves instance blockIdx.z; each instance stops on its own.
#include "common.h"

namespace ipm {

// Rows of K applied at node i to the 4-block vector x (scaled by s).
__device__ __forceinline__ void saddle_rows(const Inst& I, const double* __restrict__ x, int i, double s,
                                            double out[4]) {
  int i1, i2, i3;
  inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
  const int n = I.n;
  const double xy = x[i], xw = x[n + i], xv = x[2 * n + i];
  const double ty = I.ty[i], tw = I.tw[i], tv = I.tv[i], a = I.alpha;
  const double ATxp = inst_op<double>(I, x + 3 * n, i, i1, i2, i3, true);
  const double Axy = inst_op<double>(I, x, i, i1, i2, i3, false);
  const double xp = x[3 * n + i];
  if (I.pde == 3) {
    // Q1 (Sec. 2): M in the (1,1) block, alpha M~ and the coupling M bar
    const double My = q1_mass_track<double>(I, x, i, i1, i2, i3), Mw = q1_mass<double>(x + n, i, i1, i2, i3, I.N, I.dim);
    const double Mv = q1_mass<double>(x + 2 * n, i, i1, i2, i3, I.N, I.dim), Mp = q1_mass<double>(x + 3 * n, i, i1, i2, i3, I.N, I.dim);
    out[0] = s * (My + ty * xy + ATxp);
    out[1] = s * (a * (Mw - Mv) + tw * xw - Mp);
    out[2] = s * (-a * (Mw - Mv) + tv * xv + Mp);
    out[3] = s * (Axy - (Mw - Mv));
    return;
  }
  out[0] = s * ((obs_w(I, i) + ty) * xy + ATxp);
  out[1] = s * ((a + tw) * xw - a * xv - xp);
  out[2] = s * (-a * xw + (a + tv) * xv + xp);
  out[3] = s * (Axy - xw + xv);
}

// |K||x| row by row (all off-diagonal stencil entries are <= 0, so |A||x| = 2 diag |x| - A|x|).
__device__ __forceinline__ void saddle_rows_abs(const Inst& I, const double* __restrict__ x, int i, double out[4]) {
  int i1, i2, i3;
  inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
  const int n = I.n;
  const double xy = fabs(x[i]), xw = fabs(x[n + i]), xv = fabs(x[2 * n + i]), xp = fabs(x[3 * n + i]);
  const double ty = I.ty[i], tw = I.tw[i], tv = I.tv[i], a = I.alpha;
  const double ATxp = inst_op_abs(I, x + 3 * n, i, i1, i2, i3, true);
  const double Axy = inst_op_abs(I, x, i, i1, i2, i3, false);
  if (I.pde == 3) {
    const double My = q1_mass_track<double, true>(I, x, i, i1, i2, i3);
    const double Mw = q1_mass<double, true>(x + n, i, i1, i2, i3, I.N, I.dim);
    const double Mv = q1_mass<double, true>(x + 2 * n, i, i1, i2, i3, I.N, I.dim);
    const double Mp = q1_mass<double, true>(x + 3 * n, i, i1, i2, i3, I.N, I.dim);
    out[0] = My + ty * xy + ATxp;
    out[1] = a * (Mw + Mv) + tw * xw + Mp;
    out[2] = a * (Mw + Mv) + tv * xv + Mp;
    out[3] = Axy + Mw + Mv;
    return;
  }
  out[0] = (obs_w(I, i) + ty) * xy + ATxp;
  out[1] = (a + tw) * xw + a * xv + xp;
  out[2] = a * xw + (a + tv) * xv + xp;
  out[3] = Axy + xw + xv;
}

// Per-node inverse of the z block [a+t_w, -a; -a, a+t_v] (alpha M~ + Theta_z
// with M = I; Sec. 4.1); for Q1 the paper's alpha D~_M + Theta_z, a = alpha D_M.
__device__ __forceinline__ void apply_z_inv(const Inst& I, int i, double rw, double rv, double& zw, double& zv) {
  const double tw = I.tw[i], tv = I.tv[i], a = I.pde == 3 ? I.alpha * q1_mass_diag(I.dim) : I.alpha;
  const double det = a * (tw + tv) + tw * tv;
  zw = ((a + tv) * rw + a * rv) / det;
  zv = (a * rw + (a + tw) * rv) / det;
}

// Exact inverse of the (1,1) block of P_D at node i: 1/(O+Th_y) on y and the
// per-node 2x2 inverse on (w, v) (Sec. 4.1 with D_M = M = I).
__device__ __forceinline__ void apply_A11_inv(const Inst& I, int i, double ry, double rw, double rv, double& zy,
                                              double& zw, double& zv) {
  zy = ry / (obs_w(I, i) + I.ty[i]);
  apply_z_inv(I, i, rw, rv, zw, zv);
}

// y = K x (single instance)
__global__ void __launch_bounds__(kBS) k_saddle(const Inst* __restrict__ Dp, const double* __restrict__ x,
                                                double* __restrict__ y) {
  INST_BEGIN
  const int i = xcd_node(I.n);
  if (i >= I.n) return;
  double o[4];
  saddle_rows(I, x, i, 1.0, o);
  const int n = I.n;
  y[i] = o[0]; y[n + i] = o[1]; y[2 * n + i] = o[2]; y[3 * n + i] = o[3];
}

// R = rhs - K X, |R|_2 -> ctrl->rnorm, and |(|K||X| + |rhs|)|_2 -> ctrl->rfloor: the
// scale of the rounding error of evaluating the residual in FP64, which
// bounds the attainable relative residual.
__global__ void __launch_bounds__(kBS) k_true_residual(const Inst* __restrict__ Dp) {
  INST_BEGIN
  __shared__ double smem[2 * kBS / 64];
  const int i = xcd_node(I.n);
  double acc[2] = {0.0, 0.0};
  if (i < I.n) {
    double o[4], m[4];
    saddle_rows(I, I.X, i, 1.0, o);
    saddle_rows_abs(I, I.X, i, m);
    const int n = I.n;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double bk = I.rhs[k * n + i];
      const double rk = bk - o[k];
      I.R[k * n + i] = rk;
      acc[0] += rk * rk;
      const double mk = m[k] + fabs(bk);
      acc[1] += mk * mk;
    }
  }
  if (grid_reduce<kSum, 2, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0) {
    I.ctrl->rnorm = sqrt(acc[0]);
    I.ctrl->rfloor = sqrt(acc[1]);
  }
}

// After a Krylov cycle and its true residual: converged when the relative
// residual meets max(tol, ff * rfloor / bnorm) (ff: rounding factor); else
// another cycle from the true residual unless the iteration budget is spent.
// its_from_j: count FGMRES steps (ctrl->j) instead of MINRES iterations.
__global__ void k_krylov_mark(const Inst* __restrict__ Dp, double tol, double ff, int maxit, int its_from_j) {
  INST_BEGIN
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;  // finished in an earlier cycle
  C->its_total += its_from_j ? C->j : C->iter;
  const double bn = C->bnorm;
  const double rel = bn > 0.0 ? C->rnorm / bn : 0.0;
  C->relres = rel;
  const double lim = fmax(tol, bn > 0.0 ? ff * C->rfloor / bn : 0.0);
  if (rel <= lim) { C->want_restart = 0; return; }
  if (!(rel == rel) || C->breakdown || C->its_total >= maxit) { C->want_restart = 0; C->failed = 1; return; }
  C->want_restart = 1;
}

// Start of a Krylov solve: X = 0, want_restart = 1 (so that the first cycle
// runs), counters cleared.  bnorm comes from the Newton setup.
__global__ void __launch_bounds__(kBS) k_krylov_begin(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i < 4L * I.n) I.X[i] = 0.0;
  if (i == 0) {
    KrylovCtrl* C = I.ctrl;
    C->want_restart = 1;
    C->its_total = 0;
    C->failed = 0;
    C->relres = 0.0;
    C->iter = 0;
    C->j = 0;
    C->stop = 0;
    C->breakdown = 0;
  }
}

// Diagonal part of the preconditioner: z_{y,w,v} = A11^-1 r, and the multigrid
// right-hand side b_0 = (T) r_p (P_D) or, after k_pt_rhs, B z_A - r_p (P_T).
// Operands: explicit pointers, or (when null) the FGMRES slots r = V_j, z = Z_j.
template <typename T>
__global__ void __launch_bounds__(kBS) k_precond_diag(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                                      double* __restrict__ zx, int j, int pt, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double* r = rx ? rx : I.fV + (size_t)j * 4 * n;
  double* z = zx ? zx : I.fZ + (size_t)j * 4 * n;
  double zy, zw, zv;
  apply_A11_inv(I, i, r[i], r[n + i], r[2 * n + i], zy, zw, zv);
  if (I.pde != 3) z[i] = zy;  // Q1: the y block comes from k_cheb_block
  z[n + i] = zw; z[2 * n + i] = zv;
  if (!pt) ((T*)I.lv[0].b)[i] = (T)r[3 * n + i];
}

// Q1 (Sec. 4.1): z_y = (M + Theta_y)^-1 r_y approximated by Chebyshev
// semi-iteration with the diagonal D_M + Theta_y, whose preconditioned
// spectrum lies in [1/4, 9/4] (the 2D Q1 mass-matrix bounds): with
// theta, delta the centre and half-width of that interval and x_0 = 0,
//   x_1 = d_0 = (D_M + Theta_y)^-1 r / theta,
//   r_k = r_{k-1} - (M + Theta_y) d_{k-1},
//   d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) (D_M + Theta_y)^-1 r_k,
//   x_{k+1} = x_k + d_k,  rho_0 = delta / theta, rho_k = 1 / (2 theta / delta - rho_{k-1}).
// The steps run S per launch (temporal blocking): a workgroup takes a TT x TT
// tile of nodes with a halo of S nodes, holds r, d (two buffers), the
// diagonal and Theta_y of the region in LDS and runs steps k0 .. k0+S-1
// there; every step that reads neighbours shrinks the valid region by one
// node, so the tile's own nodes stay exact (values outside the grid are zero,
// which drops those neighbours as the mass stencil does).  Between launches
// r and d live in the q workspace (free outside the MINRES matvec), two
// buffers each by launch parity (in: launch & 1, out: the other), so no
// workgroup overwrites values another still reads as its halo; x is the
// output's y block, read and written at the tile's own nodes only.
// Operands: MINRES (mpar >= 0) the Lanczos vector v = V[1-mpar] and its
// image Z[1-mpar]; otherwise rx, zx or the FGMRES slots V_j, Z_j.  guard 1:
// skip a stopped solve; 2: skip an instance without a pending cycle.
struct ChebCoef {
  double rho[24];  // rho_k
  double theta, delta;
};

template <int TT, int S>
__global__ void __launch_bounds__(kBS) k_cheb_block(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                                    double* __restrict__ zx, int j, int mpar, int k0, int launch,
                                                    ChebCoef cf, int guard) {
  INST_BEGIN
  if ((guard == 1 && I.ctrl->stop) || (guard == 2 && !I.ctrl->want_restart)) return;
  const int N = I.N, n = I.n;
  const int t1 = blockIdx.x * TT, t2 = blockIdx.y * TT;
  if (t1 >= N || t2 >= N) return;
  constexpr int W = TT + 2 * S;
  __shared__ double R[W * W], D0[W * W], D1[W * W], DI[W * W], TY[W * W];
  const double* r = mpar >= 0 ? I.V[1 - mpar] : (rx ? rx : I.fV + (size_t)j * 4 * n);
  double* z = mpar >= 0 ? I.Z[1 - mpar] : (zx ? zx : I.fZ + (size_t)j * 4 * n);
  const int in = launch & 1, out = 1 - in;
  const double* rin = k0 == 0 ? r : I.Q + (size_t)in * n;
  const double* din = I.Q + (size_t)(2 + in) * n;
  double* rout = I.Q + (size_t)out * n;
  double* dout = I.Q + (size_t)(2 + out) * n;
  const int o1 = t1 - S, o2 = t2 - S;
  const int tid = threadIdx.x;
  for (int k = tid; k < W * W; k += kBS) {
    const int q2 = k / W, q1 = k - q2 * W;
    const int g1 = o1 + q1, g2 = o2 + q2;
    double rv = 0, dv = 0, iv = 0, tv = 0;
    if ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N) {
      const int gi = g1 + N * g2;
      tv = I.ty[gi];
      iv = 1.0 / (kQ1MassDiag + tv);
      rv = rin[gi];
      dv = k0 == 0 ? 0.0 : din[gi];
    }
    R[k] = rv; D0[k] = dv; DI[k] = iv; TY[k] = tv;
  }
  __syncthreads();
  // own-node iterate x (read only where this workgroup writes it)
  double xo[(TT * TT + kBS - 1) / kBS];
#pragma unroll
  for (int u = 0; u < (TT * TT + kBS - 1) / kBS; ++u) {
    const int k = tid + u * kBS;
    const int r2 = k / TT, r1 = k - r2 * TT;
    const int g1 = t1 + r1, g2 = t2 + r2;
    xo[u] = (k < TT * TT && g1 < N && g2 < N && k0 > 0) ? z[g1 + N * g2] : 0.0;
  }
  double* dp = D0;
  double* dn = D1;
  int m = 0;  // nodes lost at each side of the region so far
  for (int s2 = 0; s2 < S; ++s2) {
    const int k = k0 + s2;
    if (k == 0) {
      for (int q = tid; q < W * W; q += kBS) dn[q] = R[q] * DI[q] / cf.theta;
    } else {
      ++m;
      const int w = W - 2 * m;
      const double rho = cf.rho[k], rho_prev = cf.rho[k - 1], c2 = 2.0 * rho / cf.delta;
      for (int q = tid; q < w * w; q += kBS) {
        const int r2 = q / w, r1 = q - r2 * w;
        const int li = (r1 + m) + W * (r2 + m);
        const double e = (dp[li - 1] + dp[li + 1]) + dp[li - W] + dp[li + W];
        const double cn = ((dp[li - W - 1] + dp[li - W + 1]) + dp[li + W - 1]) + dp[li + W + 1];
        const double Ad = (16.0 * dp[li] + 4.0 * e + cn) * (1.0 / 36.0) + TY[li] * dp[li];
        const double res = R[li] - Ad;
        R[li] = res;
        dn[li] = rho * rho_prev * dp[li] + c2 * res * DI[li];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (TT * TT + kBS - 1) / kBS; ++u) {
      const int kk = tid + u * kBS;
      const int r2 = kk / TT, r1 = kk - r2 * TT;
      if (kk < TT * TT) xo[u] = (k == 0) ? dn[(r1 + S) + W * (r2 + S)] : xo[u] + dn[(r1 + S) + W * (r2 + S)];
    }
    double* t = dp; dp = dn; dn = t;
  }
#pragma unroll
  for (int u = 0; u < (TT * TT + kBS - 1) / kBS; ++u) {
    const int k = tid + u * kBS;
    const int r2 = k / TT, r1 = k - r2 * TT;
    const int g1 = t1 + r1, g2 = t2 + r2;
    if (k < TT * TT && g1 < N && g2 < N) {
      const int gi = g1 + N * g2, li = (r1 + S) + W * (r2 + S);
      z[gi] = xo[u];
      rout[gi] = R[li];
      dout[gi] = dp[li];
    }
  }
}

// The same semi-iteration for the trilinear mass (3D, D_M = 8/27, spectrum
// [1/8, 27/8]), one step per launch: launch k >= 1 reads d_(k-1) over the
// 27-point neighbourhood and r_(k-1) at the node (the input r itself for
// k = 1) and writes r_k, d_k and x_(k+1) = x_k + d_k; launch 0 writes d_0
// and x_1.  r and d sit in the q workspace by the parity of k (in: k & 1,
// out: the other), so no thread overwrites a value another still reads.
// Operands and guard as for k_cheb_block.
// Blocks of the 3D step: 16 x 4 x 4 nodes per workgroup (one per thread),
// their d with a one-node halo staged in LDS (zero outside the grid), so the
// 27-point mass is summed from LDS with no boundary tests or divisions.
constexpr int kCb1 = 16, kCb2 = 4, kCb3 = 4;
static_assert(kCb1 * kCb2 * kCb3 == kBS, "one node per thread");
__host__ __device__ constexpr int cheb3_blocks(int N) {
  return ((N + kCb1 - 1) / kCb1) * ((N + kCb2 - 1) / kCb2) * ((N + kCb3 - 1) / kCb3);
}

__global__ void __launch_bounds__(kBS) k_cheb_step3(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                                    double* __restrict__ zx, int j, int mpar, int k, ChebCoef cf,
                                                    int guard) {
  INST_BEGIN
  if ((guard == 1 && I.ctrl->stop) || (guard == 2 && !I.ctrl->want_restart)) return;
  const int n = I.n, N = I.N;
  // the launch's blocks are dispatched round-robin over the 8 XCDs: XCD x
  // takes the x-th contiguous eighth (a slab of block layers), so the
  // neighbouring planes of d stay in its L2
  int b = blockIdx.x;
  if ((gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
  const int nb1 = (N + kCb1 - 1) / kCb1, nb2 = (N + kCb2 - 1) / kCb2;
  if (b >= cheb3_blocks(N)) return;
  const int b1 = b % nb1, bq = b / nb1, b2 = bq % nb2, b3 = bq / nb2;
  const int tid = threadIdx.x;
  const int t1 = tid % kCb1, t2 = (tid / kCb1) % kCb2, t3 = tid / (kCb1 * kCb2);
  const int i1 = b1 * kCb1 + t1, i2 = b2 * kCb2 + t2, i3 = b3 * kCb3 + t3;
  const bool own = i1 < N && i2 < N && i3 < N;
  const int i = own ? i1 + N * (i2 + N * i3) : 0;
  const double* r = mpar >= 0 ? I.V[1 - mpar] : (rx ? rx : I.fV + (size_t)j * 4 * n);
  double* z = mpar >= 0 ? I.Z[1 - mpar] : (zx ? zx : I.fZ + (size_t)j * 4 * n);
  const int in = k & 1, out = 1 - in;
  double* dout = I.Q + (size_t)(2 + out) * n;
  const double ty = own ? I.ty[i] : 0.0;
  const double iv = 1.0 / (kQ1MassDiag3 + ty);
  if (k == 0) {
    if (!own) return;
    const double d0 = r[i] * iv / cf.theta;
    dout[i] = d0;
    z[i] = d0;
    return;
  }
  const double* rin = k == 1 ? r : I.Q + (size_t)in * n;
  const double* din = I.Q + (size_t)(2 + in) * n;
  constexpr int H1 = kCb1 + 2, H2 = kCb2 + 2, H3 = kCb3 + 2;
  __shared__ double sd[H1 * H2 * H3];
  for (int e = tid; e < H1 * H2 * H3; e += kBS) {
    const int e1 = e % H1, e2 = (e / H1) % H2, e3 = e / (H1 * H2);
    const int g1 = b1 * kCb1 - 1 + e1, g2 = b2 * kCb2 - 1 + e2, g3 = b3 * kCb3 - 1 + e3;
    sd[e] = ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N && (unsigned)g3 < (unsigned)N)
                ? din[g1 + N * (g2 + N * g3)]
                : 0.0;
  }
  __syncthreads();
  if (!own) return;
  // the 27-point mass in the order of q1_mass3 (off-grid neighbours are zeros here)
  const int li = (t1 + 1) + H1 * ((t2 + 1) + H2 * (t3 + 1));
  double f = 0, e = 0, c = 0;
#pragma unroll
  for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
    for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        const int kk = (o1 != 0) + (o2 != 0) + (o3 != 0);
        if (kk == 0) continue;
        const double v = sd[li + o1 + H1 * (o2 + H2 * o3)];
        if (kk == 1) f += v;
        else if (kk == 2) e += v;
        else c += v;
      }
  const double dv = sd[li];
  const double mass = (64.0 * dv + 16.0 * f + 4.0 * e + c) * (1.0 / 216.0);
  const double res = rin[i] - (mass + ty * dv);
  const double dn = cf.rho[k] * cf.rho[k - 1] * dv + (2.0 * cf.rho[k] / cf.delta) * res * iv;
  I.Q[(size_t)out * n + i] = res;
  dout[i] = dn;
  z[i] += dn;
}

// P_T (Sec. 4, block lower triangular [A11 0; B -S_hat]): the p block solves
// S_hat z_p = B z_A - r_p with B z_A = A z_y - z_w + z_v (M = I).
template <typename T>
__global__ void __launch_bounds__(kBS) k_pt_rhs(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                                const double* __restrict__ zx, int j, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  int i1, i2, i3;
  inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
  const int n = I.n;
  const double* r = rx ? rx : I.fV + (size_t)j * 4 * n;
  const double* z = zx ? zx : I.fZ + (size_t)j * 4 * n;
  const double Bz = I.pde == 3 ? inst_op<double>(I, z, i, i1, i2, i3, false) -
                                      (q1_mass<double>(z + n, i, i1, i2, i3, I.N, I.dim) - q1_mass<double>(z + 2 * n, i, i1, i2, i3, I.N, I.dim))
                                : inst_op<double>(I, z, i, i1, i2, i3, false) - z[n + i] + z[2 * n + i];
  ((T*)I.lv[0].b)[i] = (T)(Bz - r[3 * n + i]);
}

// Partial-observation preconditioner P_Pi (Sec. 4.3, eq. (eq:prec1)), applied
// as v2 = (alpha M~ + Theta_z)^-1 r_z, v1 = L^-1 (Mbar v2 + r_p),
// v3 = S_Pi^-1 ((O + Theta_y) v1 - r_y), with S_Pi approximated by
// (L^T + M_l) L^-1 (L + M_r), M_l = O + Theta_y and M_r = Sigma (the
// diagonal of Mbar (alpha M~ + Theta_z)^-1 Mbar^T), every solve by multigrid.
// Step a: z_w, z_v and the right-hand side Mbar v2 + r_p of the L solve.
template <typename T>
__global__ void __launch_bounds__(kBS) k_ppi_a(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                               double* __restrict__ zx, int j, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double* r = rx ? rx : I.fV + (size_t)j * 4 * n;
  double* z = zx ? zx : I.fZ + (size_t)j * 4 * n;
  double zw, zv;
  apply_z_inv(I, i, r[n + i], r[2 * n + i], zw, zv);
  z[n + i] = zw;
  z[2 * n + i] = zv;
  if (I.pde != 3) ((T*)I.lv[0].b)[i] = (T)(zw - zv + r[3 * n + i]);
}

// Q1, after step a: the right-hand side M (z_w - z_v) + r_p of the L solve
// (the coupling Mbar applies the mass to the neighbours' z block).
template <typename T>
__global__ void __launch_bounds__(kBS) k_ppi_a_q1(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                                  const double* __restrict__ zx, int j, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double* r = rx ? rx : I.fV + (size_t)j * 4 * n;
  const double* z = zx ? zx : I.fZ + (size_t)j * 4 * n;
  int i1, i2, i3;
  node_coords(i, I.N, I.dim, i1, i2, i3);
  const double Mz = q1_mass<double>(z + n, i, i1, i2, i3, I.N, I.dim) - q1_mass<double>(z + 2 * n, i, i1, i2, i3, I.N, I.dim);
  ((T*)I.lv[0].b)[i] = (T)(Mz + r[3 * n + i]);
}

// Step b: z_y = v1 (the L solve's output) and the right-hand side
// (O + Theta_y) v1 - r_y of the solve with L^T + M_l.
template <typename T>
__global__ void __launch_bounds__(kBS) k_ppi_b(const Inst* __restrict__ Dp, const double* __restrict__ rx,
                                               double* __restrict__ zx, int j, int outsel, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double* r = rx ? rx : I.fV + (size_t)j * 4 * n;
  double* z = zx ? zx : I.fZ + (size_t)j * 4 * n;
  const T* out = mg_out<T>(I, outsel);
  const double v1 = (double)out[i];
  z[i] = v1;
  if (I.pde == 3) {  // Q1: (M_O + Theta_y) v1 - r_y with the observed elements' mass
    int i1, i2, i3;
    node_coords(i, I.N, I.dim, i1, i2, i3);
    const double Mv = (double)q1_mass_track<T>(I, out, i, i1, i2, i3);
    ((T*)I.lv[0].b)[i] = (T)(Mv + I.ty[i] * v1 - r[i]);
    return;
  }
  ((T*)I.lv[0].b)[i] = (T)((obs_w(I, i) + I.ty[i]) * v1 - r[i]);
}

// Step c: the right-hand side L s of the solve with L + M_r (s: the previous
// solve's output).
template <typename T>
__global__ void __launch_bounds__(kBS) k_ppi_c(const Inst* __restrict__ Dp, int outsel, int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = xcd_node(I.n);
  if (i >= I.n) return;
  int i1, i2, i3;
  node_coords(i, I.N, I.dim, i1, i2, i3);
  const T* s = mg_out<T>(I, outsel);
  ((T*)I.lv[0].b)[i] = apply_op<T>(s, i, i1, i2, i3, I.N, I.dim, I.pde, I.h, I.eps, false);
}

// z_p = (double) multigrid output
template <typename T>
__global__ void __launch_bounds__(kBS) k_store_p(const Inst* __restrict__ Dp, double* __restrict__ zx, int j, int outsel,
                                                 int guard) {
  INST_BEGIN
  if (guard && I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  double* z = zx ? zx : I.fZ + (size_t)j * 4 * I.n;
  z[3 * I.n + i] = (double)mg_out<T>(I, outsel)[i];
}

// ---------------------------------------------------------------- MINRES

// Start of a MINRES cycle from the residual (src 0: rhs, 1: R): v_1 = r,
// v_0 = 0, w = K w = 0, tracked r = source, z_1 on the diagonal blocks,
// partial <v_1, z_1>; b_0 = (T) r_p.  Instances without a pending cycle skip.
template <typename T>
__global__ void __launch_bounds__(kBS) k_minres_init(const Inst* __restrict__ Dp, int src) {
  INST_BEGIN
  if (!I.ctrl->want_restart) return;
  __shared__ double smem[kBS / 64];
  const int i = blockIdx.x * kBS + threadIdx.x;
  double acc[1] = {0.0};
  if (i < I.n) {
    const int n = I.n;
    const double* r = src ? I.R : I.rhs;
    const double ry = r[i], rw = r[n + i], rv = r[2 * n + i], rp = r[3 * n + i];
    double zy, zw, zv;
    apply_A11_inv(I, i, ry, rw, rv, zy, zw, zv);
    double* V1 = I.V[1];
    double* Z1 = I.Z[1];
    V1[i] = ry; V1[n + i] = rw; V1[2 * n + i] = rv; V1[3 * n + i] = rp;
    const bool q1 = I.pde == 3;  // Q1: z_y from k_cheb_block, its part of <v, z> in K4
    if (!q1) Z1[i] = zy;
    Z1[n + i] = zw; Z1[2 * n + i] = zv;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = k * n + i;
      I.V[0][q] = 0.0; I.W[0][q] = 0.0; I.W[1][q] = 0.0;
      I.Rt[q] = r[q];
    }
    ((T*)I.lv[0].b)[i] = (T)rp;
    acc[0] = (q1 ? 0.0 : ry * zy) + rw * zw + rv * zv;
  }
  if (grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0)
    I.ctrl->dot_tmp = acc[0];
}

// K1: pending update of iteration j-1 (direction w, solution x), then
// q = K z_j / gamma_j and delta_j = <q, z_j/gamma_j>.  par = parity of j;
// timing = 1 only for stand-alone timing.  The solution takes the updates
// of two iterations at a time: after an odd iteration i only w_i is formed
// (its coefficient is kept in coef_x_def), after the next one
// x += c_i w_i + c_{i+1} w_{i+1} (w_i is the w read for the recurrence
// anyway), which halves the traffic of x; k_minres_flush adds what is left.
// The direction vectors stream through once per iteration (nontemporal).
__global__ void __launch_bounds__(kBS) k_minres_k1(const Inst* __restrict__ Dp, int par, int timing) {
  INST_BEGIN
  __shared__ double smem[kBS / 64];
  KrylovCtrl* C = I.ctrl;
  if (C->stop && !timing) return;
  const int pending = timing ? 1 : C->pending;
  const double* __restrict__ Zc = I.Z[par];
  const double* __restrict__ Zprev = I.Z[1 - par];
  double* __restrict__ Wsame = I.W[1 - par];
  const double* __restrict__ Wother = I.W[par];
  double* __restrict__ X = I.X;
  double* __restrict__ Q = I.Q;
  const int i = xcd_node(I.n);
  double acc[1] = {0.0};
  if (i < I.n) {
    const int n = I.n;
    if (pending) {
      const double g = C->gamma_w, a1 = C->a1, a2 = C->a2, a3 = C->a3, cx = C->coef_x, cxd = C->coef_x_def;
      // the pending update belongs to iteration C->iter; stand-alone timing
      // takes the full form (x updated) every launch
      const bool defer = !timing && (C->iter & 1);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = k * n + i;
        const double wo = __builtin_nontemporal_load(&Wother[j]);
        const double wi = (__builtin_nontemporal_load(&Zprev[j]) / g - a3 * __builtin_nontemporal_load(&Wsame[j]) -
                           a2 * wo) / a1;
        __builtin_nontemporal_store(wi, &Wsame[j]);
        if (!defer) __builtin_nontemporal_store(__builtin_nontemporal_load(&X[j]) + (cxd * wo + cx * wi), &X[j]);
      }
    }
    const double s = 1.0 / C->gamma;
    double o[4];
    saddle_rows(I, Zc, i, s, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      __builtin_nontemporal_store(o[k], &Q[k * n + i]);
      acc[0] += o[k] * (Zc[k * n + i] * s);
    }
  }
  if (grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0) {
    C->delta = acc[0];
    if (pending && !timing) C->pending = 0;
  }
}

// K2: Lanczos vector v_{j+1} (overwrites v_{j-1}), z_{j+1} on the diagonal
// blocks, partial <v_{j+1}, z_{j+1}>, b_0 = (T) v_{j+1,p} for the multigrid;
// the pending residual update with v_j and, in the last block, the stop test
// on |r_{j-1}|_2.  timing = 1 only for stand-alone timing.  The Lanczos and
// residual vectors stream through once per iteration (nontemporal).
template <typename T>
__global__ void __launch_bounds__(kBS) k_minres_k2(const Inst* __restrict__ Dp, int par, int timing) {
  INST_BEGIN
  __shared__ double smem[2 * kBS / 64];
  KrylovCtrl* C = I.ctrl;
  if (C->stop && !timing) return;
  const int rpend = timing ? 1 : C->rpend;
  const double* __restrict__ Q = I.Q;
  const double* __restrict__ Vc = I.V[par];
  double* __restrict__ Vn = I.V[1 - par];
  double* __restrict__ Zn = I.Z[1 - par];
  double* __restrict__ Rt = I.Rt;
  const int i = blockIdx.x * kBS + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (i < I.n) {
    const int n = I.n;
    const double c1 = C->delta / C->gamma, c2 = C->gamma / C->gamma_prev;
    const double rs2 = C->rs2, rc = C->rc;
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double vc = __builtin_nontemporal_load(&Vc[k * n + i]);
      v[k] = __builtin_nontemporal_load(&Q[k * n + i]) - c1 * vc - c2 * __builtin_nontemporal_load(&Vn[k * n + i]);
      __builtin_nontemporal_store(v[k], &Vn[k * n + i]);
      if (rpend) {
        const double r = rs2 * __builtin_nontemporal_load(&Rt[k * n + i]) + rc * vc;
        __builtin_nontemporal_store(r, &Rt[k * n + i]);
        acc[1] += r * r;
      }
    }
    double zy, zw, zv;
    apply_A11_inv(I, i, v[0], v[1], v[2], zy, zw, zv);
    const bool q1 = I.pde == 3;  // Q1: z_y from k_cheb_block, its part of <v, z> in K4
    if (!q1) Zn[i] = zy;
    Zn[n + i] = zw; Zn[2 * n + i] = zv;
    ((T*)I.lv[0].b)[i] = (T)v[3];
    acc[0] = (q1 ? 0.0 : v[0] * zy) + v[1] * zw + v[2] * zv;
  }
  if (grid_reduce<kSum, 2, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0) {
    C->dot_tmp = acc[0];
    if (rpend && !timing) {
      C->rpend = 0;
      C->rtrack = sqrt(acc[1]);
      if (C->rtrack <= C->rtarget || !(acc[1] == acc[1])) C->stop = 1;
    }
  }
}

// K4: z_{nb,p} from the multigrid output, the rest of <v, z>, then the scalar
// recurrence in the last block.  mode 0 starts a cycle (gamma_1; nb = 1; the
// stop target is tol |b|), mode 1 is an iteration (nb = 1 - parity).
template <typename T>
__global__ void __launch_bounds__(kBS) k_minres_k4(const Inst* __restrict__ Dp, int nb, int mode, double tol, int maxit,
                                                   int outsel) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  KrylovCtrl* C = I.ctrl;
  const int n = I.n, pde = I.pde, cl = I.coarse_lev;
  const double* __restrict__ Vn = I.V[nb];
  double* __restrict__ Zn = I.Z[nb];
  const void* x0 = I.lv[0].x;
  const void* x02 = I.lv[0].x2;
  double* partials = I.partials;
  unsigned* counter = I.counter;
  IPM_LOAD_TOGETHER(go, C, n, pde, cl, Vn, Zn, x0, x02, partials, counter);
  if (!go) return;
  __shared__ double smem[kBS / 64];
  // the multigrid output (as mg_out)
  const T* __restrict__ xmg = (const T*)((cl == 0 || !outsel) ? x0 : x02);
  const int i = blockIdx.x * kBS + threadIdx.x;
  // the stop flag is requested with the node's data and tested before the store
  const int f_stop = C->stop, f_want = C->want_restart;
  double z = 0.0, v3 = 0.0, v0 = 0.0, z0 = 0.0;
  if (i < n) {
    z = (double)xmg[i];
    v3 = Vn[3 * n + i];
    if (pde == 3) {
      v0 = Vn[i];
      z0 = Zn[i];
    }
  }
  if (mode == 0 ? !f_want : f_stop) return;
  double acc[1] = {0.0};
  if (i < n) {
    Zn[3 * n + i] = z;
    acc[0] = v3 * z;
    if (pde == 3) acc[0] += v0 * z0;
  }
  if (!grid_reduce<kSum, 1, kBS>(acc, partials, counter, gridDim.x, blockIdx.x, smem) || threadIdx.x != 0) return;
  const double dot = C->dot_tmp + acc[0];
  if (mode == 0) {
    C->iter = 0;
    C->pending = 0;
    C->rpend = 0;
    C->breakdown = 0;
    C->rtarget = tol * C->bnorm;
    C->rtrack = INFINITY;
    C->c_prev = C->c = 1.0;
    C->s_prev = C->s = 0.0;
    C->gamma_prev = 1.0;
    C->est = 1.0;
    if (!(dot > 0.0) || !isfinite(dot)) {  // zero right-hand side, or an indefinite preconditioner
      C->gamma = 1.0;
      C->eta = C->eta0 = 0.0;
      C->breakdown = (dot == 0.0) ? 0 : 1;
      C->est = 0.0;
      C->stop = 1;
      return;
    }
    const double g1 = sqrt(dot);
    C->gamma = g1;
    C->eta = C->eta0 = g1;
    C->stop = 0;
    return;
  }
  if (!(dot >= 0.0) || !isfinite(dot)) {
    C->breakdown = 1;
    C->stop = 1;
    C->pending = 0;
    return;
  }
  const double gn = sqrt(dot);
  const double g = C->gamma, d = C->delta;
  const double a0 = C->c * d - C->c_prev * C->s * g;
  const double a1 = sqrt(a0 * a0 + gn * gn);
  const double a2 = C->s * d + C->c_prev * C->c * g;
  const double a3 = C->s_prev * g;
  const double cn = a0 / a1, sn = gn / a1;
  C->a1 = a1; C->a2 = a2; C->a3 = a3;
  if (C->iter & 1) C->coef_x_def = C->coef_x;  // the previous iteration's x update waits for this one's
  C->coef_x = cn * C->eta;
  C->gamma_w = g;
  C->pending = 1;
  C->eta = -sn * C->eta;
  C->rs2 = sn * sn;
  C->rc = gn > 0.0 ? C->eta * cn / gn : 0.0;
  C->rpend = 1;
  C->c_prev = C->c; C->c = cn;
  C->s_prev = C->s; C->s = sn;
  C->gamma_prev = g; C->gamma = gn;
  C->iter += 1;
  C->est = fabs(C->eta) / C->eta0;
  if (gn == 0.0 || C->its_total + C->iter >= maxit || !isfinite(a1) || a1 == 0.0) C->stop = 1;
}

// After the loop stopped: the pending update (with the parity of the
// instance's own last iteration) and the solution updates still deferred.
__global__ void __launch_bounds__(kBS) k_minres_flush(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const KrylovCtrl* C = I.ctrl;
  const int it = C->iter;
  if (!C->want_restart || !(C->pending || (it & 1))) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double* Zi = I.Z[it & 1];
  double* Wsame = I.W[it & 1];
  const double* Wother = I.W[(it + 1) & 1];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = k * n + i;
    if (C->pending) {
      // w_it; with it even, w_(it-1) still owes its x update
      const double wi = (Zi[q] / C->gamma_w - C->a3 * Wsame[q] - C->a2 * Wother[q]) / C->a1;
      Wsame[q] = wi;
      I.X[q] += (it & 1) ? C->coef_x * wi : (C->coef_x_def * Wother[q] + C->coef_x * wi);
    } else {
      // the last K1 formed w_it (it odd) and deferred its x update
      I.X[q] += C->coef_x * Wsame[q];
    }
  }
}

// Clear the stop flag (used before timing the iteration kernels in isolation).
__global__ void k_ctrl_continue(const Inst* __restrict__ Dp) {
  INST_BEGIN
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    I.ctrl->stop = 0;
    I.ctrl->pending = 0;
  }
}

#define IPM_KRY_INST(T)                                                                          \
  template __global__ void k_precond_diag<T>(const Inst*, const double*, double*, int, int, int); \
  template __global__ void k_pt_rhs<T>(const Inst*, const double*, const double*, int, int);      \
  template __global__ void k_store_p<T>(const Inst*, double*, int, int, int);                     \
  template __global__ void k_ppi_a<T>(const Inst*, const double*, double*, int, int);              \
  template __global__ void k_ppi_a_q1<T>(const Inst*, const double*, const double*, int, int);     \
  template __global__ void k_ppi_b<T>(const Inst*, const double*, double*, int, int, int);         \
  template __global__ void k_ppi_c<T>(const Inst*, int, int);                                      \
  template __global__ void k_minres_init<T>(const Inst*, int);                                   \
  template __global__ void k_minres_k2<T>(const Inst*, int, int);                                     \
  template __global__ void k_minres_k4<T>(const Inst*, int, int, double, int, int);
IPM_KRY_INST(float)
IPM_KRY_INST(double)
#undef IPM_KRY_INST

}  // namespace ipm
