// Interior point kernels: starting point, feasibility/complementarity
// measures, barrier diagonals and Newton right-hand side, step lengths and
// the iterate update (Algorithm A.1 of the Appendix; Sec. 3).
//
// Unit-mass finite-difference form: M = D = I, L = A.  Split bounds
// (Sec. 2, eq. (split)) with u_a < 0 < u_b: z_a = 0, z_b = [u_b; -u_a], so
// the gaps are w, u_b - w, v, -u_a - v (and y - y_a, y_b - y with state
// bounds).  Every kernel serves instance blockIdx.z of the descriptor array.
#include "common.h"

namespace ipm {

// Starting point: box midpoints, p = 0, multipliers mu0 / gap with mu0 = I.mu.
__global__ void __launch_bounds__(kBS) k_init_state(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const double mu0 = I.mu;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const double ua = I.ua[i], ub = I.ub[i];
  const double w = 0.5 * ub, v = -0.5 * ua;
  I.w[i] = w;
  I.v[i] = v;
  I.p[i] = 0.0;
  I.lwa[i] = mu0 / w;
  I.lwb[i] = mu0 / (ub - w);
  I.lva[i] = mu0 / v;
  I.lvb[i] = mu0 / (-ua - v);
  if (I.has_y) {
    const double ya = I.ya[i], yb = I.yb[i], y = 0.5 * (ya + yb);
    I.y[i] = y;
    I.lya[i] = mu0 / (y - ya);
    I.lyb[i] = mu0 / (yb - y);
  } else {
    I.y[i] = 0.0;
  }
}

// inf-norms of xi_p, xi_d (eq. (prdu)) and of the complementarity products
// (eq. (gap) without the mu term) -> stat[0..2].
__global__ void __launch_bounds__(kBS) k_measures(const Inst* __restrict__ Dp) {
  INST_BEGIN
  __shared__ double smem[3 * kBS / 64];
  const int i = xcd_node(I.n);
  double r[3] = {0.0, 0.0, 0.0};
  if (i < I.n) {
    int i1, i2, i3;
    inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
    const double y = I.y[i], w = I.w[i], v = I.v[i], p = I.p[i];
    const double u = w - v;
    const double Ay = inst_op<double>(I, I.y, i, i1, i2, i3, false);
    const double ATp = inst_op<double>(I, I.p, i, i1, i2, i3, true);
    const double ua = I.ua[i], ub = I.ub[i];
    const double lwa = I.lwa[i], lwb = I.lwb[i], lva = I.lva[i], lvb = I.lvb[i];
    // unit mass, or Q1: M u, M (y - y_d) and M p in eq. (prdu)
    const bool q1 = I.pde == 3;
    const double Mu = q1 ? q1_mass<double>(I.w, i, i1, i2, i3, I.N, I.dim) - q1_mass<double>(I.v, i, i1, i2, i3, I.N, I.dim) : u;
    const double Mp = q1 ? q1_mass<double>(I.p, i, i1, i2, i3, I.N, I.dim) : p;
    r[0] = fabs(Ay - Mu - I.fhat[i]);
    double dy = (q1 ? q1_mass_track<double>(I, I.y, i, i1, i2, i3) - q1_mass_track<double>(I, I.yd, i, i1, i2, i3)
                    : obs_w(I, i) * (y - I.yd[i])) + ATp;
    double pc = nmax(nmax(w * lwa, (ub - w) * lwb), nmax(v * lva, (-ua - v) * lvb));
    if (I.has_y) {
      const double lya = I.lya[i], lyb = I.lyb[i];
      dy += -lya + lyb;
      pc = nmax(pc, nmax((y - I.ya[i]) * lya, (I.yb[i] - y) * lyb));
    }
    const double dw = I.alpha * Mu + I.beta - Mp - lwa + lwb;
    const double dv = -I.alpha * Mu + I.beta + Mp - lva + lvb;
    r[1] = nmax(fabs(dy), nmax(fabs(dw), fabs(dv)));
    r[2] = fabs(pc);
  }
  if (grid_reduce<kMax, 3, kBS>(r, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0) {
    I.stat[0] = r[0];
    I.stat[1] = r[1];
    I.stat[2] = r[2];
  }
}

// Mean of the complementarity products (eq. (gap) with mu = 0) over every
// finite bound, the duality measure of the iterate -> stat[5] (the barrier
// target of the iterate-based rule is sigma times it).
__global__ void __launch_bounds__(kBS) k_compl_mean(const Inst* __restrict__ Dp) {
  INST_BEGIN
  __shared__ double smem[kBS / 64];
  const int i = blockIdx.x * kBS + threadIdx.x;
  double acc[1] = {0.0};
  if (i < I.n) {
    const double w = I.w[i], v = I.v[i];
    acc[0] = (w * I.lwa[i] + (I.ub[i] - w) * I.lwb[i]) + (v * I.lva[i] + (-I.ua[i] - v) * I.lvb[i]);
    if (I.has_y) {
      const double y = I.y[i];
      acc[0] += (y - I.ya[i]) * I.lya[i] + (I.yb[i] - y) * I.lyb[i];
    }
  }
  if (grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0)
    I.stat[5] = acc[0] / ((I.has_y ? 6.0 : 4.0) * I.n);
}

// Barrier diagonals Theta_y, Theta_w, Theta_v (Sec. 3, below eq.
// (NewtonSystem)), the matching term M_hat = sqrt(Sigma (O + Theta_y)) with
// Sigma = (t_w + t_v) / (alpha (t_w + t_v) + t_w t_v) (eq. (Schur) and the
// M_hat of Sec. 4.2 with M = D_M = I, O the observation weights), and the
// right-hand side of eq. (NewtonSystem) at barrier I.mu; |rhs|_2 ->
// ctrl->bnorm.  The reaction term of the multigrid operator is written, in
// the V-cycle precision T, to the finest level: M_hat, or for P_Pi (Sec. 4.3)
// M_r = Sigma in slot 0 and M_l = O + Theta_y in slot 1.
template <typename T>
__global__ void __launch_bounds__(kBS) k_newton_setup(const Inst* __restrict__ Dp) {
  INST_BEGIN
  __shared__ double smem[kBS / 64];
  const int i = xcd_node(I.n);
  const double mu = I.mu;
  double acc[1] = {0.0};
  if (i < I.n) {
    int i1, i2, i3;
    inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
    const double y = I.y[i], w = I.w[i], v = I.v[i], p = I.p[i];
    const double ua = I.ua[i], ub = I.ub[i];
    const double gwb = ub - w, gvb = -ua - v;
    const double tw = I.lwa[i] / w + I.lwb[i] / gwb;
    const double tv = I.lva[i] / v + I.lvb[i] / gvb;
    double ty = 0.0, by = 0.0;
    if (I.has_y) {
      const double gya = y - I.ya[i], gyb = I.yb[i] - y;
      ty = I.lya[i] / gya + I.lyb[i] / gyb;
      by = -mu / gya + mu / gyb;
    }
    const bool q1 = I.pde == 3;
    double sig, mh;
    const double ow = obs_w(I, i);
    if (q1) {
      // Sec. 4.2 with D_M = diag(M): [D_M/alpha - (1/alpha^2)(1/t_w + 1/t_v + 1/(alpha D_M))^-1]
      // = D_M^2 (t_w + t_v) / (alpha D_M (t_w + t_v) + t_w t_v), times D_M + Theta_y, square root
      const double dm = q1_mass_diag(I.dim);
      sig = dm * dm * (tw + tv) / (I.alpha * dm * (tw + tv) + tw * tv);
      mh = I.ppi ? sig : sqrt(sig * (dm + ty));
    } else {
      sig = (tw + tv) / (I.alpha * (tw + tv) + tw * tv);
      mh = I.ppi ? sig : sqrt(sig * (ow + ty));
    }
    I.ty[i] = ty;
    I.tw[i] = tw;
    I.tv[i] = tv;
    I.mh[i] = mh;
    // heat equation: every time step's multigrid operator is I/tau + A_h + M_hat
    ((T*)I.lv[0].mh)[i] = (T)(I.pde == 2 ? mh + 1.0 / I.tau : mh);
    // P_Pi: M_l = O + Theta_y; for Q1 the lumped mass of the observed elements + Theta_y
    if (I.ppi)
      ((T*)I.lv[0].mhb)[I.n + i] =
          (T)((q1 ? (I.eobs ? q1_obs_diag(i1, i2, i3, I.N, I.dim, I.eobs) : q1_mass_diag(I.dim)) : ow) + ty);
    const double u = w - v;
    const double Ay = inst_op<double>(I, I.y, i, i1, i2, i3, false);
    const double ATp = inst_op<double>(I, I.p, i, i1, i2, i3, true);
    const double Mu = q1 ? q1_mass<double>(I.w, i, i1, i2, i3, I.N, I.dim) - q1_mass<double>(I.v, i, i1, i2, i3, I.N, I.dim) : u;
    const double Mp = q1 ? q1_mass<double>(I.p, i, i1, i2, i3, I.N, I.dim) : p;
    const double Myd = q1 ? q1_mass_track<double>(I, I.y, i, i1, i2, i3) - q1_mass_track<double>(I, I.yd, i, i1, i2, i3)
                          : ow * (y - I.yd[i]);
    const double ry = -(Myd + ATp + by);
    const double rw = -(I.alpha * Mu + I.beta - Mp - mu / w + mu / gwb);
    const double rv = -(-I.alpha * Mu + I.beta + Mp - mu / v + mu / gvb);
    const double rp = -(Ay - Mu - I.fhat[i]);
    const int n = I.n;
    double* rhs = I.rhs;
    rhs[i] = ry;
    rhs[n + i] = rw;
    rhs[2 * n + i] = rv;
    rhs[3 * n + i] = rp;
    acc[0] = ry * ry + rw * rw + rv * rv + rp * rp;
  }
  if (grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0)
    I.ctrl->bnorm = sqrt(acc[0]);
}
template __global__ void k_newton_setup<float>(const Inst*);
template __global__ void k_newton_setup<double>(const Inst*);

// Full-weighting restriction of the M_hat diagonal from level l to level l+1
// (tensor product of the weights 1/4, 1/2, 1/4); the coarse operator is the
// rediscretized stencil plus this restricted reaction term.
template <typename T>
__global__ void __launch_bounds__(kBS) k_restrict_diag(const Inst* __restrict__ Dp, int l) {
  INST_BEGIN
  if (l + 1 >= I.nlev) return;
  const Level& F = I.lv[l];
  const Level& Cv = I.lv[l + 1];
  const int ic = blockIdx.x * kBS + threadIdx.x;
  if (ic >= Cv.n) return;
  const T* __restrict__ fine = (const T*)F.mh;
  const int Nf = F.N, Nc = Cv.N, dim = I.dim;
  int j1, j2, j3;
  node_coords(ic, Nc, dim, j1, j2, j3);
  // coarse node J (1-based) sits on fine node 2J (1-based) -> 0-based 2j+1
  const int f1 = 2 * j1 + 1, f2 = 2 * j2 + 1, f3 = 2 * j3 + 1;
  double acc = 0.0;
  const double wt[3] = {0.25, 0.5, 0.25};
  if (dim == 2) {
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a)
        acc += wt[a + 1] * wt[b + 1] * (double)fine[(f1 + a) + Nf * (f2 + b)];
  } else {
    for (int c = -1; c <= 1; ++c)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a)
          acc += wt[a + 1] * wt[b + 1] * wt[c + 1] * (double)fine[(f1 + a) + Nf * ((f2 + b) + Nf * (f3 + c))];
  }
  ((T*)Cv.mh)[ic] = (T)acc;
}
template __global__ void k_restrict_diag<float>(const Inst*, int);
template __global__ void k_restrict_diag<double>(const Inst*, int);

// Multiplier steps of eqs. (zupdate1)-(zupdate4) for one bound pair.
struct DL { double a, b; };
__device__ __forceinline__ DL dlam(double la, double lb, double ga, double gb, double dx, double mu) {
  DL r;
  r.a = -(la / ga) * dx - la + mu / ga;
  r.b = (lb / gb) * dx - lb + mu / gb;
  return r;
}
__device__ __forceinline__ double box_step(double ga, double gb, double dx) {
  // largest s >= 0 keeping lo <= x + s dx <= hi, given gaps ga = x - lo, gb = hi - x
  if (dx < 0.0) return ga / (-dx);
  if (dx > 0.0) return gb / dx;
  return INFINITY;
}
__device__ __forceinline__ double pos_step(double l, double dl) { return dl < 0.0 ? l / (-dl) : INFINITY; }

// Fraction-to-boundary step lengths (Algorithm A.1): alpha_P = alpha0 min(1, max
// primal step), alpha_D likewise for the multipliers -> stat[3], stat[4].
__global__ void __launch_bounds__(kBS) k_step_lengths(const Inst* __restrict__ Dp) {
  INST_BEGIN
  __shared__ double smem[2 * kBS / 64];
  const int i = blockIdx.x * kBS + threadIdx.x;
  const double mu = I.mu;
  double r[2] = {INFINITY, INFINITY};
  if (i < I.n) {
    const int n = I.n;
    const double* X = I.X;
    const double dy = X[i], dw = X[n + i], dv = X[2 * n + i];
    const double w = I.w[i], v = I.v[i], ua = I.ua[i], ub = I.ub[i];
    const double gwa = w, gwb = ub - w, gva = v, gvb = -ua - v;
    const double lwa = I.lwa[i], lwb = I.lwb[i], lva = I.lva[i], lvb = I.lvb[i];
    double sp = nmin(box_step(gwa, gwb, dw), box_step(gva, gvb, dv));
    const DL lw = dlam(lwa, lwb, gwa, gwb, dw, mu), lv = dlam(lva, lvb, gva, gvb, dv, mu);
    double sd = nmin(nmin(pos_step(lwa, lw.a), pos_step(lwb, lw.b)), nmin(pos_step(lva, lv.a), pos_step(lvb, lv.b)));
    if (I.has_y) {
      const double y = I.y[i], gya = y - I.ya[i], gyb = I.yb[i] - y;
      const double lya = I.lya[i], lyb = I.lyb[i];
      sp = nmin(sp, box_step(gya, gyb, dy));
      const DL ly = dlam(lya, lyb, gya, gyb, dy, mu);
      sd = nmin(sd, nmin(pos_step(lya, ly.a), pos_step(lyb, ly.b)));
    }
    // a NaN direction must not pass as a huge step
    if (dy != dy || dw != dw || dv != dv) sp = NAN;
    r[0] = sp;
    r[1] = sd;
  }
  if (grid_reduce<kMin, 2, kBS>(r, I.partials, I.counter, gridDim.x, blockIdx.x, smem) && threadIdx.x == 0) {
    I.stat[3] = I.alpha0 * nmin(1.0, r[0]);
    I.stat[4] = I.alpha0 * nmin(1.0, r[1]);
  }
}

// Iterate update of Algorithm A.1: (y, w, v) += alpha_P (dy, dw, dv);
// (p, lambdas) += alpha_D (dp, dlambdas).
__global__ void __launch_bounds__(kBS) k_update(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const int n = I.n;
  const double mu = I.mu;
  const double aP = I.stat[3], aD = I.stat[4];
  const double* X = I.X;
  const double dy = X[i], dw = X[n + i], dv = X[2 * n + i], dp = X[3 * n + i];
  const double w = I.w[i], v = I.v[i], ua = I.ua[i], ub = I.ub[i];
  const double lwa = I.lwa[i], lwb = I.lwb[i], lva = I.lva[i], lvb = I.lvb[i];
  const DL lw = dlam(lwa, lwb, w, ub - w, dw, mu), lv = dlam(lva, lvb, v, -ua - v, dv, mu);
  if (I.has_y) {
    const double y = I.y[i];
    const double lya = I.lya[i], lyb = I.lyb[i];
    const DL ly = dlam(lya, lyb, y - I.ya[i], I.yb[i] - y, dy, mu);
    I.lya[i] = lya + aD * ly.a;
    I.lyb[i] = lyb + aD * ly.b;
  }
  I.y[i] += aP * dy;
  I.w[i] = w + aP * dw;
  I.v[i] = v + aP * dv;
  I.p[i] += aD * dp;
  I.lwa[i] = lwa + aD * lw.a;
  I.lwb[i] = lwb + aD * lw.b;
  I.lva[i] = lva + aD * lv.a;
  I.lvb[i] = lvb + aD * lv.b;
}

// y = A x or A^T x (FP64), single instance.
__global__ void __launch_bounds__(kBS) k_apply_op(const Inst* __restrict__ Dp, const double* __restrict__ x,
                                                  double* __restrict__ y, int transpose) {
  INST_BEGIN
  const int i = xcd_node(I.n);
  if (i >= I.n) return;
  int i1, i2, i3;
  inst_coords(I.pde, i, I.N, I.dim, i1, i2, i3);
  y[i] = inst_op<double>(I, x, i, i1, i2, i3, transpose != 0);
}

// X = 0 (4n) for every active instance.
__global__ void __launch_bounds__(kBS) k_zero_x(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i < 4L * I.n) I.X[i] = 0.0;
}

}  // namespace ipm
