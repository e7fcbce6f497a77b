// Kernels of right-preconditioned flexible GMRES (restarted), used with the
// block-triangular preconditioner P_T (Sec. 4) and for non-symmetric state
// operators.  Arnoldi with classical Gram-Schmidt applied twice, all
// reductions deterministic; the small Hessenberg least-squares problem is
// updated with Givens rotations by one thread on the device.
#include "common.h"

namespace ipm {

// w = K z (written to the next basis slot)
__global__ void __launch_bounds__(kBS) k_fg_matvec(Inst I, const double* __restrict__ z, double* __restrict__ w) {
  if (I.ctrl->stop) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  double o[4];
  saddle_rows(I, z, i, 1.0, o);
  const int n = I.n;
  w[i] = o[0]; w[n + i] = o[1]; w[2 * n + i] = o[2]; w[3 * n + i] = o[3];
}

// partials[k * nb + bx] = block part of <V_k, w>, k = blockIdx.y
__global__ void __launch_bounds__(kBS) k_fg_multidot(Inst I, const double* __restrict__ V, const double* __restrict__ w,
                                                     long n4) {
  if (I.ctrl->stop) return;
  __shared__ double smem[kBS / 64];
  const int k = blockIdx.y;
  const double* v = V + (size_t)k * n4;
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * kBS + threadIdx.x; i < n4; i += (long)gridDim.x * kBS) acc[0] += v[i] * w[i];
  block_reduce<kSum, 1, kBS>(acc, smem);
  if (threadIdx.x == 0) I.partials[(size_t)k * gridDim.x + blockIdx.x] = acc[0];
}

// hpass[k] = sum of partials (fixed order); hcol[k] += hpass[k]
__global__ void __launch_bounds__(kBS) k_fg_multidot_final(Inst I, int nk, int nb, int first) {
  KrylovCtrl* C = I.ctrl;
  if (C->stop) return;
  __shared__ double smem[kBS / 64];
  for (int k = 0; k < nk; ++k) {
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kBS) acc[0] += I.partials[(size_t)k * nb + b];
    block_reduce<kSum, 1, kBS>(acc, smem);
    if (threadIdx.x == 0) {
      C->hpass[k] = acc[0];
      C->hcol[k] = (first ? 0.0 : C->hcol[k]) + acc[0];
    }
  }
}

// w -= sum_k hpass[k] V_k
__global__ void __launch_bounds__(kBS) k_fg_orth(Inst I, const double* __restrict__ V, double* __restrict__ w, int nk,
                                                 long n4) {
  const KrylovCtrl* C = I.ctrl;
  if (C->stop) return;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  double acc = w[i];
  for (int k = 0; k < nk; ++k) acc -= C->hpass[k] * V[(size_t)k * n4 + i];
  w[i] = acc;
}

// |w|^2 -> hcol[j+1] = |w|, then the Givens update of column j and the
// residual estimate (last block, thread 0).
__global__ void __launch_bounds__(kBS) k_fg_norm_givens(Inst I, const double* __restrict__ w, long n4, int j,
                                                        double tol_abs) {
  KrylovCtrl* C = I.ctrl;
  if (C->stop) return;
  __shared__ double smem[kBS / 64];
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * kBS + threadIdx.x; i < n4; i += (long)gridDim.x * kBS) acc[0] += w[i] * w[i];
  if (!grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) || threadIdx.x != 0) return;
  double* h = C->hcol;
  h[j + 1] = sqrt(acc[0]);
  for (int i = 0; i < j; ++i) {
    const double t = C->cs[i] * h[i] + C->sn[i] * h[i + 1];
    h[i + 1] = -C->sn[i] * h[i] + C->cs[i] * h[i + 1];
    h[i] = t;
  }
  const double r = hypot(h[j], h[j + 1]);
  const double cs = r > 0.0 ? h[j] / r : 1.0, sn = r > 0.0 ? h[j + 1] / r : 0.0;
  C->cs[j] = cs;
  C->sn[j] = sn;
  const double hn = C->hcol[j + 1];
  h[j] = r;
  h[j + 1] = 0.0;
  for (int i = 0; i <= j; ++i) C->H[j * 64 + i] = h[i];
  C->g[j + 1] = -sn * C->g[j];
  C->g[j] = cs * C->g[j];
  C->j = j + 1;
  C->iter += 1;
  C->est = fabs(C->g[j + 1]);
  C->hcol[63] = hn;  // |w| before the rotation, for the normalization kernel
  if (!(r > 0.0) || !isfinite(r)) C->breakdown = 1;
  if (C->est <= tol_abs || !(hn > 0.0) || C->breakdown) C->stop = 1;
}

// v_{j+1} = w / |w|
__global__ void __launch_bounds__(kBS) k_fg_normalize(Inst I, double* __restrict__ w, long n4) {
  const KrylovCtrl* C = I.ctrl;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const double hn = C->hcol[63];
  if (hn > 0.0) w[i] = w[i] / hn;
}

// start of a cycle: v_0 = r / |r|, g = (|r|, 0, ...)
__global__ void __launch_bounds__(kBS) k_fg_start_norm(Inst I, const double* __restrict__ r, long n4) {
  __shared__ double smem[kBS / 64];
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * kBS + threadIdx.x; i < n4; i += (long)gridDim.x * kBS) acc[0] += r[i] * r[i];
  if (!grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) || threadIdx.x != 0) return;
  KrylovCtrl* C = I.ctrl;
  const double beta = sqrt(acc[0]);
  for (int k = 0; k < 64; ++k) C->g[k] = 0.0;
  C->g[0] = beta;
  C->hcol[63] = beta;
  C->j = 0;
  C->stop = beta > 0.0 ? 0 : 1;
  C->breakdown = 0;
}
__global__ void __launch_bounds__(kBS) k_fg_start_scale(Inst I, const double* __restrict__ r, double* __restrict__ v0,
                                                        long n4) {
  const KrylovCtrl* C = I.ctrl;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const double b = C->hcol[63];
  v0[i] = b > 0.0 ? r[i] / b : 0.0;
}

// back substitution H y = g over the k = ctrl->j completed steps (one thread)
__global__ void k_fg_solve_small(Inst I) {
  KrylovCtrl* C = I.ctrl;
  const int k = C->j;
  for (int i = k - 1; i >= 0; --i) {
    double s = C->g[i];
    for (int c = i + 1; c < k; ++c) s -= C->H[c * 64 + i] * C->y[c];
    C->y[i] = s / C->H[i * 64 + i];
  }
}

// x += sum_{i<k} y_i Z_i
__global__ void __launch_bounds__(kBS) k_fg_update_x(Inst I, const double* __restrict__ Z, double* __restrict__ X,
                                                     long n4) {
  const KrylovCtrl* C = I.ctrl;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const int k = C->j;
  double acc = X[i];
  for (int c = 0; c < k; ++c) acc += C->y[c] * Z[(size_t)c * n4 + i];
  X[i] = acc;
}

}  // namespace ipm
