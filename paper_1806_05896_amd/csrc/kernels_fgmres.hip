// Kernels of right-preconditioned flexible GMRES (restarted), used with the
// block-triangular preconditioner P_T (Sec. 4) and for non-symmetric state
// operators.  Arnoldi with classical Gram-Schmidt applied twice, all
// reductions deterministic; the small Hessenberg least-squares problem is
// updated with Givens rotations by one thread on the device.  Basis V_k and
// preconditioned vectors Z_k live in the instance's fV / fZ (4n each); every
// kernel serves instance blockIdx.z and each instance stops on its own.
#include "common.h"

namespace ipm {

__device__ __forceinline__ double* fg_v(const Inst& I, int k) { return I.fV + (size_t)k * 4 * I.n; }
__device__ __forceinline__ double* fg_z(const Inst& I, int k) { return I.fZ + (size_t)k * 4 * I.n; }

// V_{j+1} = K Z_j
__global__ void __launch_bounds__(kBS) k_fg_matvec(const Inst* __restrict__ Dp, int j) {
  INST_BEGIN
  if (I.ctrl->stop) return;
  const int i = xcd_node(I.n);
  if (i >= I.n) return;
  double o[4];
  saddle_rows(I, fg_z(I, j), i, 1.0, o);
  const int n = I.n;
  double* w = fg_v(I, j + 1);
  w[i] = o[0]; w[n + i] = o[1]; w[2 * n + i] = o[2]; w[3 * n + i] = o[3];
}

// partials[k * nb + bx] = block part of <V_k, V_{j+1}>, k = blockIdx.y
__global__ void __launch_bounds__(kBS) k_fg_multidot(const Inst* __restrict__ Dp, int j) {
  INST_BEGIN
  if (I.ctrl->stop) return;
  __shared__ double smem[kBS / 64];
  const int k = blockIdx.y;
  const long n4 = 4L * I.n;
  const double* __restrict__ v = fg_v(I, k);
  const double* __restrict__ w = fg_v(I, j + 1);
  double acc[1] = {0.0};
  // grid-stride loop, four strides' loads in flight before the (sequential) accumulation
  const long S = (long)gridDim.x * kBS;
  long i = (long)blockIdx.x * kBS + threadIdx.x;
  for (; i + 3 * S < n4; i += 4 * S) {
    const double v0 = v[i], v1 = v[i + S], v2 = v[i + 2 * S], v3 = v[i + 3 * S];
    const double w0 = w[i], w1 = w[i + S], w2 = w[i + 2 * S], w3 = w[i + 3 * S];
    acc[0] += v0 * w0;
    acc[0] += v1 * w1;
    acc[0] += v2 * w2;
    acc[0] += v3 * w3;
  }
  for (; i < n4; i += S) acc[0] += v[i] * w[i];
  block_reduce<kSum, 1, kBS>(acc, smem);
  if (threadIdx.x == 0) I.partials[(size_t)k * gridDim.x + blockIdx.x] = acc[0];
}

// hpass[k] = sum of partials (fixed order); hcol[k] (+)= hpass[k]
__global__ void __launch_bounds__(kBS) k_fg_multidot_final(const Inst* __restrict__ Dp, int nk, int nb, int first) {
  INST_BEGIN
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

// V_{j+1} -= sum_{k<=j} hpass[k] V_k
__global__ void __launch_bounds__(kBS) k_fg_orth(const Inst* __restrict__ Dp, int j) {
  INST_BEGIN
  const KrylovCtrl* C = I.ctrl;
  if (C->stop) return;
  const long n4 = 4L * I.n;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  double* w = fg_v(I, j + 1);
  const double* __restrict__ V = I.fV;
  const long stride = 4L * I.n;
  double acc = w[i];
  // eight basis vectors' loads in flight before the (sequential) updates
  int k = 0;
  for (; k + 8 <= j + 1; k += 8) {
    double vk[8], hk[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      vk[u] = V[(k + u) * stride + i];
      hk[u] = C->hpass[k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc -= hk[u] * vk[u];
  }
  for (; k <= j; ++k) acc -= C->hpass[k] * V[k * stride + i];
  w[i] = acc;
}

// |V_{j+1}|^2 -> hcol[j+1], then the Givens update of column j and the
// residual estimate (last block, thread 0); stop at tol |b|.
__global__ void __launch_bounds__(kBS) k_fg_norm_givens(const Inst* __restrict__ Dp, int j, double tol, int maxit) {
  INST_BEGIN
  KrylovCtrl* C = I.ctrl;
  if (C->stop) return;
  __shared__ double smem[kBS / 64];
  const long n4 = 4L * I.n;
  const double* w = fg_v(I, j + 1);
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * kBS + threadIdx.x; i < n4; i += (long)gridDim.x * kBS) acc[0] += w[i] * w[i];
  if (!grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) || threadIdx.x != 0) return;
  double* h = C->hcol;
  h[j + 1] = sqrt(acc[0]);
  const double hn = h[j + 1];
  for (int i = 0; i < j; ++i) {
    const double t = C->cs[i] * h[i] + C->sn[i] * h[i + 1];
    h[i + 1] = -C->sn[i] * h[i] + C->cs[i] * h[i + 1];
    h[i] = t;
  }
  const double r = hypot(h[j], h[j + 1]);
  const double cs = r > 0.0 ? h[j] / r : 1.0, sn = r > 0.0 ? h[j + 1] / r : 0.0;
  C->cs[j] = cs;
  C->sn[j] = sn;
  h[j] = r;
  h[j + 1] = 0.0;
  for (int i = 0; i <= j; ++i) C->H[j * 64 + i] = h[i];
  C->g[j + 1] = -sn * C->g[j];
  C->g[j] = cs * C->g[j];
  C->j = j + 1;
  C->est = fabs(C->g[j + 1]);
  C->hcol[63] = hn;  // |w| before the rotation, for the normalization kernel
  if (!(r > 0.0) || !isfinite(r)) C->breakdown = 1;
  if (C->est <= tol * C->bnorm || !(hn > 0.0) || C->breakdown || C->its_total + C->j >= maxit) C->stop = 1;
}

// V_{j+1} /= |V_{j+1}|
__global__ void __launch_bounds__(kBS) k_fg_normalize(const Inst* __restrict__ Dp, int j) {
  INST_BEGIN
  const KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;
  const long n4 = 4L * I.n;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const double hn = C->hcol[63];
  double* w = fg_v(I, j + 1);
  if (hn > 0.0) w[i] = w[i] / hn;
}

// start of a cycle from the residual (src 0: rhs, 1: R): |r| -> g = (|r|, 0, ...)
__global__ void __launch_bounds__(kBS) k_fg_start_norm(const Inst* __restrict__ Dp, int src) {
  INST_BEGIN
  KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;
  __shared__ double smem[kBS / 64];
  const long n4 = 4L * I.n;
  const double* r = src ? I.R : I.rhs;
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * kBS + threadIdx.x; i < n4; i += (long)gridDim.x * kBS) acc[0] += r[i] * r[i];
  if (!grid_reduce<kSum, 1, kBS>(acc, I.partials, I.counter, gridDim.x, blockIdx.x, smem) || threadIdx.x != 0) return;
  const double beta = sqrt(acc[0]);
  for (int k = 0; k < 64; ++k) C->g[k] = 0.0;
  C->g[0] = beta;
  C->hcol[63] = beta;
  C->j = 0;
  C->stop = beta > 0.0 ? 0 : 1;
  C->breakdown = 0;
}

// V_0 = r / |r|
__global__ void __launch_bounds__(kBS) k_fg_start_scale(const Inst* __restrict__ Dp, int src) {
  INST_BEGIN
  const KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;
  const long n4 = 4L * I.n;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const double* r = src ? I.R : I.rhs;
  const double b = C->hcol[63];
  I.fV[i] = b > 0.0 ? r[i] / b : 0.0;
}

// back substitution H y = g over the k = ctrl->j completed steps (one thread per instance)
__global__ void k_fg_solve_small(const Inst* __restrict__ Dp) {
  INST_BEGIN
  KrylovCtrl* C = I.ctrl;
  if (!C->want_restart || threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = C->j;
  for (int i = k - 1; i >= 0; --i) {
    double s = C->g[i];
    for (int c = i + 1; c < k; ++c) s -= C->H[c * 64 + i] * C->y[c];
    C->y[i] = s / C->H[i * 64 + i];
  }
}

// X += sum_{i<k} y_i Z_i
__global__ void __launch_bounds__(kBS) k_fg_update_x(const Inst* __restrict__ Dp) {
  INST_BEGIN
  const KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;
  const long n4 = 4L * I.n;
  const long i = (long)blockIdx.x * kBS + threadIdx.x;
  if (i >= n4) return;
  const int k = C->j;
  const double* __restrict__ Z = I.fZ;
  const long stride = 4L * I.n;
  double acc = I.X[i];
  // eight preconditioned vectors' loads in flight before the (sequential) updates
  int c = 0;
  for (; c + 8 <= k; c += 8) {
    double zc[8], yc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      zc[u] = Z[(c + u) * stride + i];
      yc[u] = C->y[c + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += yc[u] * zc[u];
  }
  for (; c < k; ++c) acc += C->y[c] * Z[c * stride + i];
  I.X[i] = acc;
}

}  // namespace ipm
