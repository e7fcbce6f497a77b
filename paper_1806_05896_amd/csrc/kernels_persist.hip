// Persistent MINRES for small instances: one workgroup runs a whole Krylov
// solve of eq. (NewtonSystem) with P_D (Sec. 4) -- every cycle, iteration,
// multigrid application and true-residual check -- for a 2D Poisson instance
// whose whole multigrid hierarchy fits the single-workgroup coarse kernel
// (N <= 63 with FP32 V-cycles, N <= 31 with FP64 ones).
//
// The arithmetic is that of the multi-kernel path (k_minres_init, K1, K2, the
// two V-cycles of S_hat^-1 with the (1 + Theta_y) scaling between them, K4,
// k_minres_flush, k_true_residual, k_krylov_mark), with block reductions in
// place of the grid reductions.  A small instance always takes this kernel,
// alone, in a batch or in an engine group, so its result does not depend on
// the company it is solved in.  What it saves is launch latency: the
// multi-kernel path pays about 17 launches per iteration, which for a few
// thousand nodes per field is nearly all of its time.  The Krylov vectors
// stay in global memory (a few hundred KB, L2 resident); the V-cycle's LDS
// image (zero iterates, d = 4/h^2 + M_hat, 1/d on every level) is built once
// per solve instead of once per V-cycle.
//
// Why only one workgroup: a multi-workgroup persistent kernel would need the
// Krylov vectors written by one workgroup to be visible to workgroups on
// other XCDs between phases, i.e. an agent-scope release/acquire that writes
// back and invalidates the XCD's L2 (measured here at about 3x the cost of a
// kernel boundary), so larger instances stay on the graph-captured
// multi-kernel path.
#include "common.h"

namespace ipm {

// Instances this kernel solves (the host launches it for MINRES + P_D only).
__device__ __forceinline__ bool minres_small_eligible(const Inst& I) {
  return I.coarse_p2 == 1 && I.coarse_lev == 0 && I.pde == 0 && !I.ppi && I.vcycles == 1 && I.obs == nullptr;
}

// Block sum of K values per thread, broadcast to every thread.
template <int K>
__device__ __forceinline__ void bsum(double (&v)[K], double* smem, double* bc) {
  block_reduce<kSum, K, kCoarseBS>(v, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) bc[k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = bc[k];
  __syncthreads();
}

// One application of S_hat^-1 = (A + M_hat)^-T (I + Theta_y) (A + M_hat)^-1
// (Sec. 4.2, eq. (SchurApprox)) by one V-cycle per solve on the LDS image:
// the right-hand side is level 0's b area; returns the output (padded layout
// of level 0's iterate area).
template <typename T>
__device__ __forceinline__ const T* small_schur(const Inst& I, T* lds, const int* LN, const int* LOFF, const T* LIH2,
                                                int L, const T* ainv7) {
  const int tid = threadIdx.x, N = LN[0], P = N + 2;
  T* b = lds + LOFF[0] + 2 * P * P;
  const T* a = coarse_p2_cycle<T, 5>(lds, LN, LOFF, LIH2, 0, L, (T)I.omega, I.nu_pre, I.nu_post, ainv7);
  // the scaled right-hand side of the second solve, as k_mg_scale_ty_small forms it
  P2_FOR(N) b[i] = (T)(1.0 + I.ty[i]) * a[p]; P2_END
  __syncthreads();
  return coarse_p2_cycle<T, 5>(lds, LN, LOFF, LIH2, 0, L, (T)I.omega, I.nu_pre, I.nu_post, ainv7);
}

template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_minres_small(const Inst* __restrict__ Dp, double tol, double ff,
                                                            int maxit, int max_cycles) {
  INST_BEGIN
  if (!minres_small_eligible(I)) return;
  KrylovCtrl* C = I.ctrl;
  if (!C->want_restart) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int LN[kMaxLev], LOFF[kMaxLev];
  __shared__ T LIH2[kMaxLev];
  __shared__ double red[3 * kCoarseBS / 64];
  __shared__ double bc[3];
  T* lds = (T*)lds_raw;
  const int tid = threadIdx.x, L = I.nlev, n = I.n, N0 = I.N;
  const int P0 = N0 + 2;
  // the LDS image: per level xa, xb (zero, padded), b, d, 1/d
  if (tid == 0) {
    int off = 0, N = N0;
    for (int l = 0; l < L; ++l) {
      LN[l] = N;
      LOFF[l] = off;
      const double h = 1.0 / (N + 1);
      LIH2[l] = (T)(1.0 / (h * h));
      off += coarse_p2_elems(N);
      N = (N - 1) / 2;
    }
  }
  __syncthreads();
  for (int l = 0; l < L; ++l) {
    const int N = LN[l], PP = (N + 2) * (N + 2), nl = N * N;
    T* x = lds + LOFF[l];
    for (int k = tid; k < 2 * PP; k += kCoarseBS) x[k] = (T)0;
    const double h = I.lv[l].h;
    const T diag = (T)4 * (T)(1.0 / (h * h));
    const T* __restrict__ m = (const T*)I.lv[l].mh;
    T* d = x + 2 * PP + nl;
    for (int i = tid; i < nl; i += kCoarseBS) {
      const T dv = diag + m[i];
      d[i] = dv;
      d[nl + i] = (T)1 / dv;
    }
  }
  // the inverse of the 7 x 7 level's operator, stored after the levels of the
  // Newton setup's image
  int off7, end;
  coarse_p2_inv_offsets(N0, L, off7, end);
  const T* ainv7 = nullptr;
  constexpr int n7 = kCoarseInvN * kCoarseInvN * kCoarseInvN * kCoarseInvN;
  if (off7 >= 0 && I.cpack_elems >= end + n7) {
    const T* __restrict__ src = (const T*)I.cpack + end;
    for (int e = tid; e < n7; e += kCoarseBS) lds[end + e] = src[e];
    ainv7 = lds + end;
  }
  __syncthreads();
  T* bmg = lds + LOFF[0] + 2 * P0 * P0;  // level 0's right-hand side (compact layout)

  const double bnorm = C->bnorm;
  int its_total = C->its_total;
  int failed = 0, breakdown = 0, converged = 0;
  double relres = 0.0;
  for (int cycle = 0; cycle < max_cycles && !converged && !failed; ++cycle) {
    // ---- start of a cycle (k_minres_init): v_1 = r, z_1 on the diagonal
    // blocks, the multigrid right-hand side r_p
    const double* __restrict__ r = cycle == 0 ? I.rhs : I.R;
    double acc[2] = {0.0, 0.0};
    for (int i = tid; i < n; i += kCoarseBS) {
      const double ry = r[i], rw = r[n + i], rv = r[2 * n + i], rp = r[3 * n + i];
      double zy, zw, zv;
      apply_A11_inv(I, i, ry, rw, rv, zy, zw, zv);
      I.V[1][i] = ry; I.V[1][n + i] = rw; I.V[1][2 * n + i] = rv; I.V[1][3 * n + i] = rp;
      I.Z[1][i] = zy; I.Z[1][n + i] = zw; I.Z[1][2 * n + i] = zv;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = k * n + i;
        I.V[0][q] = 0.0; I.W[0][q] = 0.0; I.W[1][q] = 0.0;
        I.Rt[q] = r[q];
      }
      bmg[i] = (T)rp;
      acc[0] += ry * zy + rw * zw + rv * zv;
    }
    {
      double t[1] = {acc[0]};
      bsum<1>(t, red, bc);
      acc[0] = t[0];
    }
    double dot_tmp = acc[0];
    {
      const T* out = small_schur<T>(I, lds, LN, LOFF, LIH2, L, ainv7);
      double t[1] = {0.0};
      P2_FOR(N0)
        const double z = (double)out[p];
        I.Z[1][3 * n + i] = z;
        t[0] += I.V[1][3 * n + i] * z;
      P2_END
      bsum<1>(t, red, bc);
      dot_tmp += t[0];
    }
    // the scalar recurrence, mode 0 (every thread holds the same values)
    double gamma_prev = 1.0, gamma, delta = 0.0, c_prev = 1.0, c = 1.0, s_prev = 0.0, s = 0.0, eta;
    double a1 = 1.0, a2 = 0.0, a3 = 0.0, coef_x = 0.0, gamma_w = 1.0, rs2 = 0.0, rc = 0.0;
    int iter = 0, pending = 0, rpend = 0, stop = 0;
    const double rtarget = tol * bnorm;
    if (!(dot_tmp > 0.0) || !isfinite(dot_tmp)) {
      breakdown = dot_tmp == 0.0 ? 0 : 1;
      gamma = 1.0;
      eta = 0.0;
      stop = 1;
    } else {
      gamma = sqrt(dot_tmp);
      eta = gamma;
    }
    // ---- iterations
    while (!stop) {
      const int par = (iter + 1) & 1;
      const double* __restrict__ Zc = I.Z[par];
      const double* __restrict__ Zp = I.Z[1 - par];
      double* __restrict__ Ws = I.W[1 - par];
      const double* __restrict__ Wo = I.W[par];
      // K1: pending direction/solution update, q = K z_j / gamma_j, delta_j
      double t1[1] = {0.0};
      const double sc = 1.0 / gamma;
      for (int i = tid; i < n; i += kCoarseBS) {
        if (pending) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int q = k * n + i;
            const double wi = (Zp[q] / gamma_w - a3 * Ws[q] - a2 * Wo[q]) / a1;
            Ws[q] = wi;
            I.X[q] += coef_x * wi;
          }
        }
        double o[4];
        saddle_rows(I, Zc, i, sc, o);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          I.Q[k * n + i] = o[k];
          t1[0] += o[k] * (Zc[k * n + i] * sc);
        }
      }
      bsum<1>(t1, red, bc);
      delta = t1[0];
      pending = 0;
      // K2: Lanczos vector, tracked residual, diagonal blocks of P_D, r_p for the multigrid
      const double* __restrict__ Vc = I.V[par];
      double* __restrict__ Vn = I.V[1 - par];
      double* __restrict__ Zn = I.Z[1 - par];
      const double cc1 = delta / gamma, cc2 = gamma / gamma_prev;
      double t2[2] = {0.0, 0.0};
      for (int i = tid; i < n; i += kCoarseBS) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = k * n + i;
          const double vc = Vc[q];
          v[k] = I.Q[q] - cc1 * vc - cc2 * Vn[q];
          Vn[q] = v[k];
          if (rpend) {
            const double rr = rs2 * I.Rt[q] + rc * vc;
            I.Rt[q] = rr;
            t2[1] += rr * rr;
          }
        }
        double zy, zw, zv;
        apply_A11_inv(I, i, v[0], v[1], v[2], zy, zw, zv);
        Zn[i] = zy; Zn[n + i] = zw; Zn[2 * n + i] = zv;
        bmg[i] = (T)v[3];
        t2[0] += v[0] * zy + v[1] * zw + v[2] * zv;
      }
      bsum<2>(t2, red, bc);
      double dotv = t2[0];
      if (rpend) {
        rpend = 0;
        const double rtrack = sqrt(t2[1]);
        if (rtrack <= rtarget || !(t2[1] == t2[1])) {
          stop = 1;
          break;
        }
      }
      // multigrid: z_{j+1,p} = S_hat^-1 v_{j+1,p}; K4: the rest of <v, z> and the recurrence
      {
        const T* out = small_schur<T>(I, lds, LN, LOFF, LIH2, L, ainv7);
        double t4[1] = {0.0};
        P2_FOR(N0)
          const double z = (double)out[p];
          Zn[3 * n + i] = z;
          t4[0] += Vn[3 * n + i] * z;
        P2_END
        bsum<1>(t4, red, bc);
        dotv += t4[0];
      }
      if (!(dotv >= 0.0) || !isfinite(dotv)) {
        breakdown = 1;
        stop = 1;
        pending = 0;
        break;
      }
      const double gn = sqrt(dotv);
      const double g = gamma, d = delta;
      const double b0 = c * d - c_prev * s * g;
      const double b1 = sqrt(b0 * b0 + gn * gn);
      const double b2 = s * d + c_prev * c * g;
      const double b3 = s_prev * g;
      const double cn = b0 / b1, sn = gn / b1;
      a1 = b1; a2 = b2; a3 = b3;
      coef_x = cn * eta;
      gamma_w = g;
      pending = 1;
      eta = -sn * eta;
      rs2 = sn * sn;
      rc = gn > 0.0 ? eta * cn / gn : 0.0;
      rpend = 1;
      c_prev = c; c = cn;
      s_prev = s; s = sn;
      gamma_prev = g; gamma = gn;
      iter += 1;
      if (gn == 0.0 || its_total + iter >= maxit || !isfinite(b1) || b1 == 0.0) stop = 1;
    }
    // ---- flush the pending update (k_minres_flush), with the parity of the last iteration
    if (pending) {
      const double* Zi = I.Z[iter & 1];
      double* Ws = I.W[iter & 1];
      const double* Wo = I.W[(iter + 1) & 1];
      for (int i = tid; i < n; i += kCoarseBS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = k * n + i;
          const double wi = (Zi[q] / gamma_w - a3 * Ws[q] - a2 * Wo[q]) / a1;
          Ws[q] = wi;
          I.X[q] += coef_x * wi;
        }
      }
      __syncthreads();
    }
    // ---- true residual R = rhs - K X and its rounding scale (k_true_residual)
    double tr[2] = {0.0, 0.0};
    for (int i = tid; i < n; i += kCoarseBS) {
      double o[4], m[4];
      saddle_rows(I, I.X, i, 1.0, o);
      saddle_rows_abs(I, I.X, i, m);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double bk = I.rhs[k * n + i];
        const double rk = bk - o[k];
        I.R[k * n + i] = rk;
        tr[0] += rk * rk;
        const double mk = m[k] + fabs(bk);
        tr[1] += mk * mk;
      }
    }
    bsum<2>(tr, red, bc);
    // ---- the cycle's verdict (k_krylov_mark)
    its_total += iter;
    relres = bnorm > 0.0 ? sqrt(tr[0]) / bnorm : 0.0;
    const double lim = fmax(tol, bnorm > 0.0 ? ff * sqrt(tr[1]) / bnorm : 0.0);
    if (relres <= lim) converged = 1;
    else if (!(relres == relres) || breakdown || its_total >= maxit) failed = 1;
    if (tid == 0) {
      C->rnorm = sqrt(tr[0]);
      C->rfloor = sqrt(tr[1]);
      C->iter = iter;
    }
  }
  if (tid == 0) {
    C->its_total = its_total;
    C->relres = relres;
    C->breakdown = breakdown;
    C->failed = converged ? 0 : 1;  // also a solve still missing the tolerance after the last cycle
    C->want_restart = 0;
    C->stop = 1;
    C->pending = 0;
    C->rpend = 0;
  }
}
template __global__ void k_minres_small<float>(const Inst*, double, double, int, int);
template __global__ void k_minres_small<double>(const Inst*, double, double, int, int);

}  // namespace ipm
