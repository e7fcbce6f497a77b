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

// Bilinear/trilinear interpolation of the coarse correction at fine node i.
template <typename T, bool SMALL = false>
__device__ __forceinline__ T prolong_node(const T* __restrict__ xc, int i, int Nf, int Nc, int dim) {
  int i1, i2, i3;
  if (SMALL) node_coords_small(i, Nf, dim, i1, i2, i3);
  else node_coords(i, Nf, dim, i1, i2, i3);
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

// guard 0: always run; 1: skip when the instance's Krylov loop stopped;
// 2: skip when the instance has no pending Krylov cycle.
__device__ __forceinline__ bool mg_skip(const Inst& I, int guard) {
  return (guard == 1 && I.ctrl->stop) || (guard == 2 && !I.ctrl->want_restart);
}
template <typename T>
__device__ __forceinline__ T* lvbuf(const Level& L, int sel) {
  return (T*)(sel ? L.x2 : L.x);
}

// One damped Jacobi sweep at level l (3D path): x[dst] = sweep(x[src]).
// Damped-Jacobi sweep (x_out = x_in + omega (b - (A + mh) x_in) / d, or
// omega b / d from a zero iterate) and residual b - (A + mh) x of the 3D
// finite-difference and Q1 levels, into the iterate buffer dst (for the
// residual the one the pre-smoothing left free, which the post-smoothing
// overwrites), in blocks of 16 x 4 x 4 nodes (one per thread): the block's input
// iterate with a one-node halo is staged in LDS (zero outside the grid), so
// the 7- or 27-point stencil is summed from LDS with no boundary tests or
// divisions, in the order of apply_op_s (the values are the same).
constexpr int kMb1 = 16, kMb2 = 4, kMb3 = 4;
static_assert(kMb1 * kMb2 * kMb3 == kBS, "one node per thread");
__host__ __device__ constexpr int mg3_blocks(int N) {
  return ((N + kMb1 - 1) / kMb1) * ((N + kMb2 - 1) / kMb2) * ((N + kMb3 - 1) / kMb3);
}
// (A x) at the block node li of the staged tile (pitches H1, H1*H2) for the
// 3D 7-point (pde 0) or Q1 27-point (pde 3) operator.
template <typename T, int H1, int H2>
__device__ __forceinline__ T mg3_apply(const T* __restrict__ a, int li, int pde, double h) {
  if (pde == 0) {
    const T ih2 = (T)(1.0 / (h * h));
    T nb = 0;
    nb += a[li - 1];
    nb += a[li + 1];
    nb += a[li - H1];
    nb += a[li + H1];
    nb += a[li - H1 * H2];
    nb += a[li + H1 * H2];
    return ih2 * ((T)6 * a[li] - nb);
  }
  T e = 0, c = 0;
#pragma unroll
  for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
    for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
        if (k < 2) continue;
        const T v = a[li + o1 + H1 * (o2 + H2 * o3)];
        if (k == 2) e += v;
        else c += v;
      }
  return (T)(1.0 / (h * h)) * ((T)(8.0 / 3.0) * a[li] - (T)(1.0 / 6.0) * e - (T)(1.0 / 12.0) * c);
}
// mode 0: Jacobi sweep (first: from a zero iterate) into x[dst]; mode 1: the
// residual b - (A + mh) x[src] into x[dst]; mode 2 (l = 0, between the two
// solves of S_hat^-1, Sec. 4.2): b = (M + Theta_y) x[src] with the Q1 mass
// (pde 3, summed as q1_mass does), else (1 + Theta_y) x[src] (x when the
// whole hierarchy ran in the coarse kernel).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_level3(const Inst* __restrict__ Dp, int l, int src, int dst, int first,
                                                   int mode, int guard) {
  INST_BEGIN
  if ((mode != 2 && l >= I.coarse_lev) || mg_skip(I, guard)) return;
  if (mode == 2 && I.coarse_lev == 0) src = 0;
  const Level& L = I.lv[l];
  const int N = L.N, pde = I.pde;
  int b = blockIdx.x;
  if ((gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);  // a slab of block layers per XCD
  if (b >= mg3_blocks(N)) return;
  const int nb1 = (N + kMb1 - 1) / kMb1, nb2 = (N + kMb2 - 1) / kMb2;
  const int b1 = b % nb1, bq = b / nb1, b2 = bq % nb2, b3 = bq / nb2;
  const int tid = threadIdx.x;
  const int t1 = tid % kMb1, t2 = (tid / kMb1) % kMb2, t3 = tid / (kMb1 * kMb2);
  const int i1 = b1 * kMb1 + t1, i2 = b2 * kMb2 + t2, i3 = b3 * kMb3 + t3;
  const bool own = i1 < N && i2 < N && i3 < N;
  const int i = own ? i1 + N * (i2 + N * i3) : 0;
  const T* __restrict__ xin = lvbuf<T>(L, src);
  T* __restrict__ xout = lvbuf<T>(L, dst);
  const T* __restrict__ bv = (const T*)L.b;
  const T* __restrict__ mh = (const T*)L.mh;
  const double h = L.h;
  const T om = (T)I.omega;
  if (mode == 2 && pde != 3) {
    if (own) ((T*)L.b)[i] = (T)(obs_w(I, i) + I.ty[i]) * xin[i];
    return;
  }
  if (mode == 0 && first) {
    if (!own) return;
    const T d = (T)op_diag(3, pde, h, I.eps, i1, i2) + mh[i];
    xout[i] = om * bv[i] / d;
    return;
  }
  constexpr int H1 = kMb1 + 2, H2 = kMb2 + 2, H3 = kMb3 + 2;
  __shared__ T sx[H1 * H2 * H3];
  for (int e = tid; e < H1 * H2 * H3; e += kBS) {
    const int e1 = e % H1, e2 = (e / H1) % H2, e3 = e / (H1 * H2);
    const int g1 = b1 * kMb1 - 1 + e1, g2 = b2 * kMb2 - 1 + e2, g3 = b3 * kMb3 - 1 + e3;
    sx[e] = ((unsigned)g1 < (unsigned)N && (unsigned)g2 < (unsigned)N && (unsigned)g3 < (unsigned)N)
                ? xin[g1 + N * (g2 + N * g3)]
                : (T)0;
  }
  __syncthreads();
  if (!own) return;
  const int li = (t1 + 1) + H1 * ((t2 + 1) + H2 * (t3 + 1));
  if (mode == 2) {
    T f = 0, e = 0, c = 0;
#pragma unroll
    for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
      for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
        for (int o1 = -1; o1 <= 1; ++o1) {
          const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
          if (k == 0) continue;
          const T v = sx[li + o1 + H1 * (o2 + H2 * o3)];
          if (k == 1) f += v;
          else if (k == 2) e += v;
          else c += v;
        }
    const T xi = sx[li];
    ((T*)L.b)[i] = ((T)64 * xi + (T)16 * f + (T)4 * e + c) * (T)(1.0 / 216.0) + (T)I.ty[i] * xi;
    return;
  }
  const T m = mh[i];
  const T xi = sx[li];
  const T Ax = mg3_apply<T, H1, H2>(sx, li, pde, h) + m * xi;
  if (mode == 1) {
    xout[i] = bv[i] - Ax;
    return;
  }
  const T d = (T)op_diag(3, pde, h, I.eps, i1, i2) + m;
  xout[i] = xi + om * (bv[i] - Ax) / d;
}

// Full-weighting restriction of level l's residual (in x[src]) to level
// l + 1's right-hand side: weights 1/4, 1/2, 1/4 per axis around fine node
// 2j + 1 (0-based) of coarse node j.
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_restrict_r(const Inst* __restrict__ Dp, int l, int src, int guard) {
  INST_BEGIN
  if (l >= I.coarse_lev || mg_skip(I, guard)) return;
  const Level& F = I.lv[l];
  const Level& C = I.lv[l + 1];
  const int ic = xcd_node(C.n);
  if (ic >= C.n) return;
  int j1, j2, j3;
  node_coords(ic, C.N, I.dim, j1, j2, j3);
  const T* __restrict__ r = lvbuf<T>(F, src);
  const int N = F.N;
  const int f = (2 * j1 + 1) + N * ((2 * j2 + 1) + (I.dim == 3 ? N * (2 * j3 + 1) : 0));
  const T wt[3] = {(T)0.25, (T)0.5, (T)0.25};
  T acc = 0;
  if (I.dim == 2) {
    for (int bb = -1; bb <= 1; ++bb)
      for (int a = -1; a <= 1; ++a) acc += wt[a + 1] * wt[bb + 1] * r[f + a + N * bb];
  } else {
    const int NN = N * N;
    for (int c = -1; c <= 1; ++c)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) acc += wt[a + 1] * wt[bb + 1] * wt[c + 1] * r[f + a + N * bb + NN * c];
  }
  ((T*)C.b)[ic] = acc;
}

// x[dst] at level l += P (level l+1's current iterate: its x if it is the
// coarse-kernel level, else x[csel]).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_prolong(const Inst* __restrict__ Dp, int l, int dst, int csel, int guard) {
  INST_BEGIN
  if (l >= I.coarse_lev || mg_skip(I, guard)) return;
  const Level& F = I.lv[l];
  const Level& C = I.lv[l + 1];
  const int i = xcd_node(F.n);
  if (i >= F.n) return;
  const T* xc = (l + 1 == I.coarse_lev) ? (const T*)C.x : lvbuf<T>(C, csel);
  lvbuf<T>(F, dst)[i] += prolong_node<T>(xc, i, F.N, C.N, I.dim);
}

// Poisson 2D specialization of the single-workgroup coarse V-cycle.  Per
// level the iterates are stored with a zero ring (pitch N+2), so sweeps need
// no boundary tests, and the diagonal d = 4/h^2 + M_hat and 1/d are staged
// once, so sweeps need no division:
//   x <- x + omega (b - d x + h^-2 (sum of neighbours)) / d.
// LDS per level: 2 (N+2)^2 + 3 N^2 elements (x, x2 padded; b, d, 1/d).
__host__ __device__ constexpr int coarse_p2_elems(int N) { return 2 * (N + 2) * (N + 2) + 3 * N * N; }

// Loop over the nodes (i1, i2) of an N x N level (N + 1 a power of two) with
// a power-of-two thread layout: no division.  Defines i (compact index) and
// p (index in the zero-ring padded layout of pitch P = N + 2).
#define P2_FOR(NN)                                                                   \
  {                                                                                  \
    const int sh_ = 31 - __builtin_clz((NN) + 1), step_ = kCoarseBS >> sh_;          \
    const int i1 = tid & ((1 << sh_) - 1);                                           \
    for (int i2 = tid >> sh_; i2 < (NN) && i1 < (NN); i2 += step_) {                 \
      const int i = i1 + (NN) * i2;                                                  \
      const int p = (i1 + 1) + ((NN) + 2) * (i2 + 1);                                \
      (void)i; (void)p;
#define P2_END \
    }          \
  }

// Largest coarse grid of the Poisson kernel (2D) and its nodes per thread.
constexpr int kCoarseP2MaxN = 63;
constexpr int kCoarseP2PerThread = (kCoarseP2MaxN * kCoarseP2MaxN + kCoarseBS - 1) / kCoarseBS;
// Nodes per thread of the widest coarse-kernel level in precision T: in FP64
// a 63 x 63 level's image (163 KB) exceeds the LDS budget, so the widest is
// 31 x 31 (961 nodes, one per thread).
template <typename T>
__host__ __device__ constexpr int p2_per_thread() { return sizeof(T) == 8 ? 1 : kCoarseP2PerThread; }

// Level l (0 = the first coarse-kernel level) of the LDS image of the
// Poisson coarse kernel holding element k of the image, or -1 past its end;
// widths halve from N0 (N_{l+1} = (N_l - 1) / 2).
__device__ __forceinline__ int coarse_p2_level(int k, int N0, int nl, int& N, int& off) {
  off = 0;
  N = N0;
  for (int l = 0; l < nl; ++l) {
    const int e = coarse_p2_elems(N);
    if (k < off + e) return l;
    off += e;
    N = (N - 1) / 2;
  }
  return -1;
}

// The LDS image of every instance's coarse levels after a Newton setup:
// per level zero iterates, a zero right-hand side, d = 4/h^2 + m and 1/d.
template <typename T>
__global__ void __launch_bounds__(kBS) k_coarse_pack(const Inst* __restrict__ Dp) {
  INST_BEGIN
  if (!I.coarse_p2) return;
  const int k = blockIdx.x * kBS + threadIdx.x;
  if (k >= I.cpack_elems) return;
  const int cl = I.coarse_lev;
  int N, off;
  const int l = coarse_p2_level(k, I.lv[cl].N, I.nlev - cl, N, off);
  T v = 0;
  if (l >= 0) {
    const int P = N + 2, n = N * N;
    const int r = k - off - 2 * P * P - n;  // index in [d | dinv]
    if (r >= 0) {
      const Level& Lv = I.lv[cl + l];
      const int i = r < n ? r : r - n;
      // the operator's diagonal: 4/h^2 (five-point) or 8/(3 h^2) (Q1), plus the reaction term
      const T dv = (I.coarse_p2 == 2 ? (T)(8.0 / (3.0 * Lv.h * Lv.h)) : (T)4 * (T)(1.0 / (Lv.h * Lv.h))) +
                   ((const T*)Lv.mh)[i];
      v = r < n ? dv : (T)1 / dv;
    }
  }
  ((T*)I.cpack)[k] = v;
}
template __global__ void k_coarse_pack<float>(const Inst*);
template __global__ void k_coarse_pack<double>(const Inst*);

// Offsets in the coarse image of a hierarchy whose top width is N0 with nl
// levels: the 7 x 7 level (-1: none) and the end of the levels, where the
// inverse of that level's operator follows (when there is one).
__host__ __device__ inline void coarse_p2_inv_offsets(int N0, int nl, int& off7, int& end) {
  off7 = -1;
  end = 0;
  for (int q = 0, N = N0; q < nl; ++q, N = (N - 1) / 2) {
    if (N == kCoarseInvN) off7 = end;
    end += coarse_p2_elems(N);
  }
}

// In-place inverse of the n x n matrix A (row-major, FP64, in LDS) by
// Gauss-Jordan elimination without pivoting (the coarse operators are
// diagonally dominant M-matrices), by the kBS threads of the workgroup; f is
// LDS scratch of n entries.
template <int n>
__device__ __forceinline__ void gauss_jordan_inverse(double* A, double* f) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    const double p = A[k * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += kBS) A[k * n + j] = j == k ? 1.0 / p : A[k * n + j] / p;
    for (int i = tid; i < n; i += kBS) f[i] = A[i * n + k];
    __syncthreads();
    for (int e = tid; e < n * n; e += kBS) {
      const int i = e / n, j = e - i * n;
      if (i != k) A[e] = j == k ? -f[i] * A[k * n + k] : A[e] - f[i] * A[k * n + j];
    }
    __syncthreads();
  }
}

// The inverse of the 7 x 7 level's operator A + M_hat (the five-point or Q1
// stencil divided by h^2 plus the reaction term, the image's diagonal d) by
// Gauss-Jordan elimination in FP64 (symmetric positive definite: no
// pivoting), symmetrized and stored after the image's levels, once per
// Newton setup; the coarse V-cycle then solves that level exactly.
template <typename T>
__global__ void __launch_bounds__(kBS) k_coarse_inv7(const Inst* __restrict__ Dp) {
  INST_BEGIN
  if (!I.coarse_p2) return;
  constexpr int M = kCoarseInvN, n = M * M, P = M + 2;
  int off7, end;
  coarse_p2_inv_offsets(I.lv[I.coarse_lev].N, I.nlev - I.coarse_lev, off7, end);
  if (off7 < 0 || I.cpack_elems < end + n * n) return;  // no 7 x 7 level, or no room for its inverse
  T* img = (T*)I.cpack;
  const T* d = img + off7 + 2 * P * P + n;
  __shared__ double A[n * n], f[n];
  const double h = 1.0 / (M + 1);
  const double off = I.coarse_p2 == 2 ? -1.0 / (3.0 * h * h) : -1.0 / (h * h);
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kBS) {
    const int r = e / n, c = e - r * n;
    const int dr1 = r % M - c % M, dr2 = r / M - c / M;
    const int a1 = dr1 < 0 ? -dr1 : dr1, a2 = dr2 < 0 ? -dr2 : dr2;
    const bool nb = I.coarse_p2 == 2 ? (a1 <= 1 && a2 <= 1 && r != c) : (a1 + a2 == 1);
    A[e] = r == c ? (double)d[r] : (nb ? off : 0.0);
  }
  __syncthreads();
  gauss_jordan_inverse<n>(A, f);
  T* inv = img + end;
  for (int e = tid; e < n * n; e += kBS) {
    const int i = e / n, j = e - i * n;
    inv[e] = (T)(0.5 * (A[e] + A[j * n + i]));
  }
}
template __global__ void k_coarse_inv7<float>(const Inst*);
template __global__ void k_coarse_inv7<double>(const Inst*);

// The LDS image of every convection-diffusion instance's coarse levels after
// a Newton setup (layout of k_mg_coarse_cd, kCoarseCDArrays arrays of n per
// level): zero iterates and right-hand side, the diagonal with the reaction
// term cd = op_diag + m, 1/cd and the four upwind neighbour coefficients of
// the node's row of A (the wind in FP64, rounded to T).
template <typename T>
__global__ void __launch_bounds__(kBS) k_coarse_pack_cd(const Inst* __restrict__ Dp) {
  INST_BEGIN
  if (I.coarse_p2 || I.pde != 1 || !I.cpack) return;
  const int k = blockIdx.x * kBS + threadIdx.x;
  if (k >= I.cpack_elems) return;
  const int cl = I.coarse_lev;
  int off = 0, q = -1;
  for (int l = cl; l < I.nlev; ++l) {
    const int e = kCoarseCDArrays * I.lv[l].n;
    if (k < off + e) {
      q = l;
      break;
    }
    off += e;
  }
  T v = 0;
  if (q >= 0) {
    const Level& Lv = I.lv[q];
    const int n = Lv.n, N = Lv.N, r = k - off, a = r / n, i = r - a * n;
    if (a >= 3) {
      const int j1 = i % N, j2 = i / N;
      const double h = Lv.h, ed = I.eps / (h * h), ih = 1.0 / h;
      double w1, w2;
      wind((j1 + 1) * h, (j2 + 1) * h, w1, w2);
      const T cd = (T)(4.0 * ed + (fabs(w1) + fabs(w2)) * ih) + ((const T*)Lv.mh)[i];
      switch (a) {
        case 3: v = cd; break;
        case 4: v = (T)1 / cd; break;
        case 5: v = (T)(-ed - fmax(w1, 0.0) * ih); break;
        case 6: v = (T)(-ed + fmin(w1, 0.0) * ih); break;
        case 7: v = (T)(-ed - fmax(w2, 0.0) * ih); break;
        default: v = (T)(-ed + fmin(w2, 0.0) * ih); break;
      }
    }
  }
  ((T*)I.cpack)[k] = v;
}
template __global__ void k_coarse_pack_cd<float>(const Inst*);
template __global__ void k_coarse_pack_cd<double>(const Inst*);

// Offsets in a convection-diffusion coarse image of nl levels from width N0:
// the 7 x 7 level (-1: none) and the end of the levels, where the inverse of
// that level's operator follows (when the image has room for it).
__host__ __device__ inline void coarse_cd_inv_offsets(int N0, int nl, int& off7, int& end) {
  off7 = -1;
  end = 0;
  for (int q = 0, N = N0; q < nl; ++q, N = (N - 1) / 2) {
    if (N == kCoarseInvN) off7 = end;
    end += kCoarseCDArrays * N * N;
  }
}

// The inverse of the 7 x 7 convection-diffusion level's operator (upwind
// stencil plus reaction term, from the image's cd and neighbour
// coefficients) by Gauss-Jordan in FP64, stored row-major after the image's
// levels, once per Newton setup; the coarse V-cycle then solves that level
// exactly, with the inverse or its transpose.
template <typename T>
__global__ void __launch_bounds__(kBS) k_coarse_inv7_cd(const Inst* __restrict__ Dp) {
  INST_BEGIN
  if (I.coarse_p2 || I.pde != 1 || !I.cpack) return;
  constexpr int M = kCoarseInvN, n = M * M;
  int off7, end;
  coarse_cd_inv_offsets(I.lv[I.coarse_lev].N, I.nlev - I.coarse_lev, off7, end);
  if (off7 < 0 || I.cpack_elems < end + n * n) return;
  T* img = (T*)I.cpack;
  const T* cf = img + off7 + 3 * n;  // cd | 1/cd | cW | cE | cS | cN
  __shared__ double A[n * n], f[n];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kBS) {
    const int r = e / n, c = e - r * n, r1 = r % M;
    double v = 0.0;
    if (c == r) v = (double)cf[r];
    else if (c == r - 1 && r1 > 0) v = (double)cf[2 * n + r];
    else if (c == r + 1 && r1 < M - 1) v = (double)cf[3 * n + r];
    else if (c == r - M) v = (double)cf[4 * n + r];
    else if (c == r + M) v = (double)cf[5 * n + r];
    A[e] = v;
  }
  __syncthreads();
  gauss_jordan_inverse<n>(A, f);
  T* inv = img + end;
  for (int e = tid; e < n * n; e += kBS) inv[e] = (T)A[e];
}
template __global__ void k_coarse_inv7_cd<float>(const Inst*);
template __global__ void k_coarse_inv7_cd<double>(const Inst*);

// Loop over the nodes of an N x N level with NT threads (thread t), as P2_FOR.
#define P2_FOR_T(NN, T_, NT_)                                                        \
  {                                                                                  \
    const int sh_ = 31 - __builtin_clz((NN) + 1), step_ = (NT_) >> sh_;             \
    const int i1 = (T_) & ((1 << sh_) - 1);                                          \
    for (int i2 = (T_) >> sh_; i2 < (NN) && i1 < (NN); i2 += step_) {                \
      const int i = i1 + (NN) * i2;                                                  \
      const int p = (i1 + 1) + ((NN) + 2) * (i2 + 1);                                \
      (void)i; (void)p;

// Off-diagonal part of the level operator at padded node p, with the sign
// flipped: (sum of the four neighbours) / h^2 for the five-point stencil
// (ST = 5), (sum of the eight neighbours) / (3 h^2) for the Q1 stiffness
// (ST = 9); ihs is 1/h^2 or 1/(3 h^2).
template <typename T, int ST>
__device__ __forceinline__ T p2_nb(const T* __restrict__ a, int p, int P, T ihs) {
  if constexpr (ST == 5) {
    return ihs * (a[p - 1] + a[p + 1] + a[p - P] + a[p + P]);
  } else {
    return ihs * ((a[p - 1] + a[p + 1] + a[p - P] + a[p + P]) +
                  (a[p - P - 1] + a[p - P + 1] + a[p + P - 1] + a[p + P + 1]));
  }
}

// Per-thread node loop of the coarse kernel's levels with the per-node
// values held in registers: the nodes of a thread at level N are
// (i1, i20 + j step), j < R (the P2_FOR_T layout, unrolled), and R nodes per
// thread cover the widest level (R NT >= N (N + 1)).
#define P2_FOR_R(R_)                                                   \
  _Pragma("unroll") for (int j = 0; j < (R_); ++j) {                   \
    const int i2 = i20 + j * step;                                     \
    if (i2 < N && i1 < N) {                                            \
      const int i = i1 + N * i2;                                       \
      const int p = (i1 + 1) + P * (i2 + 1);                           \
      (void)i; (void)p;
#define P2_END_R \
    }            \
  }

// Descent at level l: nu_pre damped-Jacobi sweeps from zero, the residual and
// its full-weighting restriction to level l + 1's right-hand side.  With REG
// the right-hand side, d and 1/d of the thread's nodes are read from LDS once
// and kept in registers; without it every sweep reads them from LDS (fewer
// registers, for kernels that hold other state across the cycle).
template <typename T, int NT, int ST = 5, bool REG = true>
__device__ __forceinline__ void p2_down(int nu_pre, T* lds, const int* LN, const int* LOFF, const T* LIH2, int l,
                                        int tid, T om, unsigned& alt) {
  constexpr int R = p2_per_thread<T>();
  // the widest level in LDS: 63 x 63 in FP32, 31 x 31 in FP64 (the coarse level choice keeps to these)
  static_assert(R * NT >= (sizeof(T) == 8 ? 31 * 32 : kCoarseP2MaxN * (kCoarseP2MaxN + 1)), "nodes per thread");
  const int N = LN[l], P = N + 2, n = N * N;
  const T ih2 = ST == 5 ? LIH2[l] : LIH2[l] * (T)(1.0 / 3.0);
  T* a = lds + LOFF[l];
  T* c = a + P * P;
  const T* b = c + P * P;
  const T* d = b + n;
  const T* dinv = d + n;
  const int sh = 31 - __builtin_clz(N + 1), step = NT >> sh, i1 = tid & ((1 << sh) - 1), i20 = tid >> sh;
  if constexpr (REG) {
    T rb[R], rd[R], rdi[R];
    P2_FOR_R(R) rb[j] = b[i]; rd[j] = d[i]; rdi[j] = dinv[i]; P2_END_R
    for (int s = 0; s < nu_pre; ++s) {
      if (s == 0) {
        P2_FOR_R(R) c[p] = om * rb[j] * rdi[j]; P2_END_R
      } else {
        P2_FOR_R(R) c[p] = a[p] + om * (rb[j] - rd[j] * a[p] + p2_nb<T, ST>(a, p, P, ih2)) * rdi[j]; P2_END_R
      }
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
    P2_FOR_R(R) c[p] = rb[j] - rd[j] * a[p] + p2_nb<T, ST>(a, p, P, ih2); P2_END_R
  } else {
    for (int s = 0; s < nu_pre; ++s) {
      if (s == 0) {
        P2_FOR_T(N, tid, NT) c[p] = om * b[i] * dinv[i]; P2_END
      } else {
        P2_FOR_T(N, tid, NT) c[p] = a[p] + om * (b[i] - d[i] * a[p] + p2_nb<T, ST>(a, p, P, ih2)) * dinv[i]; P2_END
      }
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
    P2_FOR_T(N, tid, NT) c[p] = b[i] - d[i] * a[p] + p2_nb<T, ST>(a, p, P, ih2); P2_END
  }
  __syncthreads();
  const int Nc = LN[l + 1];
  T* bc = lds + LOFF[l + 1] + 2 * (Nc + 2) * (Nc + 2);
  {
    const int shc = 31 - __builtin_clz(Nc + 1), msk = (1 << shc) - 1, stepc = NT >> shc;
    const int j1 = tid & msk;
    for (int j2 = tid >> shc; j2 < Nc && j1 < Nc; j2 += stepc) {
      const int ic = j1 + Nc * j2;
      const int p = (2 * j1 + 2) + P * (2 * j2 + 2);  // fine node 2j+1 (0-based) in padded coordinates
      bc[ic] = (T)0.25 * c[p] + (T)0.125 * (c[p - 1] + c[p + 1] + c[p - P] + c[p + P]) +
               (T)0.0625 * (c[p - 1 - P] + c[p + 1 - P] + c[p - 1 + P] + c[p + 1 + P]);
    }
  }
  __syncthreads();
}

// Ascent at level l: bilinear prolongation of level l + 1's iterate (in xb
// when bit l + 1 of alt is set) added to the iterate, nu_post sweeps (the
// right-hand side, d and 1/d of the thread's nodes in registers with REG).
template <typename T, int NT, int ST = 5, bool REG = true>
__device__ __forceinline__ void p2_up(int nu_post, T* lds, const int* LN, const int* LOFF, const T* LIH2, int l,
                                      int tid, T om, unsigned& alt) {
  constexpr int R = p2_per_thread<T>();
  const int N = LN[l], P = N + 2, n = N * N;
  const int Nc = LN[l + 1], Pc = Nc + 2;
  const T ih2 = ST == 5 ? LIH2[l] : LIH2[l] * (T)(1.0 / 3.0);
  T* base = lds + LOFF[l];
  const int ca = (alt >> l) & 1u;
  T* a = base + ca * P * P;
  T* c = base + (1 - ca) * P * P;
  const T* b = base + 2 * P * P;
  const T* d = b + n;
  const T* dinv = d + n;
  const T* xc = lds + LOFF[l + 1] + ((alt >> (l + 1)) & 1u) * Pc * Pc;
  // bilinear interpolation: fine 1-based F maps to coarse F/2 (even) or the two neighbours (odd);
  // in padded coarse coordinates the boundary nodes are the zero ring
#define P2_PROLONG_ADD                                                                                          \
  {                                                                                                             \
    const int F1 = i1 + 1, F2 = i2 + 1;                                                                         \
    const int lo1 = F1 >> 1, hi1 = (F1 + 1) >> 1, lo2 = F2 >> 1, hi2 = (F2 + 1) >> 1;                           \
    a[F1 + P * F2] +=                                                                                           \
        (T)0.25 * (xc[lo1 + Pc * lo2] + xc[hi1 + Pc * lo2] + xc[lo1 + Pc * hi2] + xc[hi1 + Pc * hi2]);          \
  }
  if constexpr (REG) {
    const int sh = 31 - __builtin_clz(N + 1), step = NT >> sh, i1 = tid & ((1 << sh) - 1), i20 = tid >> sh;
    T rb[R], rd[R], rdi[R];
    P2_FOR_R(R)
      rb[j] = b[i]; rd[j] = d[i]; rdi[j] = dinv[i];
      P2_PROLONG_ADD
    P2_END_R
    __syncthreads();
    for (int s = 0; s < nu_post; ++s) {
      P2_FOR_R(R) c[p] = a[p] + om * (rb[j] - rd[j] * a[p] + p2_nb<T, ST>(a, p, P, ih2)) * rdi[j]; P2_END_R
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
  } else {
    P2_FOR_T(N, tid, NT) P2_PROLONG_ADD P2_END
    __syncthreads();
    for (int s = 0; s < nu_post; ++s) {
      P2_FOR_T(N, tid, NT) c[p] = a[p] + om * (b[i] - d[i] * a[p] + p2_nb<T, ST>(a, p, P, ih2)) * dinv[i]; P2_END
      __syncthreads();
      T* t = a; a = c; c = t;
      alt ^= 1u << l;
    }
  }
#undef P2_PROLONG_ADD
}

// The V-cycle of the Poisson coarse kernel on the LDS image (level tables
// LN, LOFF, LIH2 set, top-level right-hand side in place): pre-smoothing,
// residual and restriction down to the single-node grid, its exact solve,
// prolongation and post-smoothing back up.  Returns the top level's final
// iterate (padded layout) in LDS.
template <typename T, int ST = 5, bool REG = true>
__device__ __forceinline__ const T* coarse_p2_cycle(T* lds, const int* LN, const int* LOFF, const T* LIH2, int cl,
                                                    int L, T om, int nu_pre, int nu_post, const T* ainv7 = nullptr) {
  const int tid = threadIdx.x;
  unsigned alt = 0;  // bit l: level l's iterate sits in xb
  // with the inverse of the 7 x 7 level's operator (ainv7, row-major 49 x 49
  // in LDS) the descent stops there and that level is solved exactly
  int lx = L - 1;
  if (ainv7)
    for (int l = cl; l < L; ++l)
      if (LN[l] == kCoarseInvN) lx = l;
  for (int l = cl; l < lx; ++l) p2_down<T, kCoarseBS, ST, REG>(nu_pre, lds, LN, LOFF, LIH2, l, tid, om, alt);
  if (LN[lx] == kCoarseInvN && ainv7) {
    constexpr int n = kCoarseInvN * kCoarseInvN, P = kCoarseInvN + 2;
    // with no descent before it the right-hand side was written by the threads
    // owning its nodes in the sweeps, not by the rows' threads here
    if (lx == cl) __syncthreads();
    T* a = lds + LOFF[lx];
    const T* b = a + 2 * P * P;
    if (tid < n) {
      T acc = 0;
      for (int c = 0; c < n; ++c) acc += ainv7[tid * n + c] * b[c];
      a[(tid % kCoarseInvN + 1) + P * (tid / kCoarseInvN + 1)] = acc;
    }
    __syncthreads();
  } else {
    // coarsest grid (one node): exact solve
    const int l = lx, N = LN[l], P = N + 2, n = N * N;
    T* a = lds + LOFF[l];
    const T* b = a + 2 * P * P;
    const T* dinv = b + 2 * n;
    P2_FOR_T(N, tid, kCoarseBS) a[p] = b[i] * dinv[i]; P2_END
    __syncthreads();
  }
  for (int l = lx - 1; l >= cl; --l) p2_up<T, kCoarseBS, ST, REG>(nu_post, lds, LN, LOFF, LIH2, l, tid, om, alt);
  const int N = LN[cl], P = N + 2;
  return lds + LOFF[cl] + ((alt >> cl) & 1u) * P * P;
}

// Convection-diffusion (2D upwind) coarse levels in one workgroup.  Per level
// the operator's coefficients are evaluated once per launch (the wind in
// FP64, rounded to T) and staged in LDS: the diagonal with the reaction term
// cd = op_diag + m, its inverse, and the four neighbour coefficients of the
// node's row of A (west, east, south, north).  A row of A^T takes the
// neighbours' coefficients towards this node (the east neighbour's west
// coefficient, ...).  LDS per level: x, x2, b, cd, 1/cd, cW, cE, cS, cN
// (kCoarseCDArrays arrays of n).
// Levels of the widest coarse hierarchy (63, 31, 15, 7, 3, 1).
constexpr int kCoarseP2Levels = kCoarseLevels;

template <typename T>
__device__ __forceinline__ T cd_row(const T* __restrict__ x, const T* __restrict__ cf, int i, int i1, int i2, int N,
                                    int n, bool tr) {
  const T* cW = cf + 2 * n;
  const T* cE = cf + 3 * n;
  const T* cS = cf + 4 * n;
  const T* cN = cf + 5 * n;
  T r = cf[i] * x[i];
  if (!tr) {
    if (i1 > 0) r += cW[i] * x[i - 1];
    if (i1 < N - 1) r += cE[i] * x[i + 1];
    if (i2 > 0) r += cS[i] * x[i - N];
    if (i2 < N - 1) r += cN[i] * x[i + N];
  } else {
    if (i1 < N - 1) r += cW[i + 1] * x[i + 1];
    if (i1 > 0) r += cE[i - 1] * x[i - 1];
    if (i2 < N - 1) r += cS[i + N] * x[i + N];
    if (i2 > 0) r += cN[i - N] * x[i - N];
  }
  return r;
}

// Descent and ascent of the convection-diffusion coarse V-cycle at level l
// by the NT threads of the workgroup.
template <typename T, int NT>
__device__ __forceinline__ void cd_down(T* lds, const int* LN, const int* LOFF, int l, int tid, T om, int nu, bool tr,
                                        unsigned& alt) {
  const int N = LN[l], n = N * N;
  T* a = lds + LOFF[l];
  T* c = a + n;
  const T* B = a + 2 * n;
  const T* cf = a + 3 * n;
  for (int sw = 0; sw < nu; ++sw) {
    P2_FOR_T(N, tid, NT)
      c[i] = sw == 0 ? om * B[i] * cf[n + i] : a[i] + om * (B[i] - cd_row<T>(a, cf, i, i1, i2, N, n, tr)) * cf[n + i];
    P2_END
    __syncthreads();
    T* t = a; a = c; c = t;
    alt ^= 1u << l;
  }
  P2_FOR_T(N, tid, NT) c[i] = B[i] - cd_row<T>(a, cf, i, i1, i2, N, n, tr); P2_END
  __syncthreads();
  const int Nc = LN[l + 1];
  T* Bc = lds + LOFF[l + 1] + 2 * Nc * Nc;
  P2_FOR_T(Nc, tid, NT)
    const int f = (2 * i1 + 1) + N * (2 * i2 + 1);
    Bc[i] = (T)0.25 * c[f] + (T)0.125 * (c[f - 1] + c[f + 1] + c[f - N] + c[f + N]) +
            (T)0.0625 * (c[f - 1 - N] + c[f + 1 - N] + c[f - 1 + N] + c[f + 1 + N]);
  P2_END
  __syncthreads();
}

template <typename T, int NT>
__device__ __forceinline__ void cd_up(T* lds, const int* LN, const int* LOFF, int l, int tid, T om, int nu, bool tr,
                                      unsigned& alt) {
  const int N = LN[l], n = N * N, Nc = LN[l + 1];
  const int ca = (alt >> l) & 1u;
  T* a = lds + LOFF[l] + ca * n;
  T* c = lds + LOFF[l] + (1 - ca) * n;
  const T* B = lds + LOFF[l] + 2 * n;
  const T* cf = lds + LOFF[l] + 3 * n;
  const T* xc = lds + LOFF[l + 1] + ((alt >> (l + 1)) & 1u) * Nc * Nc;
  P2_FOR_T(N, tid, NT) a[i] += prolong_node<T, true>(xc, i, N, Nc, 2); P2_END
  __syncthreads();
  for (int sw = 0; sw < nu; ++sw) {
    P2_FOR_T(N, tid, NT) c[i] = a[i] + om * (B[i] - cd_row<T>(a, cf, i, i1, i2, N, n, tr)) * cf[n + i]; P2_END
    __syncthreads();
    T* t = a; a = c; c = t;
    alt ^= 1u << l;
  }
}

template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_mg_coarse_cd(const Inst* __restrict__ Dp, int transpose, int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int p2 = I.coarse_p2, pde = I.pde, cl = I.coarse_lev, L = I.nlev, N0 = I.cN0, nu_pre = I.nu_pre,
            nu_post = I.nu_post, elems = I.cpack_elems;
  const double omega = I.omega;
  const KrylovCtrl* ctrl = I.ctrl;
  const T* __restrict__ bg = (const T*)I.cb;
  T* __restrict__ xg = (T*)I.cx;
  const T* __restrict__ img = (const T*)I.cpack;
  IPM_LOAD_TOGETHER(go, p2, pde, cl, L, N0, nu_pre, nu_post, elems, omega, ctrl, bg, xg, img);
  if (!go || p2 || pde != 1) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int LN[kMaxLev], LOFF[kMaxLev];
  T* lds = (T*)lds_raw;
  const bool tr = transpose != 0;
  const int tid = threadIdx.x;
  const T om = (T)omega;
  // Staging, all global loads in flight together with the stop flag: the
  // levels' image (zero iterates and right-hand sides, the upwind
  // coefficients, d and 1/d, built by k_coarse_pack_cd at the Newton setup;
  // layout x | x2 | b | cd | 1/cd | cW | cE | cS | cN per level) in 16-byte
  // pieces, and the top level's right-hand side at the node this thread owns
  // in the sweeps (the widest level is at most 31 x 31: one node per thread).
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  constexpr int VE = 16 / (int)sizeof(T);
  constexpr int MAXV = (int)((150 * 1024 / 16 + kCoarseBS - 1) / kCoarseBS);
  typedef unsigned int piece_t __attribute__((ext_vector_type(4)));
  const bool vec = ((uintptr_t)img & 15) == 0;
  const int nvec = vec ? elems / VE : 0;
  piece_t rv[MAXV];
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    const int v = tid + j * kCoarseBS;
    if (v < nvec) rv[j] = reinterpret_cast<const piece_t*>(img)[v];
  }
  const int sh0 = 31 - __builtin_clz(N0 + 1), j1 = tid & ((1 << sh0) - 1), j2 = tid >> sh0;
  const bool own = j1 < N0 && j2 < N0;
  const T breg = own ? bg[j1 + N0 * j2] : (T)0;
  // uniform over the workgroup, before any LDS or global store
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    const int v = tid + j * kCoarseBS;
    if (v < nvec) reinterpret_cast<piece_t*>(lds)[v] = rv[j];
  }
  for (int k = nvec * VE + tid; k < elems; k += kCoarseBS) lds[k] = img[k];  // the tail (all of it if unaligned)
  if (tid < kCoarseP2Levels && cl + tid < L) {
    const int q = tid;
    int off = 0;
    for (int r = 0; r < q; ++r) {
      const int Nr = ((N0 + 1) >> r) - 1;
      off += kCoarseCDArrays * Nr * Nr;
    }
    LN[cl + q] = ((N0 + 1) >> q) - 1;
    LOFF[cl + q] = off;
  }
  __syncthreads();
  // the top level's right-hand side over the image's zeros, each node by the
  // thread that owns it in the sweeps (the only thread that reads it back)
  if (own) lds[2 * N0 * N0 + j1 + N0 * j2] = breg;
  // with the inverse of the 7 x 7 level's operator after the levels, the
  // descent stops there and that level is solved exactly (A^-T b for the
  // transposed operator)
  constexpr int n7 = kCoarseInvN * kCoarseInvN;
  int off7, end;
  coarse_cd_inv_offsets(N0, L - cl, off7, end);
  const bool inv = off7 >= 0 && elems >= end + n7 * n7;
  int lx = L - 1;
  if (inv)
    for (int q = 0; q < L - cl; ++q)
      if (((N0 + 1) >> q) - 1 == kCoarseInvN) lx = cl + q;
  unsigned alt = 0;  // bit l: level l's iterate sits in x2
  for (int l = cl; l < lx; ++l) cd_down<T, kCoarseBS>(lds, LN, LOFF, l, tid, om, nu_pre, tr, alt);
  if (inv) {
    // with no descent before it the right-hand side was written by the
    // threads owning its nodes, not by the rows' threads here
    if (lx == cl) __syncthreads();
    T* X = lds + LOFF[lx];
    const T* B = X + 2 * n7;
    const T* Ai = lds + end;
    if (tid < n7) {
      T acc = 0;
      for (int c = 0; c < n7; ++c) acc += (tr ? Ai[c * n7 + tid] : Ai[tid * n7 + c]) * B[c];
      X[tid] = acc;
    }
    __syncthreads();
  } else {
    const int N = LN[L - 1], n = N * N;
    T* X = lds + LOFF[L - 1];
    P2_FOR(N) X[i] = X[2 * n + i] * X[4 * n + i]; P2_END
    __syncthreads();
  }
  for (int l = lx - 1; l >= cl; --l) cd_up<T, kCoarseBS>(lds, LN, LOFF, l, tid, om, nu_post, tr, alt);
  const int N = LN[cl];
  const T* xs = lds + LOFF[cl] + ((alt >> cl) & 1u) * N * N;
  P2_FOR(N) xg[i] = xs[i]; P2_END
}
template __global__ void k_mg_coarse_cd<float>(const Inst*, int, int);
template __global__ void k_mg_coarse_cd<double>(const Inst*, int, int);


template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_mg_coarse_p2(const Inst* __restrict__ Dp, int guard) {
  static_assert(kCoarseP2Levels == 6, "the descriptor loads below name six levels");
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int kind = I.coarse_p2, cl = I.coarse_lev, L = I.nlev, N0 = I.cN0, nu_pre = I.nu_pre, nu_post = I.nu_post;
  const int elems = I.cpack_elems;
  const double omega = I.omega;
  const KrylovCtrl* ctrl = I.ctrl;
  const T* __restrict__ bg = (const T*)I.cb;
  T* __restrict__ xg = (T*)I.cx;
  const T* __restrict__ img = (const T*)I.cpack;
  const double ih0 = I.cih2[0], ih1 = I.cih2[1], ih2 = I.cih2[2], ih3 = I.cih2[3], ih4 = I.cih2[4], ih5 = I.cih2[5];
  IPM_LOAD_TOGETHER(go, kind, cl, L, N0, nu_pre, nu_post, elems, omega, ctrl, bg, xg, img, ih0, ih1, ih2, ih3, ih4,
                    ih5);
  if (!go || !kind) return;
  const double cih2[kCoarseP2Levels] = {ih0, ih1, ih2, ih3, ih4, ih5};
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int LN[kMaxLev], LOFF[kMaxLev];
  __shared__ T LIH2[kMaxLev];
  T* lds = (T*)lds_raw;
  const int tid = threadIdx.x;
  // Staging, all global loads in flight together with the stop flag: the
  // coarse levels' image (zero iterates and right-hand sides, d = 4/h^2 + m or
  // 8/(3 h^2) + m and 1/d of every level, built by k_coarse_pack at the Newton
  // setup) in 16-byte pieces, and level cl's right-hand side at the nodes
  // this thread owns in the sweeps.  The iterates' zero rings are never
  // written; their interiors and the lower levels' right-hand sides are
  // written before they are read.
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  constexpr int VE = 16 / (int)sizeof(T);                                // elements per piece
  constexpr int MAXV = (int)((150 * 1024 / 16 + kCoarseBS - 1) / kCoarseBS);  // pieces per thread (LDS budget)
  const bool vec = ((uintptr_t)img & 15) == 0;  // slot images start on 16 bytes (the host rounds the stride)
  const int nvec = vec ? elems / VE : 0;
  typedef unsigned int piece_t __attribute__((ext_vector_type(4)));
  piece_t rv[MAXV];
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    const int v = tid + j * kCoarseBS;
    if (v < nvec) rv[j] = reinterpret_cast<const piece_t*>(img)[v];
  }
  constexpr int R = p2_per_thread<T>();
  const int sh = 31 - __builtin_clz(N0 + 1), step = kCoarseBS >> sh, i1 = tid & ((1 << sh) - 1), i20 = tid >> sh;
  T breg[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i2 = i20 + j * step;
    if (i2 < N0 && i1 < N0) breg[j] = bg[i1 + N0 * i2];
  }
  // uniform over the workgroup, before any LDS or global store
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
#pragma unroll
  for (int j = 0; j < MAXV; ++j) {
    const int v = tid + j * kCoarseBS;
    if (v < nvec) reinterpret_cast<piece_t*>(lds)[v] = rv[j];
  }
  for (int k = nvec * VE + tid; k < elems; k += kCoarseBS) lds[k] = img[k];  // the tail (all of it if unaligned)
  if (tid < kCoarseP2Levels && cl + tid < L) {
    // level widths, offsets and 1/h^2 from the top width (h = 1 / (N + 1))
    const int q = tid;
    int off = 0;
    for (int r = 0; r < q; ++r) off += coarse_p2_elems(((N0 + 1) >> r) - 1);
    LN[cl + q] = ((N0 + 1) >> q) - 1;
    LOFF[cl + q] = off;
    LIH2[cl + q] = (T)cih2[q];
  }
  __syncthreads();
  {
    // level cl's right-hand side over the image's zeros: each node by the
    // thread that owns it in the sweeps, the only thread that reads it back
    T* b0 = lds + 2 * (N0 + 2) * (N0 + 2);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i2 = i20 + j * step;
      if (i2 < N0 && i1 < N0) b0[i1 + N0 * i2] = breg[j];
    }
  }
  // coarse_p2 2: the Q1 nine-point stiffness
  int off7, end;
  coarse_p2_inv_offsets(N0, L - cl, off7, end);
  // copied with the image, which holds it after its levels (the per-time-step
  // images of the heat equation do not: there the V-cycle runs to one node)
  const T* ainv7 = off7 >= 0 && elems >= end + kCoarseInvN * kCoarseInvN * kCoarseInvN * kCoarseInvN ? lds + end
                                                                                                   : nullptr;
  const T* a = kind == 2 ? coarse_p2_cycle<T, 9>(lds, LN, LOFF, LIH2, cl, L, (T)omega, nu_pre, nu_post, ainv7)
                         : coarse_p2_cycle<T, 5>(lds, LN, LOFF, LIH2, cl, L, (T)omega, nu_pre, nu_post, ainv7);
  {
    const int N = LN[cl];
    P2_FOR(N) xg[i] = a[p]; P2_END
  }
}
template __global__ void k_mg_coarse_p2<float>(const Inst*, int);
template __global__ void k_mg_coarse_p2<double>(const Inst*, int);

// Heat equation, whole hierarchy in one workgroup (every step's coarse_lev
// is 0, one V-cycle per step): a whole block substitution of L + M_hat
// (dir = 1: steps 0..nt-1) or of its transpose (dir = -1: nt-1..0) in one
// launch.  Step t's right-hand side takes the previous step's solution / tau
// (held in registers), its V-cycle runs on its LDS image, and its solution
// goes to its level-0 x; the arithmetic is that of k_heat_couple followed by
// k_mg_coarse_p2 per step.  The iterate areas of the image are copied once:
// every V-cycle writes each interior iterate value before reading it (the
// first pre-smoothing sweep starts from zero) and never writes the zero
// rings, so later steps copy only d and 1/d of each level.
// d and 1/d of every level of the largest image, and per thread.
// Per-step image elements the heat kernel reloads at every time step: the
// levels' d and 1/d, and the inverse of the 7 x 7 level's operator.
constexpr int kHeatInv = kCoarseInvN * kCoarseInvN * kCoarseInvN * kCoarseInvN;
constexpr int kHeatDD = 2 * (63 * 63 + 31 * 31 + 15 * 15 + 7 * 7 + 3 * 3 + 1) + kHeatInv;
constexpr int kHeatDD64 = 2 * (31 * 31 + 15 * 15 + 7 * 7 + 3 * 3 + 1) + kHeatInv;  // FP64: widest 31 (p2_per_thread)
template <typename T>
constexpr int heat_dd_per_thread() { return ((sizeof(T) == 8 ? kHeatDD64 : kHeatDD) + kCoarseBS - 1) / kCoarseBS; }

template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_heat_sweep_p2(const Inst* __restrict__ Dp, int dir, int guard) {
  INST_BEGIN
  if (mg_skip(I, guard)) return;
  // the step descriptors are read-only during the kernel: reading them
  // through the constant address space keeps their loads scalar (the
  // kernel's global stores would otherwise force vector reloads)
  typedef const __attribute__((address_space(4))) Inst CInst;
  CInst* steps = (CInst*)I.hsteps;
  const int nt = I.nt;
  CInst& I0 = steps[0];
  if (!I0.coarse_p2 || I0.coarse_lev != 0) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int LN[kMaxLev], LOFF[kMaxLev];
  __shared__ T LIH2[kMaxLev];
  T* lds = (T*)lds_raw;
  const int L = I0.nlev, nu_pre = I0.nu_pre, nu_post = I0.nu_post;
  const T om = (T)I0.omega;
  const double tau = I0.tau;
  const int tid = threadIdx.x;
  const int N0 = I0.lv[0].N, n0 = N0 * N0;
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
  // the inverse of each step's 7 x 7 level operator, when its image holds one
  // (the V-cycle then solves that level exactly)
  int off7, end;
  coarse_p2_inv_offsets(N0, L, off7, end);
  const bool inv = off7 >= 0 && I0.cpack_elems >= end + kHeatInv;
  // image offsets of this thread's share of the levels' d and 1/d and of the
  // inverse (-1: none), so that each step issues all its loads at once
  int ddo[heat_dd_per_thread<T>()];
#pragma unroll
  for (int j = 0; j < heat_dd_per_thread<T>(); ++j) {
    int e = tid + j * kCoarseBS, o = -1;
    for (int l = 0; l < L; ++l) {
      const int N = LN[l], m = 2 * N * N;
      if (e < m) {
        o = LOFF[l] + 2 * (N + 2) * (N + 2) + N * N + e;
        break;
      }
      e -= m;
    }
    // past the levels e counts from their end (every level was subtracted)
    if (o < 0 && inv && e < kHeatInv) o = end + e;
    ddo[j] = o;
  }
  // the next step's right-hand side and d, 1/d are loaded while the current
  // step's V-cycle runs (the barriers wait for LDS operations only)
  T xreg[p2_per_thread<T>()], bnext[p2_per_thread<T>()], ddnext[heat_dd_per_thread<T>()];
  auto prefetch = [&](CInst& Sn) {
    const T* __restrict__ bg = (const T*)Sn.lv[0].b;
    const T* __restrict__ pk = (const T*)Sn.cpack;
#pragma unroll
    for (int j = 0; j < p2_per_thread<T>(); ++j) {
      const int i = tid + j * kCoarseBS;
      bnext[j] = i < n0 ? bg[i] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < heat_dd_per_thread<T>(); ++j) ddnext[j] = ddo[j] >= 0 ? pk[ddo[j]] : (T)0;
  };
  prefetch(steps[dir > 0 ? 0 : nt - 1]);
  for (int k = 0; k < nt; ++k) {
    const int t = dir > 0 ? k : nt - 1 - k;
    CInst& St = steps[t];
    T breg[p2_per_thread<T>()];
#pragma unroll
    for (int j = 0; j < p2_per_thread<T>(); ++j) {
      T v = bnext[j];
      if (k > 0) v = (T)((double)v + (double)xreg[j] / tau);
      breg[j] = v;
    }
    if (k == 0) {
      const T* __restrict__ pk = (const T*)St.cpack;
      for (int e = tid; e < St.cpack_elems; e += kCoarseBS) lds[e] = pk[e];
    } else {
#pragma unroll
      for (int j = 0; j < heat_dd_per_thread<T>(); ++j)
        if (ddo[j] >= 0) lds[ddo[j]] = ddnext[j];
    }
    __syncthreads();
    {
      T* b = lds + 2 * (N0 + 2) * (N0 + 2);
#pragma unroll
      for (int j = 0; j < p2_per_thread<T>(); ++j) {
        const int i = tid + j * kCoarseBS;
        if (i < n0) b[i] = breg[j];
      }
    }
    __syncthreads();
    if (k + 1 < nt) prefetch(steps[dir > 0 ? t + 1 : t - 1]);
    const T* a = coarse_p2_cycle<T, 5, false>(lds, LN, LOFF, LIH2, 0, L, om, nu_pre, nu_post, inv ? lds + end : nullptr);
    T* xg = (T*)St.lv[0].x;
    {
      const int P = N0 + 2;
#pragma unroll
      for (int j = 0; j < p2_per_thread<T>(); ++j) {
        const int i = tid + j * kCoarseBS;
        T v = 0;
        if (i < n0) {
          const int i2 = i / N0, i1 = i - i2 * N0;
          v = a[(i1 + 1) + P * (i2 + 1)];
          xg[i] = v;
        }
        xreg[j] = v;
      }
    }
    __syncthreads();
  }
}
template __global__ void k_heat_sweep_p2<float>(const Inst*, int, int);
template __global__ void k_heat_sweep_p2<double>(const Inst*, int, int);

// b_0 = (1 + Theta_y) x between the two solves of S_hat^-1 (3D path); x is
// the first solve's level-0 output (x or x2 by outsel, x when the whole
// hierarchy ran in the coarse kernel).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_scale_ty(const Inst* __restrict__ Dp, int outsel, int guard) {
  INST_BEGIN
  if (mg_skip(I, guard)) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const T* x = (const T*)((I.coarse_lev == 0 || !outsel) ? I.lv[0].x : I.lv[0].x2);
  if (I.pde == 3) {  // Q1: the middle factor of S_hat is M + Theta_y (Sec. 4.2)
    int i1, i2, i3;
    node_coords(i, I.N, I.dim, i1, i2, i3);
    ((T*)I.lv[0].b)[i] = q1_mass<T>(x, i, i1, i2, i3, I.N, I.dim) + (T)I.ty[i] * x[i];
    return;
  }
  ((T*)I.lv[0].b)[i] = (T)(obs_w(I, i) + I.ty[i]) * x[i];
}

// Block substitution of the heat equation's L + M_hat (Sec. 4.4; the block
// below the diagonal is -I/tau): before the multigrid solve of time step t
// (descriptor of that step) its right-hand side takes the neighbouring
// step's solution, b_t += x_{t-dir} / tau, dir = 1 forward (L + M_hat),
// dir = -1 backward (the transpose).  Consecutive steps' arrays are n apart.
template <typename T>
__global__ void __launch_bounds__(kBS) k_heat_couple(const Inst* __restrict__ Dp, int dir, int outsel, int guard) {
  INST_BEGIN
  if (mg_skip(I, guard)) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const T* __restrict__ nb = mg_out<T>(I, outsel) - (ptrdiff_t)dir * I.n;
  T* __restrict__ b = (T*)I.lv[0].b;
  b[i] = (T)((double)b[i] + (double)nb[i] / I.tau);
}

// b_0 = (1 + Theta_y) x for the instances of a 2D batch whose whole
// hierarchy runs in the coarse kernel (the others scale inside their first
// descent kernel).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_scale_ty_small(const Inst* __restrict__ Dp, int guard) {
  INST_BEGIN
  if (I.coarse_lev != 0 || mg_skip(I, guard)) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  ((T*)I.lv[0].b)[i] = (T)(obs_w(I, i) + I.ty[i]) * ((const T*)I.lv[0].x)[i];
}

// Reaction term of the multigrid operator for the next solves (slot 0:
// M_hat, or M_r for P_Pi; 1: M_l = O + Theta_y; 2: zero, the operator L
// alone): the descriptors' level and coarse-image pointers move to the slot
// (stream ordered, so it also works inside captured graphs).  Slot 0 is the
// state the host copies of the descriptors assume.
__global__ void k_mg_select(Inst* __restrict__ Dp, int slot) {
  Inst& I = Dp[blockIdx.z];
  const int l = threadIdx.x;
  if (l < I.nlev) {
    Level& L = I.lv[l];
    L.mh = (char*)L.mhb + (size_t)slot * L.n * (I.mg_fp32 ? 4 : 8);
  }
  if (l == 0 && I.cpackb)
    I.cpack = (char*)I.cpackb + (size_t)slot * I.cpack_slot * (I.mg_fp32 ? 4 : 8);
}

// k-cycle multigrid solve of (A + M_hat) x = b at level 0 (vcycles = k > 1):
// x_1 = V b, x_{j+1} = x_j + V (b - (A + M_hat) x_j), V the V-cycle from a
// zero guess (symmetric, so the k-cycle operator is too).  After V-cycle j
// (output: the solution for j = 1, else a correction) this kernel forms
// s_j = s_{j-1} + output (s_0 = 0) in kc_s[j & 1] and the next right-hand
// side b - (A + M_hat) s_j into level 0's b (the solve's own right-hand side
// is kept in kc_b0 at j = 1).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_kc_resid(const Inst* __restrict__ Dp, int outsel, int transpose, int j,
                                                     int guard) {
  INST_BEGIN
  if (mg_skip(I, guard)) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  const Level& L0 = I.lv[0];
  const T* __restrict__ out = mg_out<T>(I, outsel);
  const T* __restrict__ sp = (const T*)I.kc_s[(j + 1) & 1];
  T* __restrict__ sn = (T*)I.kc_s[j & 1];
  T* __restrict__ b = (T*)L0.b;
  T* __restrict__ b0 = (T*)I.kc_b0;
  int i1, i2, i3;
  node_coords(i, L0.N, I.dim, i1, i2, i3);
  const bool tr = transpose != 0;
  T bo, si, ax;
  if (j == 1) {
    bo = b[i];
    b0[i] = bo;
    si = out[i];
    ax = apply_op<T>(out, i, i1, i2, i3, L0.N, I.dim, I.pde, L0.h, I.eps, tr);
  } else {
    bo = b0[i];
    si = sp[i] + out[i];
    ax = apply_op<T>(sp, i, i1, i2, i3, L0.N, I.dim, I.pde, L0.h, I.eps, tr) +
         apply_op<T>(out, i, i1, i2, i3, L0.N, I.dim, I.pde, L0.h, I.eps, tr);
  }
  sn[i] = si;
  b[i] = bo - (ax + ((const T*)L0.mh)[i] * si);
}

// End of a k-cycle solve: output = s_{k-1} + output (the last correction).
template <typename T>
__global__ void __launch_bounds__(kBS) k_mg_kc_final(const Inst* __restrict__ Dp, int outsel, int k, int guard) {
  INST_BEGIN
  if (mg_skip(I, guard)) return;
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= I.n) return;
  T* __restrict__ out = (T*)mg_out<T>(I, outsel);
  out[i] += ((const T*)I.kc_s[(k - 1) & 1])[i];
}

#define IPM_MG_INST(T)                                                              \
  template __global__ void k_mg_kc_resid<T>(const Inst*, int, int, int, int);         \
  template __global__ void k_mg_kc_final<T>(const Inst*, int, int, int);              \
  template __global__ void k_mg_level3<T>(const Inst*, int, int, int, int, int, int); \
  template __global__ void k_mg_restrict_r<T>(const Inst*, int, int, int);           \
  template __global__ void k_mg_prolong<T>(const Inst*, int, int, int, int);          \
  template __global__ void k_mg_scale_ty<T>(const Inst*, int, int);                   \
  template __global__ void k_mg_scale_ty_small<T>(const Inst*, int);                   \
  template __global__ void k_heat_couple<T>(const Inst*, int, int, int);
IPM_MG_INST(float)
IPM_MG_INST(double)
#undef IPM_MG_INST


// ---------------------------------------------------------------- fused 2D level kernels
//
// Generic 2D operator (convection-diffusion; the Poisson instances take the
// kernels specialised for the constant stencil).  Descent at level l: nu
// damped-Jacobi sweeps from a zero iterate, the residual, and its
// full-weighting restriction, for a tile of TC x TC coarse
// nodes in one workgroup (temporal blocking in LDS: the sweeps run on a
// region that shrinks by one node per sweep).  Writes the smoothed iterate
// of the tile's own fine nodes and the coarse right-hand side.
constexpr int kTC = 8;    // coarse nodes per tile side (down kernel)
constexpr int kTF = 16;   // fine nodes per tile side (up kernel)

__host__ __device__ constexpr int down_width(int nu) { return 2 * kTC + 1 + 2 * nu; }
__host__ __device__ constexpr int up_width(int nu) { return kTF + 2 * nu; }

template <typename T>
__device__ __forceinline__ T jacobi_lds(const T* __restrict__ xa, const T* __restrict__ bs, const T* __restrict__ ms,
                                        int li, int W, int g1, int g2, int N, int pde, double h, double eps,
                                        double omega, bool tr) {
  const T m = ms[li];
  const T d = (T)op_diag(2, pde, h, eps, g1, g2) + m;
  const T xi = xa[li];
  const T Ax = apply_op_s<T>(xa, li, g1, g2, 0, N, W, 0, 2, pde, h, eps, tr) + m * xi;
  return xi + (T)omega * (bs[li] - Ax) / d;
}

// bsrc: right-hand side of level l; if ty != nullptr the right-hand side is
// (1 + Theta_y) bsrc (start of the second solve of S_hat^-1, level 0 only).
template <typename T, int NU>
__global__ void __launch_bounds__(kBS) k_mg_down2d(const Inst* __restrict__ Dp, int l, int scaled, int transpose,
                                                   int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int p2 = I.coarse_p2, cl = I.coarse_lev, pde = I.pde;
  const KrylovCtrl* ctrl = I.ctrl;
  const int N = I.lv[l].N, Nc = I.lv[l + 1].N;
  const double h = I.lv[l].h, eps = I.eps, om = I.omega;
  // scaled (level 0 only): the right-hand side is (1 + Theta_y) times the
  // first solve's output (level 0's x2)
  const T* __restrict__ bsrc = (const T*)(scaled ? I.lv[l].x2 : I.lv[l].b);
  const double* __restrict__ ty = scaled ? I.ty : nullptr;
  const double* __restrict__ obs = I.obs;
  const T* __restrict__ mh = (const T*)I.lv[l].mh;
  T* __restrict__ xout = (T*)I.lv[l].x;
  T* __restrict__ bfine = (T*)I.lv[l].b;
  T* __restrict__ bcoarse = (T*)I.lv[l + 1].b;
  IPM_LOAD_TOGETHER(go, p2, cl, pde, ctrl, N, Nc, h, eps, om, bsrc, ty, obs, mh, xout, bfine, bcoarse);
  if (!go || p2 || l >= cl) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  if ((int)(blockIdx.x * kTC) >= Nc || (int)(blockIdx.y * kTC) >= Nc) return;
  constexpr int nu = NU;
  constexpr int W = down_width(NU);
  T* bs = (T*)lds_raw;
  T* ms = bs + W * W;
  T* xa = ms + W * W;
  T* xb = xa + W * W;
  const int J1 = blockIdx.x * kTC, J2 = blockIdx.y * kTC;
  const int o1 = 2 * J1 - nu, o2 = 2 * J2 - nu;  // global fine coords of LDS (0, 0)
  const bool tr = transpose != 0;
  const int tid = threadIdx.x;
  // the stop flag is requested with the tile's data and tested before the
  // first global store (the staging writes LDS only)
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  for (int k = tid; k < W * W; k += kBS) {
    const int g1 = o1 + k % W, g2 = o2 + k / W;
    T bv = 0, mv = 0;
    if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N) {
      const int gi = g1 + N * g2;
      bv = bsrc[gi];
      if (ty) bv = (T)((obs ? obs[gi] : 1.0) + ty[gi]) * bv;
      mv = mh[gi];
    }
    bs[k] = bv;
    ms[k] = mv;
  }
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  __syncthreads();
  if (ty) {
    // keep the scaled right-hand side for the ascent (the tile's own fine nodes)
    for (int k = tid; k < 4 * kTC * kTC; k += kBS) {
      const int q1 = nu + k % (2 * kTC), q2 = nu + k / (2 * kTC);
      const int g1 = o1 + q1, g2 = o2 + q2;
      if (g1 < N && g2 < N) bfine[g1 + N * g2] = bs[q1 + W * q2];
    }
  }
  // first sweep from zero on the whole region
  for (int k = tid; k < W * W; k += kBS) {
    const int g1 = o1 + k % W, g2 = o2 + k / W;
    T v = 0;
    if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N) v = (T)om * bs[k] / ((T)op_diag(2, pde, h, eps, g1, g2) + ms[k]);
    xa[k] = v;
  }
  __syncthreads();
  T* a = xa;
  T* c = xb;
#pragma unroll
  for (int s = 1; s < nu; ++s) {
    const int lo = s, hi = W - s;  // region shrinks by one node per sweep
    const int w = hi - lo;
    for (int k = tid; k < w * w; k += kBS) {
      const int q1 = lo + k % w, q2 = lo + k / w;
      const int li = q1 + W * q2;
      const int g1 = o1 + q1, g2 = o2 + q2;
      T v = 0;
      if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N) v = jacobi_lds<T>(a, bs, ms, li, W, g1, g2, N, pde, h, eps, om, tr);
      c[li] = v;
    }
    __syncthreads();
    T* t = a; a = c; c = t;
  }
  // write the tile's own fine nodes of the smoothed iterate
  for (int k = tid; k < 4 * kTC * kTC; k += kBS) {
    const int q1 = nu + k % (2 * kTC), q2 = nu + k / (2 * kTC);
    const int g1 = o1 + q1, g2 = o2 + q2;
    if (g1 < N && g2 < N) xout[g1 + N * g2] = a[q1 + W * q2];
  }
  // residual on the restriction stencil region [nu, W - nu) into c
  {
    const int lo = nu, w = 2 * kTC + 1;
    for (int k = tid; k < w * w; k += kBS) {
      const int q1 = lo + k % w, q2 = lo + k / w;
      const int li = q1 + W * q2;
      const int g1 = o1 + q1, g2 = o2 + q2;
      T r = 0;
      if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N)
        r = bs[li] - (apply_op_s<T>(a, li, g1, g2, 0, N, W, 0, 2, pde, h, eps, tr) + ms[li] * a[li]);
      c[li] = r;
    }
  }
  __syncthreads();
  // full weighting onto the tile's coarse nodes
  {
    const int j1 = tid % kTC, j2 = tid / kTC;
    const int c1 = J1 + j1, c2 = J2 + j2;
    if (tid < kTC * kTC && c1 < Nc && c2 < Nc) {
      const int q1 = nu + 2 * j1 + 1, q2 = nu + 2 * j2 + 1;  // fine 2c+1 in LDS coordinates
      const int li = q1 + W * q2;
      const T v = (T)0.25 * c[li] + (T)0.125 * (c[li - 1] + c[li + 1] + c[li - W] + c[li + W]) +
                  (T)0.0625 * (c[li - 1 - W] + c[li + 1 - W] + c[li - 1 + W] + c[li + 1 + W]);
      bcoarse[c1 + Nc * c2] = v;
    }
  }
}

// Ascent at level l: x = xpre + P xc, then nu damped-Jacobi sweeps, for a
// tile of TF x TF fine nodes (halo nu in LDS).
template <typename T, int NU>
__global__ void __launch_bounds__(kBS) k_mg_up2d(const Inst* __restrict__ Dp, int l, int transpose, int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int p2 = I.coarse_p2, cl = I.coarse_lev, pde = I.pde;
  const KrylovCtrl* ctrl = I.ctrl;
  const int N = I.lv[l].N, Nc = I.lv[l + 1].N;
  const double h = I.lv[l].h, eps = I.eps, om = I.omega;
  const void* xc1 = I.lv[l + 1].x;
  const void* xc2 = I.lv[l + 1].x2;
  const T* __restrict__ xpre = (const T*)I.lv[l].x;
  const T* __restrict__ mh = (const T*)I.lv[l].mh;
  const T* __restrict__ b = (const T*)I.lv[l].b;
  T* __restrict__ xout = (T*)I.lv[l].x2;
  IPM_LOAD_TOGETHER(go, p2, cl, pde, ctrl, N, Nc, h, eps, om, xc1, xc2, xpre, mh, b, xout);
  if (!go || p2 || l >= cl) return;
  // the coarse iterate: the coarse kernel's output at the coarsest level here
  const T* __restrict__ xc = (const T*)(l + 1 == cl ? xc1 : xc2);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  if ((int)(blockIdx.x * kTF) >= N || (int)(blockIdx.y * kTF) >= N) return;
  constexpr int nu = NU;
  constexpr int W = up_width(NU);
  T* bs = (T*)lds_raw;
  T* ms = bs + W * W;
  T* xa = ms + W * W;
  T* xb = xa + W * W;
  const int o1 = blockIdx.x * kTF - nu, o2 = blockIdx.y * kTF - nu;
  const bool tr = transpose != 0;
  const int tid = threadIdx.x;
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  for (int k = tid; k < W * W; k += kBS) {
    const int g1 = o1 + k % W, g2 = o2 + k / W;
    T bv = 0, mv = 0, xv = 0;
    if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N) {
      const int gi = g1 + N * g2;
      bv = b[gi];
      mv = mh[gi];
      xv = xpre[gi] + prolong_node<T>(xc, gi, N, Nc, 2);
    }
    bs[k] = bv;
    ms[k] = mv;
    xa[k] = xv;
  }
  // uniform over the workgroup
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  __syncthreads();
  T* a = xa;
  T* c = xb;
#pragma unroll
  for (int s = 0; s < nu; ++s) {
    const int lo = s + 1, hi = W - s - 1;
    const int w = hi - lo;
    for (int k = tid; k < w * w; k += kBS) {
      const int q1 = lo + k % w, q2 = lo + k / w;
      const int li = q1 + W * q2;
      const int g1 = o1 + q1, g2 = o2 + q2;
      T v = 0;
      if (g1 >= 0 && g1 < N && g2 >= 0 && g2 < N) v = jacobi_lds<T>(a, bs, ms, li, W, g1, g2, N, pde, h, eps, om, tr);
      c[li] = v;
    }
    __syncthreads();
    T* t = a; a = c; c = t;
  }
  for (int k = tid; k < kTF * kTF; k += kBS) {
    const int q1 = nu + k % kTF, q2 = nu + k / kTF;
    const int g1 = o1 + q1, g2 = o2 + q2;
    if (g1 < N && g2 < N) xout[g1 + N * g2] = a[q1 + W * q2];
  }
}

#define IPM_MG2_INST(T, NU)                                                        \
  template __global__ void k_mg_down2d<T, NU>(const Inst*, int, int, int, int);  \
  template __global__ void k_mg_up2d<T, NU>(const Inst*, int, int, int);
#define IPM_MG2_INST_ALL(T) IPM_MG2_INST(T, 1) IPM_MG2_INST(T, 2) IPM_MG2_INST(T, 3) IPM_MG2_INST(T, 4) \
  IPM_MG2_INST(T, 5) IPM_MG2_INST(T, 6)
IPM_MG2_INST_ALL(float)
IPM_MG2_INST_ALL(double)
#undef IPM_MG2_INST_ALL
#undef IPM_MG2_INST

}  // namespace ipm
