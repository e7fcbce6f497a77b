// Single-workgroup coarse V-cycle for the 3D Poisson levels (Sec. 4.2: the
// Schur approximation's factor A + M_hat inverted by the multigrid's coarsest
// levels, 15^3 and below), A the 7-point finite-difference stencil
// (6 x - the six neighbours) / h^2 or the trilinear Q1 stiffness
// (8/3 x - (the 12 edge neighbours) / 6 - (the 8 corner neighbours) / 12) / h^2
// (Sec. 2), plus the restricted reaction term m.
//
// The iterates are stored with a zero ring (pitch N + 2), so sweeps read
// their neighbours without boundary tests; each thread owns the same slots of
// a (N + 1)^3 slot cube at every sweep of a level (no division), and keeps
// the reaction term and 1/d of its nodes, and the top level's right-hand
// side, in registers for the whole cycle.  LDS per level: the two iterates
// (padded) and the right-hand side (compact, written by the restriction).
// Included by libipmpde.hip after kernels_mg.hip.

namespace ipm {

// Levels of the widest hierarchy (15, 7, 3, 1) and the top level's slots per
// thread (16^3 slots); the lower levels have at most 8^3 slots, one per thread.
constexpr int kF3Levels = 4;
constexpr int kF3TopSlots = 16 * 16 * 16 / kCoarseBS;

__host__ __device__ constexpr int coarse_f3_elems(int N) { return 2 * (N + 2) * (N + 2) * (N + 2) + N * N * N; }

// Loop over the thread's slots of an N^3 level (N + 1 a power of two): slot
// s = tid + j * kCoarseBS at (s mod M, (s / M) mod M, s / M^2), M = N + 1.
// Defines i (compact index) and p (index in the zero-ring layout).
#define F3_FOR(S, NN)                                                                   \
  {                                                                                     \
    const int k_ = 31 - __builtin_clz((NN) + 1), m_ = (1 << k_) - 1, P_ = (NN) + 2;     \
    _Pragma("unroll") for (int j = 0; j < (S); ++j) {                                   \
      const int s_ = tid + j * kCoarseBS;                                               \
      const int i1 = s_ & m_, i2 = (s_ >> k_) & m_, i3 = s_ >> (2 * k_);                \
      if (i1 < (NN) && i2 < (NN) && i3 < (NN)) {                                        \
        const int i = i1 + (NN) * (i2 + (NN) * i3);                                     \
        const int p = (i1 + 1) + P_ * ((i2 + 1) + P_ * (i3 + 1));                       \
        (void)i; (void)p;
#define F3_END \
      }        \
    }          \
  }

// Sum of the six neighbours of padded node p (pitch P), in the order of the
// generic stencil (x-1, x+1, y-1, y+1, z-1, z+1).
template <typename T>
__device__ __forceinline__ T f3_nb(const T* __restrict__ a, int p, int P) {
  const int PP = P * P;
  return ((((a[p - 1] + a[p + 1]) + a[p - P]) + a[p + P]) + a[p - PP]) + a[p + PP];
}

// Residual b - (A + m) x at padded node p of a level with 1/h^2 = ih2 (Q1:
// the 27-point stiffness, its sums in the order of the generic stencil).
template <typename T, bool Q1>
__device__ __forceinline__ T f3_res(const T* __restrict__ a, int p, int P, T ih2, T b, T m) {
  if constexpr (!Q1) {
    return b - (ih2 * ((T)6 * a[p] - f3_nb<T>(a, p, P)) + m * a[p]);
  } else {
    const int PP = P * P;
    T e = 0, c = 0;
#pragma unroll
    for (int o3 = -1; o3 <= 1; ++o3)
#pragma unroll
      for (int o2 = -1; o2 <= 1; ++o2)
#pragma unroll
        for (int o1 = -1; o1 <= 1; ++o1) {
          const int k = (o1 != 0) + (o2 != 0) + (o3 != 0);
          if (k < 2) continue;
          const T v = a[p + o1 + P * o2 + PP * o3];
          if (k == 2) e += v;
          else c += v;
        }
    return b - (ih2 * ((T)(8.0 / 3.0) * a[p] - (T)(1.0 / 6.0) * e - (T)(1.0 / 12.0) * c) + m * a[p]);
  }
}

// The operator's diagonal at a level of width M - 1 (h = 1 / M).
template <typename T, bool Q1>
__device__ __forceinline__ T f3_diag(int M) {
  if constexpr (!Q1) return (T)6 * (T)(M * M);
  const double h = 1.0 / M;
  return (T)(8.0 / (3.0 * h * h));
}

// Level q's geometry from the top width N0: width, pitch and LDS offset.
__device__ __forceinline__ void f3_level(int N0, int q, int& N, int& off) {
  off = 0;
  for (int r = 0; r < q; ++r) off += coarse_f3_elems(((N0 + 1) >> r) - 1);
  N = ((N0 + 1) >> q) - 1;
}

// Descent at level Q (compile-time, so the per-slot registers stay
// registers): nu_pre sweeps from zero, the residual, and its full weighting
// into level Q + 1's right-hand side.  rb, rm, rd: the thread's b, m, 1/d.
template <typename T, int S, bool Q1>
__device__ __forceinline__ void f3_down(T* lds, int N0, int Q, int nu_pre, T om, unsigned& alt, const T* rb,
                                        const T* rm, const T* rd) {
  const int tid = threadIdx.x;
  int N, off, Nc, offc;
  f3_level(N0, Q, N, off);
  f3_level(N0, Q + 1, Nc, offc);
  const int P = N + 2, P3 = P * P * P;
  const T ih2 = (T)((N + 1) * (N + 1));
  T* a = lds + off;
  T* c = a + P3;
  for (int s = 0; s < nu_pre; ++s) {
    if (s == 0) {
      F3_FOR(S, N) c[p] = om * rb[j] * rd[j]; F3_END
    } else {
      F3_FOR(S, N) c[p] = a[p] + om * f3_res<T, Q1>(a, p, P, ih2, rb[j], rm[j]) * rd[j]; F3_END
    }
    __syncthreads();
    T* t = a; a = c; c = t;
    alt ^= 1u << Q;
  }
  F3_FOR(S, N) c[p] = f3_res<T, Q1>(a, p, P, ih2, rb[j], rm[j]); F3_END
  __syncthreads();
  const int Pc = Nc + 2;
  T* bc = lds + offc + 2 * Pc * Pc * Pc;
  const int PP = P * P;
  F3_FOR(1, Nc)
    const int f = (2 * i1 + 2) + P * ((2 * i2 + 2) + P * (2 * i3 + 2));  // fine node 2j+1 (0-based), padded
    T acc = 0;
    for (int cc = -1; cc <= 1; ++cc)
      for (int bb = -1; bb <= 1; ++bb)
        for (int aa = -1; aa <= 1; ++aa) {
          const T w = (aa ? (T)0.25 : (T)0.5) * (bb ? (T)0.25 : (T)0.5) * (cc ? (T)0.25 : (T)0.5);
          acc += w * c[f + aa + P * bb + PP * cc];
        }
    bc[i] = acc;
  F3_END
  __syncthreads();
}

// Ascent at level Q: trilinear prolongation of level Q + 1's iterate added to
// the iterate, nu_post sweeps.
template <typename T, int S, bool Q1>
__device__ __forceinline__ void f3_up(T* lds, int N0, int Q, int nu_post, T om, unsigned& alt, const T* rb,
                                      const T* rm, const T* rd) {
  const int tid = threadIdx.x;
  int N, off, Nc, offc;
  f3_level(N0, Q, N, off);
  f3_level(N0, Q + 1, Nc, offc);
  const int P = N + 2, P3 = P * P * P, Pc = Nc + 2;
  const T ih2 = (T)((N + 1) * (N + 1));
  const int ca = (alt >> Q) & 1u;
  T* a = lds + off + ca * P3;
  T* c = lds + off + (1 - ca) * P3;
  const T* xc = lds + offc + ((alt >> (Q + 1)) & 1u) * Pc * Pc * Pc;
  F3_FOR(S, N)
    // fine 1-based F: coarse F/2 when even, its two neighbours when odd; the
    // padded coarse grid's ring (indices 0 and Nc + 1) is the zero boundary
    const int l1 = (i1 + 1) >> 1, h1 = (i1 + 2) >> 1, l2 = (i2 + 1) >> 1, h2 = (i2 + 2) >> 1;
    const int l3 = (i3 + 1) >> 1, h3 = (i3 + 2) >> 1;
    const T s0 = (xc[l1 + Pc * (l2 + Pc * l3)] + xc[h1 + Pc * (l2 + Pc * l3)]) +
                 (xc[l1 + Pc * (h2 + Pc * l3)] + xc[h1 + Pc * (h2 + Pc * l3)]);
    const T s1 = (xc[l1 + Pc * (l2 + Pc * h3)] + xc[h1 + Pc * (l2 + Pc * h3)]) +
                 (xc[l1 + Pc * (h2 + Pc * h3)] + xc[h1 + Pc * (h2 + Pc * h3)]);
    a[p] += (T)0.125 * (s0 + s1);
  F3_END
  __syncthreads();
  for (int s = 0; s < nu_post; ++s) {
    F3_FOR(S, N) c[p] = a[p] + om * f3_res<T, Q1>(a, p, P, ih2, rb[j], rm[j]) * rd[j]; F3_END
    __syncthreads();
    T* t = a; a = c; c = t;
    alt ^= 1u << Q;
  }
}

// Exact solve at the single-node level Q: x = b / d (slot 0 of thread 0).
template <typename T>
__device__ __forceinline__ void f3_solve1(T* lds, int N0, int Q, T b, T dinv) {
  int N, off;
  f3_level(N0, Q, N, off);
  if (threadIdx.x == 0) lds[off + 1 + 3 * (1 + 3 * 1)] = b * dinv;  // padded (1, 1, 1), pitch 3
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kCoarseBS) k_mg_coarse_f3(const Inst* __restrict__ Dp, int guard) {
  const Inst& I = Dp[blockIdx.z];
  int go = I.active;
  const int dim = I.dim, pde = I.pde, cl = I.coarse_lev, L = I.nlev, nu_pre = I.nu_pre, nu_post = I.nu_post;
  const double omega = I.omega;
  const KrylovCtrl* ctrl = I.ctrl;
  IPM_LOAD_TOGETHER(go, dim, pde, cl, L, nu_pre, nu_post, omega, ctrl);
  if (!go || dim != 3 || (pde != 0 && pde != 3)) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = (T*)lds_raw;
  const int tid = threadIdx.x, nl = L - cl;
  // global loads, in flight together with the stop flags: level cl's width,
  // right-hand side and output, every level's reaction term
  const int N0 = I.lv[cl].N;
  const T* __restrict__ bg = (const T*)I.lv[cl].b;
  T* __restrict__ xg = (T*)I.lv[cl].x;
  const T* __restrict__ mg0 = (const T*)I.lv[cl].mh;
  const T* __restrict__ mg1 = nl > 1 ? (const T*)I.lv[cl + 1].mh : nullptr;
  const T* __restrict__ mg2 = nl > 2 ? (const T*)I.lv[cl + 2].mh : nullptr;
  const T* __restrict__ mg3 = nl > 3 ? (const T*)I.lv[cl + 3].mh : nullptr;
  const int f_stop = ctrl->stop, f_want = ctrl->want_restart;
  T rb0[kF3TopSlots], rm0[kF3TopSlots], rd0[kF3TopSlots];
  F3_FOR(kF3TopSlots, N0) rb0[j] = bg[i]; rm0[j] = mg0[i]; F3_END
  // levels 1..3: one slot each (their widths are at most 7)
  T rb1[1] = {0}, rm1[1] = {0}, rd1[1] = {0}, rb2[1] = {0}, rm2[1] = {0}, rd2[1] = {0};
  T rb3[1] = {0}, rm3[1] = {0}, rd3[1] = {0};
  {
    const int N1 = ((N0 + 1) >> 1) - 1, N2 = ((N0 + 1) >> 2) - 1, N3 = ((N0 + 1) >> 3) - 1;
    if (nl > 1) { F3_FOR(1, N1) rm1[0] = mg1[i]; F3_END }
    if (nl > 2) { F3_FOR(1, N2) rm2[0] = mg2[i]; F3_END }
    if (nl > 3) { F3_FOR(1, N3) rm3[0] = mg3[i]; F3_END }
  }
  // uniform over the workgroup, before any LDS or global store
  if ((guard == 1 && f_stop) || (guard == 2 && !f_want)) return;
  // zero iterates (their rings stay zero) and right-hand sides
  {
    int tot = 0;
    for (int q = 0; q < nl; ++q) tot += coarse_f3_elems(((N0 + 1) >> q) - 1);
    for (int k = tid; k < tot; k += kCoarseBS) lds[k] = (T)0;
  }
  __syncthreads();
  const T om = (T)omega;
  // the cycle for the stencil Q1 (compile time, so the per-slot values stay in registers)
  auto cycle = [&](auto q1c) {
    constexpr bool Q1 = decltype(q1c)::value;
    // 1/d with d = the operator's diagonal + m (h = 1 / (N + 1))
#pragma unroll
    for (int j = 0; j < kF3TopSlots; ++j) rd0[j] = (T)1 / (f3_diag<T, Q1>(N0 + 1) + rm0[j]);
    const int M1 = (N0 + 1) >> 1, M2 = (N0 + 1) >> 2, M3 = (N0 + 1) >> 3;
    rd1[0] = (T)1 / (f3_diag<T, Q1>(M1) + rm1[0]);
    rd2[0] = (T)1 / (f3_diag<T, Q1>(M2) + rm2[0]);
    rd3[0] = (T)1 / (f3_diag<T, Q1>(M3) + rm3[0]);
    unsigned alt = 0;  // bit q: level q's iterate sits in x2
    // descent; level q's right-hand side below the top comes from the restriction
    auto rhs = [&](int q, T* rb) {
      int N, off;
      f3_level(N0, q, N, off);
      const T* b = lds + off + 2 * (N + 2) * (N + 2) * (N + 2);
      F3_FOR(1, N) rb[0] = b[i]; F3_END
    };
    if (nl > 1) f3_down<T, kF3TopSlots, Q1>(lds, N0, 0, nu_pre, om, alt, rb0, rm0, rd0);
    if (nl > 2) { rhs(1, rb1); f3_down<T, 1, Q1>(lds, N0, 1, nu_pre, om, alt, rb1, rm1, rd1); }
    if (nl > 3) { rhs(2, rb2); f3_down<T, 1, Q1>(lds, N0, 2, nu_pre, om, alt, rb2, rm2, rd2); }
    // the single-node level
    if (nl == 1) f3_solve1<T>(lds, N0, 0, rb0[0], rd0[0]);
    if (nl == 2) { rhs(1, rb1); f3_solve1<T>(lds, N0, 1, rb1[0], rd1[0]); }
    if (nl == 3) { rhs(2, rb2); f3_solve1<T>(lds, N0, 2, rb2[0], rd2[0]); }
    if (nl == 4) { rhs(3, rb3); f3_solve1<T>(lds, N0, 3, rb3[0], rd3[0]); }
    // ascent
    if (nl > 3) f3_up<T, 1, Q1>(lds, N0, 2, nu_post, om, alt, rb2, rm2, rd2);
    if (nl > 2) f3_up<T, 1, Q1>(lds, N0, 1, nu_post, om, alt, rb1, rm1, rd1);
    if (nl > 1) f3_up<T, kF3TopSlots, Q1>(lds, N0, 0, nu_post, om, alt, rb0, rm0, rd0);
    const T* a = lds + (alt & 1u) * (N0 + 2) * (N0 + 2) * (N0 + 2);
    F3_FOR(kF3TopSlots, N0) xg[i] = a[p]; F3_END
  };
  if (pde == 3) cycle(std::true_type{});
  else cycle(std::false_type{});
}
template __global__ void k_mg_coarse_f3<float>(const Inst*, int);
template __global__ void k_mg_coarse_f3<double>(const Inst*, int);

#undef F3_FOR
#undef F3_END

}  // namespace ipm
