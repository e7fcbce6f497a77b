// Kernel timing entry point (included by libipmpde.hip): launches one hot
// kernel back to back between two HIP events on the caller's stream.

template <typename T>
static double vcycle_bytes(const Inst& I) {
  // algorithmic bytes of one V-cycle: every grid-level sweep reads x, b, M_hat
  // and writes x (the first reads b, M_hat only); restriction reads x, b, M_hat
  // and writes the coarse b; prolongation reads the coarse x and updates x;
  // the single-workgroup kernel reads b and the level diagonals and writes x.
  const double e = sizeof(T);
  double b = 0;
  for (int l = 0; l < I.coarse_lev; ++l) {
    const double n = I.lv[l].n, nc = I.lv[l + 1].n;
    b += (3 * n + (I.nu_pre - 1) * 4 * n) * e;     // pre-smoothing
    b += (3 * n + nc) * e;                         // residual + restriction
    b += (2 * n + nc) * e;                         // prolongation + correction
    b += I.nu_post * 4 * n * e;                    // post-smoothing
  }
  for (int l = I.coarse_lev; l < I.nlev; ++l) b += I.lv[l].n * e;  // coarse diagonals (M_hat)
  b += 2 * I.lv[I.coarse_lev].n * e;
  return b;
}

template <typename T>
static void launch_down(ipmpde_problem* P, hipStream_t s) {
  const Inst& I = P->I;
  const size_t ldd = 4 * (size_t)down_width(I.nu_pre) * down_width(I.nu_pre) * sizeof(T);
  const int nt = div_up(I.lv[1].N, kTC);
  launch_down2d<T>(I.nu_pre, dim3(nt, nt), ldd, s, I, 0, (const T*)I.lv[0].b, (const double*)nullptr, (T*)I.lv[0].x, 0, 0);
}
template <typename T>
static void launch_up(ipmpde_problem* P, hipStream_t s) {
  const Inst& I = P->I;
  const size_t ldu = 4 * (size_t)up_width(I.nu_post) * up_width(I.nu_post) * sizeof(T);
  const int nt = div_up(I.lv[0].N, kTF);
  launch_up2d<T>(I.nu_post, dim3(nt, nt), ldu, s, I, 0, (const T*)I.lv[0].x, (const T*)I.lv[1].x2, (T*)I.lv[0].x2, 0, 0);
}

extern "C" int ipmpde_time_kernel(ipmpde_problem* P, const ipmpde_options* opts, int kernel, int reps,
                                  ipmpde_stream stream, double* avg_ms, double* bytes) {
  if (!P || !avg_ms || !bytes) return fail(IPMPDE_EINVAL, "NULL argument");
  if (reps < 1 || reps > 100000) return fail(IPMPDE_EINVAL, "reps out of range");
  if ((kernel == 4 || kernel == 5) && (P->dim != 2 || P->nlev < 2))
    return fail(IPMPDE_EINVAL, "fused level kernels exist for 2D grids with at least two levels");
  ipmpde_options o;
  resolve_opts(opts, &o);
  TRY(check_options(P, o));
  if (!P->setup_done || P->setup_fp32 != (o.mg_precision == IPMPDE_FP32))
    return fail(IPMPDE_EINVAL, "no Newton setup for this multigrid precision");
  select_mg(P, o);
  hipStream_t s = S(stream);
  const Inst& I = P->I;
  const double n = P->n;
  const bool f32 = o.mg_precision == IPMPDE_FP32;
  const double e = f32 ? 4.0 : 8.0;
  hipLaunchKernelGGL(k_ctrl_continue, dim3(1), dim3(1), 0, s, I.ctrl, 0.0);
  auto launch = [&]() {
    switch (kernel) {
      case 0:
        hipLaunchKernelGGL(k_saddle, dim3(nblk(P->n)), dim3(kBS), 0, s, I, (const double*)P->Z[0], P->Q);
        break;
      case 1:
        if (f32)
          hipLaunchKernelGGL(k_mg_jacobi<float>, dim3(nblk(P->n)), dim3(kBS), 0, s, I, 0, (const float*)I.lv[0].x,
                             (float*)I.lv[0].x2, 0, 0, 0);
        else
          hipLaunchKernelGGL(k_mg_jacobi<double>, dim3(nblk(P->n)), dim3(kBS), 0, s, I, 0, (const double*)I.lv[0].x,
                             (double*)I.lv[0].x2, 0, 0, 0);
        break;
      case 2:
        if (f32) hipLaunchKernelGGL(k_minres_k2<float>, dim3(nblk(P->n)), dim3(kBS), 0, s, I, (const double*)P->Q,
                                    (const double*)P->V[0], P->R, P->Z[1]);
        else hipLaunchKernelGGL(k_minres_k2<double>, dim3(nblk(P->n)), dim3(kBS), 0, s, I, (const double*)P->Q,
                                (const double*)P->V[0], P->R, P->Z[1]);
        break;
      case 3:
        if (f32) { float* x; mg_vcycle<float>(P, 0, 0, s, &x); }
        else { double* x; mg_vcycle<double>(P, 0, 0, s, &x); }
        break;
      case 6:
        hipLaunchKernelGGL(k_minres_k1, dim3(nblk(P->n)), dim3(kBS), 0, s, I, (const double*)P->Z[1],
                           (const double*)P->Z[0], P->W[0], (const double*)P->W[1], P->X, P->Q, P->KW[0],
                           (const double*)P->KW[1], P->Rt, 1);
        break;
      case 4:
        if (f32) launch_down<float>(P, s);
        else launch_down<double>(P, s);
        break;
      case 5:
        if (f32) launch_up<float>(P, s);
        else launch_up<double>(P, s);
        break;
    }
  };
  switch (kernel) {
    case 0: *bytes = 11.0 * n * 8; break;
    case 1: *bytes = 4.0 * n * e; break;
    case 2: *bytes = 22.0 * n * 8 + n * e; break;
    case 3: *bytes = f32 ? vcycle_bytes<float>(I) : vcycle_bytes<double>(I); break;
    case 4: *bytes = (3.0 * n + I.lv[1].n) * e; break;  // reads b, M_hat; writes x, coarse b
    case 5: *bytes = (4.0 * n + I.lv[1].n) * e; break;  // reads x, b, M_hat, coarse x; writes x
    // K1: reads z_j, z_{j-1}, w x2, x, q, Kw x2, r (36n) and Theta_y,w,v (3n); writes w, x, Kw, r, q (20n)
    case 6: *bytes = 59.0 * n * 8; break;

    default: return fail(IPMPDE_EINVAL, "unknown kernel id");
  }
  // the timed K2 writes into R instead of a Lanczos vector: copy something bounded there first
  if (kernel == 2) HIP_TRY(hipMemcpyAsync(P->R, P->V[1], 4 * (size_t)P->n * 8, hipMemcpyDeviceToDevice, s));
  launch();  // warm-up
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch();
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  *avg_ms = ms / reps;
  return IPMPDE_OK;
}
