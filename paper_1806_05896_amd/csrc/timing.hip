// Kernel timing entry points (included by libipmpde.hip): one hot-path
// kernel launched back to back between two HIP events on the caller's
// stream, for a single problem or a batch (then one launch serves every
// instance and the bytes are summed over them).

template <typename T>
static double vcycle_bytes(const Inst& I) {
  // algorithmic bytes of one 2D V-cycle: per fine level the descent kernel
  // reads b and M_hat and writes x and the coarse b; the ascent kernel reads
  // x, b, M_hat and the coarse x and writes x2; the single-workgroup kernel
  // reads its top-level b and every level's M_hat and writes its x.
  const double e = sizeof(T);
  double b = 0;
  for (int l = 0; l < I.coarse_lev; ++l) {
    const double n = I.lv[l].n, nc = I.lv[l + 1].n;
    b += (3 * n + nc) * e + (4 * n + nc) * e;
  }
  for (int l = I.coarse_lev; l < I.nlev; ++l) b += I.lv[l].n * e;
  b += 2 * I.lv[I.coarse_lev].n * e;
  return b;
}

// Algorithmic bytes one launch of `kernel` moves for one instance.
static bool kernel_bytes(const Inst& I, int kernel, bool f32, double* bytes) {
  const double n = I.n, e = f32 ? 4.0 : 8.0;
  switch (kernel) {
    case 0: *bytes = 11.0 * n * 8; return true;
    // K2: reads q, v_j, v_{j-1}, r (16n) and Theta_y,w,v (3n); writes v, r (8n), z_y,w,v (3n), b_0
    case 2: *bytes = 30.0 * n * 8 + n * e; return true;
    case 3: *bytes = f32 ? vcycle_bytes<float>(I) : vcycle_bytes<double>(I); return true;
    case 4: *bytes = (3.0 * n + I.lv[1].n) * e; return true;  // reads b, M_hat; writes x, coarse b
    case 5: *bytes = (4.0 * n + I.lv[1].n) * e; return true;  // reads x, b, M_hat, coarse x; writes x2
    // K1: reads z_j, z_{j-1}, w x2, x (20n) and Theta_y,w,v (3n); writes w, x, q (12n)
    case 6: *bytes = 35.0 * n * 8; return true;
    // single-workgroup coarse kernel: its LDS image (Poisson) or the levels' M_hat, the top b and x
    case 7: {
      const int cl = I.coarse_lev;
      double img = 0;
      for (int l = cl; l < I.nlev; ++l) img += I.coarse_p2 ? coarse_p2_elems(I.lv[l].N) : I.lv[l].n;
      *bytes = (img + 2.0 * I.lv[cl].n) * e;
      return true;
    }
    default: return false;
  }
}

static int time_kernel_group(Group* G, const ipmpde_options& o, int kernel, int reps, hipStream_t s, double* avg_ms,
                             double* bytes) {
  if (reps < 1 || reps > 100000) return fail(IPMPDE_EINVAL, "reps out of range");
  for (int i = 0; i < G->count; ++i) {
    const ipmpde_problem* P = G->probs[i];
    if (!P->setup_done || P->setup_group != G || P->setup_fp32 != (o.mg_precision == IPMPDE_FP32))
      return fail(IPMPDE_EINVAL, "no Newton setup for this multigrid precision");
    if ((kernel == 3 || kernel == 4 || kernel == 5 || kernel == 7) &&
        (P->pde == IPMPDE_HEAT || P->pde == IPMPDE_POISSON_Q1))
      return fail(IPMPDE_EINVAL, "time kernels 0, 2 or 6 for heat-equation and Q1 problems");
    if ((kernel == 3 || kernel == 4 || kernel == 5) && (P->dim != 2 || P->nlev < 2))
      return fail(IPMPDE_EINVAL, "the fused level kernels exist for 2D grids with at least two levels");
  }
  if (kernel == 0 && G->count != 1) return fail(IPMPDE_EINVAL, "the saddle matvec is timed for single problems");
  for (int i = 0; i < G->count; ++i) G->H[i].active = 1;
  TRY(group_select(G, o));
  TRY(group_sync(G, s));
  const bool f32 = G->fp32;
  double total = 0;
  for (int i = 0; i < G->count; ++i) {
    double b = 0;
    if (!kernel_bytes(G->H[i], kernel, f32, &b)) return fail(IPMPDE_EINVAL, "unknown kernel id");
    total += b;
  }
  *bytes = total;
  const Inst& I0 = G->H[0];
  hipLaunchKernelGGL(k_ctrl_continue, dim3(1, 1, G->zc), dim3(64), 0, s, G->D);
  auto launch = [&]() {
    switch (kernel) {
      case 0:
        hipLaunchKernelGGL(k_saddle, gz(G, G->max_n), dim3(kBS), 0, s, G->D, (const double*)I0.Z[0], I0.Q);
        break;
      case 2:
        if (f32) hipLaunchKernelGGL(k_minres_k2<float>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, 1, 1);
        else hipLaunchKernelGGL(k_minres_k2<double>, gz(G, G->max_n), dim3(kBS), 0, s, G->D, 1, 1);
        break;
      case 3:
        if (f32) mg_vcycle<float>(G, 0, 0, 0, s);
        else mg_vcycle<double>(G, 0, 0, 0, s);
        break;
      case 4:
        if (f32) launch_down_level<float>(G, 0, 0, 0, 0, s);
        else launch_down_level<double>(G, 0, 0, 0, 0, s);
        break;
      case 5:
        if (f32) launch_up_level<float>(G, 0, 0, 0, s);
        else launch_up_level<double>(G, 0, 0, 0, s);
        break;
      case 6:
        hipLaunchKernelGGL(k_minres_k1, gz(G, G->max_n), dim3(kBS), 0, s, G->D, 1, 1);
        break;
      case 7:
        if (f32) launch_coarse<float>(G, 0, 0, s);
        else launch_coarse<double>(G, 0, 0, s);
        break;
    }
  };
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
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  *avg_ms = ms / reps;
  return IPMPDE_OK;
}

extern "C" int ipmpde_time_kernel(ipmpde_problem* P, const ipmpde_options* opts, int kernel, int reps,
                                  ipmpde_stream stream, double* avg_ms, double* bytes) {
  if (!P || !avg_ms || !bytes) return fail(IPMPDE_EINVAL, "NULL argument");
  ipmpde_options o;
  TRY(resolve_opts(opts, &o));
  if (!P->self) return fail(IPMPDE_EINVAL, "no Newton setup for this multigrid precision");
  return time_kernel_group(P->self, o, kernel, reps, S(stream), avg_ms, bytes);
}

extern "C" int ipmpde_batch_time_kernel(ipmpde_batch* B, const ipmpde_options* opts, int kernel, int reps,
                                        ipmpde_stream stream, double* avg_ms, double* bytes) {
  if (!B || !avg_ms || !bytes) return fail(IPMPDE_EINVAL, "NULL argument");
  ipmpde_options o;
  TRY(resolve_opts(opts, &o));
  return time_kernel_group(B->G, o, kernel, reps, S(stream), avg_ms, bytes);
}
