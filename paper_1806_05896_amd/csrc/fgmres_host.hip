// Host loop of restarted, right-preconditioned FGMRES (included by libipmpde.hip).

static int ensure_fgmres(ipmpde_problem* P, int restart) {
  if (P->fV && P->f_restart >= restart) return IPMPDE_OK;
  const size_t n4 = 4 * (size_t)P->n;
  TRY(dalloc_t(P, &P->fV, (size_t)(restart + 1) * n4));
  TRY(dalloc_t(P, &P->fZ, (size_t)restart * n4));
  P->f_restart = restart;
  return IPMPDE_OK;
}

static int fg_multidot_blocks(long n4) { return std::min(nblk(n4), 256); }

__global__ void k_fg_reset_iter(KrylovCtrl* C) { C->iter = 0; }

template <typename T>
static void fgmres_step(ipmpde_problem* P, int pt, int j, double tol_abs, hipStream_t s) {
  const long n4 = 4L * P->n;
  const Inst& I = P->I;
  double* vj = P->fV + (size_t)j * n4;
  double* zj = P->fZ + (size_t)j * n4;
  double* w = P->fV + (size_t)(j + 1) * n4;
  precond_apply_t<T>(P, pt, vj, zj, 1, s);
  hipLaunchKernelGGL(k_fg_matvec, dim3(nblk(P->n)), dim3(kBS), 0, s, I, (const double*)zj, w);
  const int nbm = fg_multidot_blocks(n4);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_fg_multidot, dim3(nbm, j + 1), dim3(kBS), 0, s, I, (const double*)P->fV, (const double*)w, n4);
    hipLaunchKernelGGL(k_fg_multidot_final, dim3(1), dim3(kBS), 0, s, I, j + 1, nbm, pass == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_fg_orth, dim3(nblk(n4)), dim3(kBS), 0, s, I, (const double*)P->fV, w, j + 1, n4);
  }
  hipLaunchKernelGGL(k_fg_norm_givens, dim3(nbm), dim3(kBS), 0, s, I, (const double*)w, n4, j, tol_abs);
  hipLaunchKernelGGL(k_fg_normalize, dim3(nblk(n4)), dim3(kBS), 0, s, I, w, n4);
}

template <typename T>
static int fgmres_solve(ipmpde_problem* P, const ipmpde_options& o, hipStream_t s, int* its, double* relres) {
  const long n4 = 4L * P->n;
  const int m = o.restart;
  const int pt = o.precond == IPMPDE_PT;
  HIP_TRY(hipMemsetAsync(P->X, 0, n4 * sizeof(double), s));
  TRY(read_ctrl(P, s));
  const double bnorm = P->ctrl_h->bnorm;
  *its = 0;
  *relres = 0.0;
  if (!(bnorm > 0.0)) {
    if (bnorm != bnorm) return fail(IPMPDE_EBREAKDOWN, "NaN in the Newton right-hand side");
    return IPMPDE_OK;
  }
  const double tol_abs = o.krylov_tol * bnorm;
  const double* src = P->rhs;
  int total = 0;
  const int nbm = fg_multidot_blocks(n4);
  const int step = 4;
  for (int cycle = 0; cycle < 1000; ++cycle) {
    hipLaunchKernelGGL(k_fg_start_norm, dim3(nbm), dim3(kBS), 0, s, P->I, src, n4);
    hipLaunchKernelGGL(k_fg_start_scale, dim3(nblk(n4)), dim3(kBS), 0, s, P->I, src, P->fV, n4);
    hipLaunchKernelGGL(k_fg_reset_iter, dim3(1), dim3(1), 0, s, P->I.ctrl);
    TRY(read_ctrl(P, s));
    if (!P->ctrl_h->stop) {
      const int mm = std::min(m, o.krylov_maxit - total);
      for (int j0 = 0; j0 < mm; j0 += step) {
        for (int j = j0; j < std::min(j0 + step, mm); ++j) fgmres_step<T>(P, pt, j, tol_abs, s);
        HIP_TRY(hipGetLastError());
        TRY(read_ctrl(P, s));
        if (P->ctrl_h->stop) break;
      }
      hipLaunchKernelGGL(k_fg_solve_small, dim3(1), dim3(1), 0, s, P->I);
      hipLaunchKernelGGL(k_fg_update_x, dim3(nblk(n4)), dim3(kBS), 0, s, P->I, (const double*)P->fZ, P->X, n4);
    }
    hipLaunchKernelGGL(k_true_residual, dim3(nblk(P->n)), dim3(kBS), 0, s, P->I, P->X, P->rhs, P->R);
    TRY(read_ctrl(P, s));
    total += P->ctrl_h->j;
    const double rel = P->ctrl_h->rnorm / bnorm;
    *its = total;
    *relres = rel;
    if (rel <= std::max(o.krylov_tol, floor_factor() * P->ctrl_h->rfloor / bnorm)) return IPMPDE_OK;
    if (!(rel == rel)) return fail(IPMPDE_EBREAKDOWN, "NaN in the Krylov iterate");
    if (P->ctrl_h->breakdown && P->ctrl_h->j == 0) return fail(IPMPDE_EKRYLOV, "FGMRES breakdown");
    if (total >= o.krylov_maxit) return fail(IPMPDE_EKRYLOV, "Krylov iteration limit reached");
    src = P->R;
  }
  return fail(IPMPDE_EKRYLOV, "FGMRES did not converge");
}
