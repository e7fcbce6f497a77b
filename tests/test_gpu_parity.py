"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: operators and the saddle matvec are FP64 stencil sums, compared
at 1e-13 relative; Newton directions are compared through the oracle's
FP64 sparse matrix (relative residual <= 1e-9, the Krylov target 1e-10 plus
the conditioning slack of FP64 accumulation) and against the direct solve;
whole IPM runs must match the oracle's control and state to relative L2
<= 1e-6 at the same IPM tolerance, with the same iteration count."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import workloads as W
from tests._oracle_error import fp64_oracle_error  # noqa: E402
from oracle.fd import discretize, operator_matrix  # noqa: E402
from oracle.ipm import IPMOptions, initial_state, ipm_step, newton_matrix, newton_rhs, newton_solve  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _api():
    from paper_1806_05896_amd import Options, Problem
    return Options, Problem


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _load_state(prob, st, has_y):
    for f, a in (("y", st.y), ("w", st.w), ("v", st.v), ("p", st.p), ("lam_wa", st.lwa), ("lam_wb", st.lwb),
                 ("lam_va", st.lva), ("lam_vb", st.lvb)):
        prob.set_field(f, a)
    if has_y:
        prob.set_field("lam_ya", st.lya)
        prob.set_field("lam_yb", st.lyb)


@pytest.mark.parametrize("dim,N,pde", [(2, 3, "poisson"), (2, 31, "poisson"), (2, 127, "poisson"),
                                       (3, 7, "poisson"), (3, 31, "poisson"), (2, 7, "convdiff"),
                                       (2, 63, "convdiff")])
def test_operator_parity(dim, N, pde):
    Options, Problem = _api()
    print(f"[operator] dim={dim} N={N} pde={pde}", flush=True)
    data = W.poisson2d_small(N=N) if dim == 2 else W.poisson3d_127(N=N)
    if pde == "convdiff":
        data.pde, data.eps = "convdiff", 1.0 / 200
    rng = np.random.default_rng(N)
    x = rng.normal(size=data.n)
    A = operator_matrix(dim, N, pde, data.eps)
    with Problem(data) as prob:
        xt = torch.tensor(x, device="cuda", dtype=torch.float64)
        for tr in (False, True):
            y = prob.apply_operator(xt, transpose=tr).cpu().numpy()
            ref = (A.T if tr else A) @ x
            assert _rel(y, ref) <= 1e-13, (tr, _rel(y, ref))


def _generic_state(data, steps=2):
    disc = discretize(data)
    opts = IPMOptions(sigma=data.sigma)
    st = initial_state(data, opts)
    for _ in range(steps):
        st, _ = ipm_step(data, disc, st, opts, st.mu * opts.sigma)
    return disc, st


CASES = {
    "poisson_small": lambda: W.poisson2d_small(seed=0),
    "poisson_box63": lambda: W.poisson2d_511(seed=0, N=63),
    "poisson3d_15": lambda: W.poisson3d_127(seed=0, N=15),
    "convdiff_31": lambda: W.convdiff2d_255(seed=0, N=31),
}


def _rhs_magnitude(data, disc, st, mu):
    """Sum of the absolute values of the terms of each right-hand-side entry of eq. (NewtonSystem)."""
    absA = abs(disc.A)
    ry = np.abs(st.y) + np.abs(data.y_d) + absA.T @ np.abs(st.p)
    if data.y_a is not None:
        ry = ry + mu / np.abs(st.y - data.y_a) + mu / np.abs(data.y_b - st.y)
    au = data.alpha * (np.abs(st.w) + np.abs(st.v))
    rw = au + data.beta + np.abs(st.p) + mu / np.abs(st.w) + mu / np.abs(data.u_b - st.w)
    rv = au + data.beta + np.abs(st.p) + mu / np.abs(st.v) + mu / np.abs(-data.u_a - st.v)
    rp = absA @ np.abs(st.y) + np.abs(st.w) + np.abs(st.v) + np.abs(disc.f_hat)
    return np.concatenate([ry, rw, rv, rp])


@pytest.mark.parametrize("case", list(CASES))
def test_saddle_matvec_parity(case):
    Options, Problem = _api()
    print(f"[saddle] {case}", flush=True)
    data = CASES[case]()
    disc, st = _generic_state(data)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        prob.newton_setup(mu, Options())
        # elementwise rounding bound: 32 ulps of the sum of the magnitudes of the terms
        assert np.all(np.abs(prob.query_rhs() - b) <= 32 * np.finfo(float).eps * _rhs_magnitude(data, disc, st, mu))
        x = np.random.default_rng(1).normal(size=4 * data.n)
        y = prob.apply_saddle(torch.tensor(x, device="cuda", dtype=torch.float64)).cpu().numpy()
        assert _rel(y, K @ x) <= 1e-13


@pytest.mark.parametrize("vcycles", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["poisson_small", "convdiff_31", "poisson3d_15"])
def test_pd_preconditioner_symmetric_positive(case, prec, vcycles):
    """P_D^-1 must be symmetric positive definite for MINRES (exactly so in FP64),
    also with k-cycle multigrid solves."""
    Options, Problem = _api()
    print(f"[precond] {case} {prec} vcycles={vcycles}", flush=True)
    data = CASES[case]()
    disc, st = _generic_state(data)
    mu = st.mu * data.sigma
    opts = Options(mg_precision=prec, vcycles=vcycles)
    rng = np.random.default_rng(3)
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        prob.newton_setup(mu, opts)
        x = rng.normal(size=4 * data.n)
        z = rng.normal(size=4 * data.n)
        Px = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
        Pz = prob.apply_precond(torch.tensor(z, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    asym = abs(Px @ z - x @ Pz) / (np.linalg.norm(Px) * np.linalg.norm(z))
    assert asym <= (1e-13 if prec == "fp64" else 1e-5), asym
    assert Px @ x > 0 and Pz @ z > 0


@pytest.mark.parametrize("krylov,precond,prec", [("minres", "pd", "fp64"), ("minres", "pd", "fp32"),
                                                 ("fgmres", "pt", "fp32"), ("fgmres", "pd", "fp64")])
@pytest.mark.parametrize("case", list(CASES))
def test_newton_direction_parity(case, krylov, precond, prec):
    """The Krylov direction solves the oracle's FP64 Newton system (eq. (NewtonSystem))."""
    Options, Problem = _api()
    print(f"[newton] {case} {krylov} {precond} {prec}", flush=True)
    data = CASES[case]()
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    ref = np.concatenate(newton_solve(data, disc, st, mu))
    opts = Options(krylov=krylov, precond=precond, mg_precision=prec)
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        info = prob.newton_direction(mu, opts)
        d = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    res = np.linalg.norm(b - K @ d) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} relres(gpu)={info['relres']:.2e} relres(oracle K)={res:.2e}", flush=True)
    assert info["rc"] == 0
    assert res <= 1e-9
    assert _rel(d, ref) <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ipm_parity_poisson_small(prec):
    """Whole solve on the 31x31 Poisson workload (MINRES + P_D)."""
    Options, Problem = _api()
    print(f"[ipm] poisson2d_small {prec}", flush=True)
    data = W.poisson2d_small(seed=0)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    with Problem(data) as prob:
        rc = prob.solve(Options(mg_precision=prec))
        u, y = prob.query("u"), prob.query("y")
        s = prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e} "
          f"FP64-oracle error u={fp64_oracle_error(data, IPMOptions(sigma=data.sigma), ref):.2e}")
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


@pytest.mark.parametrize("case,krylov,precond", [("poisson_box63", "minres", "pd"), ("poisson3d_15", "minres", "pd"),
                                                 ("convdiff_31", "fgmres", "pt"), ("convdiff_31", "minres", "pd"),
                                                 ("poisson_box63", "fgmres", "pt")])
def test_ipm_parity_cases(case, krylov, precond):
    Options, Problem = _api()
    print(f"[ipm] {case} {krylov} {precond}", flush=True)
    data = CASES[case]()
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov=krylov, precond=precond))
        u, y = prob.query("u"), prob.query("y")
        s = prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e} "
          f"FP64-oracle error u={fp64_oracle_error(data, IPMOptions(sigma=data.sigma), ref):.2e}")
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


@pytest.mark.parametrize("seed,N", [(10, 31), (0, 63)])
def test_ipm_parity_central_mu_rule(seed, N):
    """The iterate-based barrier target (mu_rule="central") against the oracle
    running the same rule, on the state-constrained workload shape; seed 10 is
    the instance on which the fixed decrease of Algorithm A.1 breaks down at 63^2."""
    Options, Problem = _api()
    print(f"[ipm-central] poisson2d seed={seed} N={N}", flush=True)
    data = W.poisson2d_511(seed=seed, N=N)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma, mu_rule="central"))
    assert ref.status == "converged"
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, mu_rule="central"))
        u, y = prob.query("u"), prob.query("y")
        s = prob.stats()
    err = fp64_oracle_error(data, IPMOptions(sigma=data.sigma, mu_rule="central"), ref)
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e} "
          f"FP64-oracle error u={err:.2e}")
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["poisson_small", "poisson_box63", "convdiff_31", "poisson3d_15", "poisson_box255"])
def test_schur_multigrid_quality(case, prec):
    """The multigrid application of S_hat^-1 (Sec. 4.2, eq. (SchurApprox)) is close to the exact
    S_hat^-1 = (A + M_hat)^-T (I + Theta_y) (A + M_hat)^-1 built here with SciPy: one V-cycle per
    solve with 2+2 damped Jacobi sweeps must reduce the error below 0.35 (a V-cycle that is wrong
    anywhere - restriction, prolongation, coarse solve - lands well above that)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.ipm import barrier_diagonals
    Options, Problem = _api()
    print(f"[mg-quality] {case} {prec}", flush=True)
    data = W.poisson2d_511(seed=0, N=255) if case == "poisson_box255" else CASES[case]()
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    ty, tw, tv = barrier_diagonals(data, st)
    a = data.alpha
    mh = np.sqrt((tw + tv) / (a * (tw + tv) + tw * tv) * (1 + ty))
    Am = (disc.A + sp.diags(mh)).tocsc()
    lu = spla.splu(Am)
    r = np.random.default_rng(7).normal(size=data.n)
    exact = lu.solve((1 + ty) * lu.solve(r), trans="T")
    opts = Options(mg_precision=prec)
    x = np.zeros(4 * data.n)
    x[3 * data.n:] = r
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        prob.newton_setup(mu, opts)
        z = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    err = _rel(z[3 * data.n:], exact)
    print(f"  rel err of S_hat^-1 by multigrid: {err:.3f}", flush=True)
    assert err <= 0.35


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_schur_multigrid_quality_3d_cubes(prec):
    """The fused 3D level kernels (FP32 31^3: one cube descent and ascent above the coarse
    kernel's 15^3; FP64 with 2+2 or 3+3 sweeps takes the one-node-per-thread kernels, whose
    cubes would not fit the LDS) apply S_hat^-1 (Sec. 4.2) as the V-cycle should: against the exact SciPy
    (A + M_hat)^-T (I + Theta_y) (A + M_hat)^-1 at the IPM's starting point, one cycle of
    2+2 sweeps below 0.45 and of 3+3 below 0.35 (the one-node-per-thread kernels they replace
    give 0.426 and 0.322 on this input; a wrong restriction, prolongation or coarse solve lands
    near or above 1), and k = 1, 2, 4 cycles contracting geometrically (FP64)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.ipm import barrier_diagonals
    Options, Problem = _api()
    print(f"[mg-quality-3d] {prec}", flush=True)
    data = W.poisson3d_127(seed=0, N=31)
    disc, st = _generic_state(data, steps=0)
    mu = st.mu * data.sigma
    ty, tw, tv = barrier_diagonals(data, st)
    a = data.alpha
    mh = np.sqrt((tw + tv) / (a * (tw + tv) + tw * tv) * (1 + ty))
    lu = spla.splu((disc.A + sp.diags(mh)).tocsc())
    r = np.random.default_rng(7).normal(size=data.n)
    exact = lu.solve((1 + ty) * lu.solve(r), trans="T")
    x = np.zeros(4 * data.n)
    x[3 * data.n:] = r
    errs = {}
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        for k, nu in ([(1, 2), (2, 2), (4, 2), (1, 3)] if prec == "fp64" else [(1, 2), (1, 3)]):
            opts = Options(mg_precision=prec, vcycles=k, nu_pre=nu, nu_post=nu)
            prob.newton_setup(mu, opts)
            z = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
            errs[(k, nu)] = _rel(z[3 * data.n:], exact)
    print("  rel err by (k, nu):", {k: f"{e:.3e}" for k, e in errs.items()}, flush=True)
    assert errs[(1, 2)] <= 0.45 and errs[(1, 3)] <= 0.35
    if prec == "fp64":
        assert errs[(2, 2)] <= 0.5 * errs[(1, 2)] and errs[(4, 2)] <= 0.5 * errs[(2, 2)]


@pytest.mark.parametrize("case", ["poisson_small", "convdiff_31", "poisson3d_15", "poisson_box255"])
def test_kcycle_multigrid_contracts(case):
    """k V-cycles per multigrid solve (x_{j+1} = x_j + V(b - (A + M_hat) x_j)) approach the
    exact S_hat^-1 geometrically: each doubling of k at least halves the error (FP64)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.ipm import barrier_diagonals
    Options, Problem = _api()
    print(f"[kcycle] {case}", flush=True)
    data = W.poisson2d_511(seed=0, N=255) if case == "poisson_box255" else CASES[case]()
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    ty, tw, tv = barrier_diagonals(data, st)
    a = data.alpha
    mh = np.sqrt((tw + tv) / (a * (tw + tv) + tw * tv) * (1 + ty))
    lu = spla.splu((disc.A + sp.diags(mh)).tocsc())
    r = np.random.default_rng(7).normal(size=data.n)
    exact = lu.solve((1 + ty) * lu.solve(r), trans="T")
    x = np.zeros(4 * data.n)
    x[3 * data.n:] = r
    errs = {}
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        for k in (1, 2, 4):
            opts = Options(mg_precision="fp64", vcycles=k)
            prob.newton_setup(mu, opts)
            z = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
            errs[k] = _rel(z[3 * data.n:], exact)
    print("  rel err by k:", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    assert errs[2] <= 0.5 * errs[1] and errs[4] <= 0.5 * errs[2]


def test_hard_instance_central_rule_kcycles():
    """Seed 10 at 63^2: the instance on which the fixed decrease breaks down.  With the
    iterate-based target and 3 V-cycles of 3+3 sweeps per multigrid solve (the lean
    1-cycle preconditioner needs more than the Krylov limit late in this solve) the GPU
    follows the oracle's trajectory: same iteration count, stopping test met (independent
    CPU measures), control and state within 1e-6."""
    from oracle.ipm import measures
    Options, Problem = _api()
    data = W.poisson2d_511(seed=10, N=63)
    print("[hard] seed 10 N=63 central vcycles=3", flush=True)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma, mu_rule="central"))
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, mu_rule="central", vcycles=3, nu_pre=3, nu_post=3,
                                krylov_maxit=2000))
        s = prob.stats()
        u = prob.query("u")
        q = prob.query
        from oracle.ipm import IPMState
        st = IPMState(q("y"), q("w"), q("v"), q("p"), q("lam_wa"), q("lam_wb"), q("lam_va"), q("lam_vb"), mu=s.mu)
        st.lya, st.lyb = q("lam_ya"), q("lam_yb")
    xs = measures(data, discretize(data), st)
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} max/step={max(s.hist_krylov[:s.nli])} "
          f"measures={xs} rel u vs oracle={_rel(u, ref.u):.2e}", flush=True)
    assert rc == 0 and max(xs) <= 1e-6 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6
