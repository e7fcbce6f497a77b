"""GPU parity for the heat equation, all time steps at once (Sec. 4.4): the
space-time operator, the Newton right-hand side and saddle matvec, the
preconditioner with its block forward/backward substitution over the time
steps, Newton directions and whole IPM solves, all through the C ABI and
against the CPU oracle.  Tolerances as in test_gpu_parity.py: FP64 stencil
sums at 1e-13 relative, Newton directions at relative residual <= 1e-9 on
the oracle's sparse system, whole solves at relative L2 <= 1e-6 with the
same IPM iteration count."""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle.fd import discretize  # noqa: E402
from oracle.ipm import IPMOptions, newton_matrix, newton_rhs, newton_solve  # noqa: E402
from tests.test_gpu_parity import _generic_state, _load_state, _rel, _rhs_magnitude  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _api():
    from paper_1806_05896_amd import Batch, Options, Problem
    return Batch, Options, Problem


def _with_data(N, nt, seed=2):
    """Nonzero source, boundary data and initial state (all folded into f_hat)."""
    d = W.heat2d(seed=seed, N=N, nt=nt)
    rng = np.random.default_rng(100 + N + nt)
    x1, x2 = W.interior_coords(2, N)
    d.y0 = 0.3 * np.sin(math.pi * x1) * np.sin(2 * math.pi * x2)
    d.f = 0.5 * rng.normal(size=d.n)
    g1, g2 = W.all_coords(2, N)
    d.g = 0.1 * (g1 + g2)
    return d


def _state_bounded(N, nt):
    """State bounds y in [-0.1, 0.5]: the upper bound is active on about 10% of the nodes."""
    d = W.heat2d(seed=6, N=N, nt=nt)
    d.y_a = np.full(d.n, -0.1)
    d.y_b = np.full(d.n, 0.5)
    return d


CASES = {
    "heat_7x10": lambda: W.heat2d(seed=0, N=7, nt=10),
    "heat_sb_7x8": lambda: _state_bounded(7, 8),
    "heat_15x25": lambda: W.heat2d(seed=1, N=15, nt=25),
    "heat_data_7x6": lambda: _with_data(7, 6),
    "heat_31x1": lambda: W.heat2d(seed=3, N=31, nt=1),
}


@functools.lru_cache(maxsize=None)
def _oracle(case):
    data = CASES[case]()
    return oracle.solve(data, IPMOptions(sigma=data.sigma))


@pytest.mark.parametrize("N,nt", [(3, 4), (15, 25), (63, 7)])
def test_heat_operator_parity(N, nt):
    _, Options, Problem = _api()
    print(f"[heat operator] N={N} nt={nt}", flush=True)
    data = W.heat2d(N=N, nt=nt)
    A = discretize(data).A
    x = np.random.default_rng(N * nt).normal(size=data.n)
    with Problem(data) as prob:
        xt = torch.tensor(x, device="cuda", dtype=torch.float64)
        for tr in (False, True):
            y = prob.apply_operator(xt, transpose=tr).cpu().numpy()
            ref = (A.T if tr else A) @ x
            assert _rel(y, ref) <= 1e-13, (tr, _rel(y, ref))


@pytest.mark.parametrize("case", ["heat_7x10", "heat_data_7x6", "heat_31x1", "heat_sb_7x8"])
def test_heat_rhs_and_saddle_matvec(case):
    """Newton right-hand side (with y0, g and f folded into f_hat) and the saddle matvec."""
    _, Options, Problem = _api()
    print(f"[heat saddle] {case}", flush=True)
    data = CASES[case]()
    disc, st = _generic_state(data)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        prob.newton_setup(mu, Options())
        assert np.all(np.abs(prob.query_rhs() - b) <= 32 * np.finfo(float).eps * _rhs_magnitude(data, disc, st, mu))
        x = np.random.default_rng(1).normal(size=4 * data.n)
        y = prob.apply_saddle(torch.tensor(x, device="cuda", dtype=torch.float64)).cpu().numpy()
        assert _rel(y, K @ x) <= 1e-13


@pytest.mark.parametrize("vcycles", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_heat_pd_symmetric_positive(prec, vcycles):
    """The block substitutions use the same per-step multigrid operator forward
    and backward, so P_D^-1 stays symmetric positive definite."""
    _, Options, Problem = _api()
    print(f"[heat precond] {prec} vcycles={vcycles}", flush=True)
    data = CASES["heat_15x25"]()
    disc, st = _generic_state(data)
    mu = st.mu * data.sigma
    opts = Options(mg_precision=prec, vcycles=vcycles)
    rng = np.random.default_rng(3)
    with Problem(data) as prob:
        _load_state(prob, st, False)
        prob.newton_setup(mu, opts)
        x = rng.normal(size=4 * data.n)
        z = rng.normal(size=4 * data.n)
        Px = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
        Pz = prob.apply_precond(torch.tensor(z, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    asym = abs(Px @ z - x @ Pz) / (np.linalg.norm(Px) * np.linalg.norm(z))
    assert asym <= (1e-13 if prec == "fp64" else 1e-5), asym
    assert Px @ x > 0 and Pz @ z > 0


def test_heat_schur_solve_is_block_substitution():
    """With exact per-step solves the Schur block would be exactly
    (L + M_hat)^-T (O + Theta_y) (L + M_hat)^-1; with k-cycle multigrid solves
    (8 V-cycles of 4 + 4 sweeps per step) the p block of P_D^-1 must approach it."""
    _, Options, Problem = _api()
    data = CASES["heat_7x10"]()
    disc, st = _generic_state(data)
    mu = st.mu * data.sigma
    from oracle.ipm import barrier_diagonals
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    ty, tw, tv = barrier_diagonals(data, st)
    sig = (tw + tv) / (data.alpha * (tw + tv) + tw * tv)
    mhat = np.sqrt(sig * (1.0 + ty))
    B = (disc.A + sp.diags(mhat)).tocsc()
    r = np.random.default_rng(7).normal(size=data.n)
    ref = spla.spsolve(B.T.tocsc(), (1.0 + ty) * spla.spsolve(B, r))
    x = np.zeros(4 * data.n)
    x[3 * data.n:] = r
    opts = Options(mg_precision="fp64", vcycles=8, nu_pre=4, nu_post=4)
    with Problem(data) as prob:
        _load_state(prob, st, False)
        prob.newton_setup(mu, opts)
        z = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    print(f"  rel err {_rel(z[3 * data.n:], ref):.2e}", flush=True)
    assert _rel(z[3 * data.n:], ref) <= 1e-8, _rel(z[3 * data.n:], ref)


@pytest.mark.parametrize("krylov,precond,prec", [("minres", "pd", "fp64"), ("minres", "pd", "fp32"),
                                                 ("fgmres", "pt", "fp32"), ("fgmres", "pd", "fp64")])
@pytest.mark.parametrize("case", ["heat_7x10", "heat_15x25"])
def test_heat_newton_direction_parity(case, krylov, precond, prec):
    _, Options, Problem = _api()
    print(f"[heat newton] {case} {krylov} {precond} {prec}", flush=True)
    data = CASES[case]()
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    ref = np.concatenate(newton_solve(data, disc, st, mu))
    opts = Options(krylov=krylov, precond=precond, mg_precision=prec)
    with Problem(data) as prob:
        _load_state(prob, st, False)
        info = prob.newton_direction(mu, opts)
        d = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    res = np.linalg.norm(b - K @ d) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} relres(gpu)={info['relres']:.2e} relres(oracle K)={res:.2e}", flush=True)
    assert info["rc"] == 0
    assert res <= 1e-9
    assert _rel(d, ref) <= 1e-6


@pytest.mark.parametrize("case,krylov,precond,prec", [("heat_7x10", "minres", "pd", "fp32"),
                                                      ("heat_7x10", "fgmres", "pt", "fp64"),
                                                      ("heat_data_7x6", "fgmres", "pt", "fp32"),
                                                      ("heat_15x25", "fgmres", "pt", "fp32"),
                                                      ("heat_15x25", "minres", "pd", "fp64"),
                                                      ("heat_31x1", "minres", "pd", "fp32"),
                                                      ("heat_sb_7x8", "minres", "pd", "fp32"),
                                                      ("heat_sb_7x8", "fgmres", "pt", "fp64")])
def test_heat_ipm_parity(case, krylov, precond, prec):
    _, Options, Problem = _api()
    print(f"[heat ipm] {case} {krylov} {precond} {prec}", flush=True)
    data = CASES[case]()
    ref = _oracle(case)
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov=krylov, precond=precond, mg_precision=prec))
        u, y, p = prob.query("u"), prob.query("y"), prob.query("p")
        s = prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e}")
    assert ref.status == "converged"
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6 and _rel(p, ref.p) <= 1e-6


def test_heat_refusals():
    """P_Pi, batches mixing heat and steady problems, heat batches outside the
    one-launch substitution, and the per-level timers are refused."""
    Batch, Options, Problem = _api()
    from paper_1806_05896_amd import _lib as L
    data = CASES["heat_7x10"]()
    with Problem(data) as prob, Problem(W.poisson2d_small(N=15)) as steady, \
            Problem(W.heat2d(seed=5, N=63, nt=3)) as big:
        with pytest.raises(Exception):
            prob.solve(Options(krylov="fgmres", precond="ppi"), raise_on_error=True)
        with pytest.raises(Exception):
            Batch([prob, steady])
        with pytest.raises(Exception):  # FP64 V-cycles at 63^2 need per-step launches
            Batch([prob, big]).solve(Options(sigma=data.sigma, mg_precision="fp64"))
        rc = prob.solve(Options(sigma=data.sigma))
        assert rc == L.OK
        with pytest.raises(Exception):
            prob.time_kernel(3, reps=1)


@pytest.mark.parametrize("krylov,precond", [("fgmres", "pt"), ("minres", "pd")])
def test_heat_batch_equals_solo(krylov, precond):
    """Heat problems of different sizes and step counts solved as one batch
    (one workgroup per instance in the substitution kernel) give bit-identical
    iterates and the same iteration counts as solo solves."""
    Batch, Options, Problem = _api()
    datas = [W.heat2d(seed=1, N=15, nt=25), W.heat2d(seed=2, N=31, nt=10), W.heat2d(seed=0, N=7, nt=12)]
    opts = Options(sigma=0.25, krylov=krylov, precond=precond, mg_precision="fp32")
    solo = []
    for d in datas:
        with Problem(d) as p:
            assert p.solve(opts) == 0
            solo.append((p.query("u"), p.query("y"), p.stats()))
    probs = [Problem(d) for d in datas]
    try:
        b = Batch(probs)
        b.solve(opts)
        for p, (u, y, st) in zip(probs, solo):
            s = p.stats()
            assert s.status == 0 and s.nli == st.nli and s.krylov_its == st.krylov_its
            np.testing.assert_array_equal(p.query("u"), u)
            np.testing.assert_array_equal(p.query("y"), y)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("prec,vcycles", [("fp64", 1), ("fp32", 2)])
def test_heat_direction_per_step_launches(prec, vcycles):
    """63^2 x 7 steps with FP64 V-cycles (the finest level runs outside the
    single-workgroup kernel) or k-cycle solves: the substitution takes one
    multigrid launch sequence per time step.  The Newton direction must solve
    the oracle's sparse system to the Krylov tolerance."""
    _, Options, Problem = _api()
    print(f"[heat per-step] {prec} vcycles={vcycles}", flush=True)
    data = W.heat2d(seed=4, N=63, nt=7)
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    opts = Options(krylov="fgmres", precond="pt", mg_precision=prec, vcycles=vcycles)
    with Problem(data) as prob:
        _load_state(prob, st, False)
        info = prob.newton_direction(mu, opts)
        d = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    res = np.linalg.norm(b - K @ d) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} relres(oracle K)={res:.2e}", flush=True)
    assert info["rc"] == 0 and res <= 1e-9
