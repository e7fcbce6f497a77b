"""GPU parity for trilinear Q1 elements in 3D (Sec. 2, eq. (pb_fe_lin) on
the unit cube): the 27-point stiffness and mass, the Newton right-hand side
and saddle matvec, the Chebyshev semi-iteration of the (1,1) block on the
3D mass interval [1/8, 27/8], Newton directions and whole solves, through
the C ABI against the CPU oracle.

The oracle factors the whole Newton system (no per-node elimination with
a consistent mass), which limits its direct solves to 15^3; at 31^3, where
the multigrid's fine-level kernels run (smaller grids fit the single
workgroup coarse kernel), the GPU directions are checked against the
oracle's own system matrix and right-hand side instead."""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle.fd import discretize  # noqa: E402
from oracle.ipm import IPMOptions, IPMState, barrier_diagonals, newton_matrix, newton_rhs, newton_solve  # noqa: E402
from tests.test_gpu_parity import _generic_state, _load_state, _rel  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _api():
    from paper_1806_05896_amd import Batch, Options, Problem
    return Batch, Options, Problem


def _bounded(N, seed=0):
    """State bounds [-0.06, 0.06], active at the optimum (|y| reaches 0.087 without them)."""
    d = W.poisson3d_q1(seed=seed, N=N)
    d.y_a = np.full(d.n, -0.06)
    d.y_b = np.full(d.n, 0.06)
    return d


def _with_data(N):
    """Nonzero source and boundary data (folded into f_hat through M and L)."""
    d = W.poisson3d_q1(seed=3, N=N)
    rng = np.random.default_rng(N)
    d.f = 0.3 * rng.normal(size=d.n)
    g1, g2, g3 = W.all_coords(3, N)
    d.g = 0.05 * (1 + g1 - g2 + 0.5 * g3)
    return d


CASES = {
    "q1_3d_7": lambda: W.poisson3d_q1(seed=0, N=7),
    "q1_3d_sb_7": lambda: _bounded(7),
    "q1_3d_data_7": lambda: _with_data(7),
    "q1_3d_15": lambda: W.poisson3d_q1(seed=0, N=15),
    "q1_3d_sb_15": lambda: _bounded(15),
    "q1_3d_sb_31": lambda: _bounded(31),
    "q1_3d_31": lambda: W.poisson3d_q1(seed=1, N=31),
}


def _synthetic_state(data, seed=0):
    """An interior point (every bound strict, every multiplier positive) with
    multipliers spread over three orders of magnitude, for sizes at which
    the oracle's IPM steps are too slow."""
    rng = np.random.default_rng(seed)
    n = data.n
    if data.y_a is not None:
        y = data.y_a + (data.y_b - data.y_a) * rng.uniform(0.2, 0.8, n)
    else:
        y = rng.normal(0.0, 0.05, n)
    w = data.u_b * rng.uniform(0.1, 0.9, n)
    v = -data.u_a * rng.uniform(0.1, 0.9, n)
    lam = lambda: 10.0 ** rng.uniform(-3.0, 0.0, n)  # noqa: E731
    st = IPMState(y, w, v, rng.normal(0.0, 1e-2, n), lam(), lam(), lam(), lam(), mu=0.04)
    if data.y_a is not None:
        st.lya, st.lyb = lam(), lam()
    return discretize(data), st


def _state(case):
    data = CASES[case]()
    if data.N >= 31:
        return (data,) + _synthetic_state(data)
    return (data,) + _generic_state(data)


def _rhs_magnitude(data, disc, st, mu):
    """Sum of the magnitudes of the terms of each right-hand-side entry."""
    aA, aM = abs(disc.A), abs(disc.Mc)
    ry = aM @ (np.abs(st.y) + np.abs(data.y_d)) + aA.T @ np.abs(st.p)
    if data.y_a is not None:
        ry = ry + mu / np.abs(st.y - data.y_a) + mu / np.abs(data.y_b - st.y)
    au = data.alpha * (aM @ (np.abs(st.w) + np.abs(st.v)))
    rw = au + data.beta + aM @ np.abs(st.p) + mu / np.abs(st.w) + mu / np.abs(data.u_b - st.w)
    rv = au + data.beta + aM @ np.abs(st.p) + mu / np.abs(st.v) + mu / np.abs(-data.u_a - st.v)
    rp = aA @ np.abs(st.y) + aM @ (np.abs(st.w) + np.abs(st.v)) + np.abs(disc.f_hat)
    return np.concatenate([ry, rw, rv, rp])


@pytest.mark.parametrize("N", [3, 7, 31, 63])
def test_q1_3d_operator_parity(N):
    _, Options, Problem = _api()
    print(f"[q1 3d operator] N={N}", flush=True)
    data = W.poisson3d_q1(N=N)
    A = discretize(data).A
    x = np.random.default_rng(N).normal(size=data.n)
    with Problem(data) as prob:
        xt = torch.tensor(x, device="cuda", dtype=torch.float64)
        for tr in (False, True):
            y = prob.apply_operator(xt, transpose=tr).cpu().numpy()
            assert _rel(y, (A.T if tr else A) @ x) <= 1e-13


@pytest.mark.parametrize("case", ["q1_3d_7", "q1_3d_sb_7", "q1_3d_data_7", "q1_3d_sb_31"])
def test_q1_3d_rhs_and_saddle_matvec(case):
    _, Options, Problem = _api()
    print(f"[q1 3d saddle] {case}", flush=True)
    data, disc, st = _state(case)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st)
    b = newton_rhs(data, disc, st, mu)
    opts = Options(krylov="fgmres", precond="pd")
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        prob.newton_setup(mu, opts)
        assert np.all(np.abs(prob.query_rhs() - b) <= 64 * np.finfo(float).eps * _rhs_magnitude(data, disc, st, mu))
        x = np.random.default_rng(1).normal(size=4 * data.n)
        y = prob.apply_saddle(torch.tensor(x, device="cuda", dtype=torch.float64)).cpu().numpy()
        assert _rel(y, K @ x) <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_q1_3d_pd_symmetric_positive(prec):
    """P_D^-1 with the fixed Chebyshev polynomial and the 3D multigrid stays
    symmetric positive definite (MINRES needs it)."""
    _, Options, Problem = _api()
    data, disc, st = _state("q1_3d_sb_31")
    mu = st.mu * data.sigma
    opts = Options(krylov="minres", precond="pd", mg_precision=prec)
    rng = np.random.default_rng(3)
    with Problem(data) as prob:
        _load_state(prob, st, True)
        prob.newton_setup(mu, opts)
        x = rng.normal(size=4 * data.n)
        z = rng.normal(size=4 * data.n)
        Px = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
        Pz = prob.apply_precond(torch.tensor(z, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    asym = abs(Px @ z - x @ Pz) / (np.linalg.norm(Px) * np.linalg.norm(z))
    assert asym <= (1e-13 if prec == "fp64" else 1e-5), asym
    assert Px @ x > 0 and Pz @ z > 0


@pytest.mark.parametrize("case", ["q1_3d_sb_7", "q1_3d_sb_31"])
def test_q1_3d_chebyshev_block(case):
    """The y block of P_D^-1 is 20 Chebyshev steps for (M + Theta_y) z = r on
    [1/8, 27/8]: its energy-norm error against the exact solve is at most
    2 ((sqrt(27) - 1) / (sqrt(27) + 1))^20 (condition number 27)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    _, Options, Problem = _api()
    data, disc, st = _state(case)
    mu = st.mu * data.sigma
    ty, _, _ = barrier_diagonals(data, st)
    B = (disc.Mt + sp.diags(ty)).tocsc()
    r = np.random.default_rng(5).normal(size=data.n)
    exact = spla.spsolve(B, r)
    assert np.linalg.norm(B @ exact - r) <= 1e-13 * np.linalg.norm(r)
    x = np.zeros(4 * data.n)
    x[:data.n] = r
    opts = Options(krylov="fgmres", precond="pd", mg_precision="fp64")
    with Problem(data) as prob:
        _load_state(prob, st, True)
        prob.newton_setup(mu, opts)
        z = prob.apply_precond(torch.tensor(x, device="cuda", dtype=torch.float64), opts).cpu().numpy()
    e = z[:data.n] - exact
    err = math.sqrt(e @ (B @ e)) / math.sqrt(exact @ (B @ exact))
    q = (math.sqrt(27.0) - 1) / (math.sqrt(27.0) + 1)
    print(f"  energy-norm error {err:.2e} (bound {2 * q ** 20:.2e})", flush=True)
    assert err <= 2 * q ** 20


COMBOS = [("fgmres", "pd", "fp64"), ("fgmres", "pd", "fp32"), ("fgmres", "pt", "fp32"), ("fgmres", "pt", "fp64"),
          ("minres", "pd", "fp32"), ("minres", "pd", "fp64")]


@functools.lru_cache(maxsize=None)
def _direct_case(case):
    """State, Newton system and the oracle's direct solution (cached: the
    factorization takes seconds at 15^3)."""
    data = CASES[case]()
    disc, st = _generic_state(data, steps=3)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st).tocsr()
    b = newton_rhs(data, disc, st, mu)
    ref = np.concatenate(newton_solve(data, disc, st, mu))
    return data, st, mu, K, b, ref


@pytest.mark.parametrize("krylov,precond,prec", COMBOS)
@pytest.mark.parametrize("case", ["q1_3d_sb_7", "q1_3d_sb_15"])
def test_q1_3d_newton_direction_parity(case, krylov, precond, prec):
    _, Options, Problem = _api()
    print(f"[q1 3d newton] {case} {krylov} {precond} {prec}", flush=True)
    data, st, mu, K, b, ref = _direct_case(case)
    opts = Options(krylov=krylov, precond=precond, mg_precision=prec)
    with Problem(data) as prob:
        _load_state(prob, st, True)
        info = prob.newton_direction(mu, opts)
        d = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    res = np.linalg.norm(b - K @ d) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} relres(gpu)={info['relres']:.2e} relres(oracle K)={res:.2e}", flush=True)
    assert info["rc"] == 0
    assert res <= 1e-9
    assert _rel(d, ref) <= 1e-6


@pytest.mark.parametrize("krylov,precond,prec", COMBOS)
@pytest.mark.parametrize("case", ["q1_3d_sb_31", "q1_3d_31"])
def test_q1_3d_newton_direction_solves_oracle_system(case, krylov, precond, prec):
    """At 31^3 (fine multigrid levels on the level kernels): the GPU direction
    solves the oracle's system to the Krylov tolerance 1e-10, or to the FP64
    attainable-accuracy floor where that is larger."""
    _, Options, Problem = _api()
    print(f"[q1 3d newton31] {case} {krylov} {precond} {prec}", flush=True)
    data, disc, st = _state(case)
    mu = st.mu * data.sigma
    K = newton_matrix(data, disc, st).tocsr()
    b = newton_rhs(data, disc, st, mu)
    opts = Options(krylov=krylov, precond=precond, mg_precision=prec)
    with Problem(data) as prob:
        _load_state(prob, st, data.y_a is not None)
        info = prob.newton_direction(mu, opts)
        d = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    res = np.linalg.norm(b - K @ d) / np.linalg.norm(b)
    floor = 16 * np.finfo(float).eps * np.linalg.norm(abs(K) @ np.abs(d) + np.abs(b)) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} relres(gpu)={info['relres']:.2e} relres(oracle K)={res:.2e}", flush=True)
    assert info["rc"] == 0
    assert res <= max(1e-10, floor) * 1.01


# Whole solves with active state bounds take the FP64 multigrid: once Theta_y
# passes ~1e8 the FP32 transpose solve of the Schur approximation no longer
# preconditions the Q1 system (the consistent mass couples constrained and
# free nodes); an exact FP32 solve shows the same on the CPU.
#
# The state-bounded 15^3 instance (both barrier rules) is tested below
# against stored oracle solutions, with FGMRES(60): P_T's iteration counts
# grow with Theta_y there and FGMRES(30) stagnates.


@pytest.mark.parametrize("case,krylov,precond,prec", [("q1_3d_7", "minres", "pd", "fp32"),
                                                      ("q1_3d_7", "fgmres", "pt", "fp64"),
                                                      ("q1_3d_7", "fgmres", "pt", "fp32"),
                                                      ("q1_3d_sb_7", "fgmres", "pt", "fp64"),
                                                      ("q1_3d_sb_7", "minres", "pd", "fp64"),
                                                      ("q1_3d_data_7", "fgmres", "pd", "fp32"),
                                                      ("q1_3d_15", "fgmres", "pt", "fp32")])
def test_q1_3d_ipm_parity(case, krylov, precond, prec):
    _, Options, Problem = _api()
    print(f"[q1 3d ipm] {case} {krylov} {precond} {prec}", flush=True)
    data = CASES[case]()
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov=krylov, precond=precond, mg_precision=prec))
        u, y, p = prob.query("u"), prob.query("y"), prob.query("p")
        s = prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e}",
          flush=True)
    assert ref.status == "converged"
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6 and _rel(p, ref.p) <= 1e-6


def test_q1_3d_batch_equals_solo():
    Batch, Options, Problem = _api()
    datas = [_bounded(7), W.poisson3d_q1(seed=0, N=15), W.poisson3d_q1(seed=1, N=31)]
    opts = Options(sigma=0.2, krylov="fgmres", precond="pt", mg_precision="fp64")
    solo = []
    for d in datas:
        with Problem(d) as p:
            assert p.solve(opts) == 0
            solo.append((p.query("u"), p.stats()))
    probs = [Problem(d) for d in datas]
    try:
        Batch(probs).solve(opts)
        for p, (u, st) in zip(probs, solo):
            s = p.stats()
            assert s.status == 0 and s.nli == st.nli and s.krylov_its == st.krylov_its
            np.testing.assert_array_equal(p.query("u"), u)
    finally:
        for p in probs:
            p.close()


@pytest.mark.parametrize("rule", ["central", "paper"])
def test_q1_3d_state_bounded_15(rule):
    """The state-bounded 15^3 instance (FGMRES + P_T, FP64 multigrid) under the
    iterate-based barrier rule and under the paper's fixed decrease, against
    the oracle's solutions under the same rule, stored by
    tests/golden/make_oracle_solutions.py (its runs take minutes): equal
    iteration count and rel-L2 <= 1e-6 in u, y and p.

    P_T loses strength on this problem as the iterate approaches the state
    bounds.  Under the iterate-based rule, FGMRES iterations per IPM step grow
    from 9 to about 530 (k = 27).  FGMRES(30) then stagnates between restarts:
    up to 3800 iterations per step, over the default limit of 500 from k = 22,
    after which the trajectory leaves the oracle's.  Under the fixed decrease
    the oracle itself needs 47 iterations (mu down to 1e-33 with step lengths
    of 0.03-0.3).  So the solve runs FGMRES(60) with a limit of 4000, and every
    Newton system then reaches 1e-10 under both rules."""
    import json
    import os
    _, Options, Problem = _api()
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", f"q1_3d_sb15_{rule}_oracle.npz"), allow_pickle=False)
    data = _bounded(15)
    print(f"[q1 3d sb15 {rule}] fgmres(60) pt fp64", flush=True)
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov="fgmres", precond="pt", mg_precision="fp64",
                                mu_rule=rule, restart=60, krylov_maxit=4000))
        u, y, p = prob.query("u"), prob.query("y"), prob.query("p")
        s = prob.stats()
    hist = json.loads(str(g["history"]))
    for k in range(min(s.nli, len(hist) - 1)):
        print(f"    k={k} mu {s.hist_mu[k]:.3e}/{hist[k]['mu']:.3e} alpha_P {s.hist_alpha_p[k]:.4f}/"
              f"{hist[k]['alpha_P']:.4f} krylov {s.hist_krylov[k]} relres {s.hist_krylov_relres[k]:.1e}", flush=True)
    print(f"  rc={rc} nli={s.nli}/{int(g['nli'])} its={s.krylov_its} rel u={_rel(u, g['u']):.2e} "
          f"y={_rel(y, g['y']):.2e} p={_rel(p, g['p']):.2e} FP64-oracle error u={float(g['oracle_error_u']):.2e}",
          flush=True)
    assert str(g["status"]) == "converged"
    assert rc == 0 and s.nli == int(g["nli"])
    assert _rel(u, g["u"]) <= 1e-6 and _rel(y, g["y"]) <= 1e-6 and _rel(p, g["p"]) <= 1e-6
