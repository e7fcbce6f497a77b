"""Partial observation (Sec. 4.3): observation weights O in the tracking term
and the preconditioner P_Pi of eq. (eq:prec1) with FGMRES, against the
oracle (which solves the full Newton system directly)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle.fd import discretize  # noqa: E402
from oracle.ipm import IPMOptions, IPMState, initial_state, ipm_step, newton_matrix, newton_rhs  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _load_state(prob, st, has_y):
    for f, a in (("y", st.y), ("w", st.w), ("v", st.v), ("p", st.p), ("lam_wa", st.lwa), ("lam_wb", st.lwb),
                 ("lam_va", st.lva), ("lam_vb", st.lvb)):
        prob.set_field(f, a)
    if has_y:
        prob.set_field("lam_ya", st.lya)
        prob.set_field("lam_yb", st.lyb)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("N", [31, 63])
def test_ppi_ipm_parity(N, prec):
    from paper_1806_05896_amd import Options, Problem
    data = W.poisson2d_partial(seed=0, N=N)
    print(f"[ppi] N={N} {prec}", flush=True)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    assert ref.status == "converged"
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov="fgmres", precond="ppi", mg_precision=prec))
        u, y, s = prob.query("u"), prob.query("y"), prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e} y={_rel(y, ref.y):.2e}",
          flush=True)
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


def test_singular_block_needs_ppi():
    from paper_1806_05896_amd import Options, Problem
    from paper_1806_05896_amd import _lib as L
    data = W.poisson2d_partial(seed=0, N=15)
    with Problem(data) as prob:
        with pytest.raises(L.IpmpdeError) as ei:
            prob.solve(Options(sigma=data.sigma), raise_on_error=True)
        assert ei.value.code == L.EINVAL


@pytest.mark.parametrize("krylov,precond", [("minres", "pd"), ("fgmres", "pt"), ("fgmres", "ppi")])
def test_positive_observation_weights(krylov, precond):
    """Weights 1 on the observed square and 0.25 elsewhere (O > 0, so every
    preconditioner applies): parity with the oracle."""
    from paper_1806_05896_amd import Options, Problem
    data = W.poisson2d_partial(seed=1, N=31)
    data.obs = 0.25 + 0.75 * data.obs
    print(f"[obs>0] {krylov} {precond}", flush=True)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov=krylov, precond=precond))
        u, y, s = prob.query("u"), prob.query("y"), prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e}", flush=True)
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


def test_ppi_with_state_bounds():
    """Partial observation with state bounds: O + Theta_y is positive but tiny at
    unobserved nodes far from the bounds, the case P_Pi is designed for."""
    from paper_1806_05896_amd import Options, Problem
    data = W.poisson2d_partial(seed=1, N=31)
    data.y_a = np.full(data.n, -0.3)
    data.y_b = np.full(data.n, 0.4)
    print("[ppi+box]", flush=True)
    ref = oracle.solve(data, IPMOptions(sigma=data.sigma))
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov="fgmres", precond="ppi"))
        u, y, s = prob.query("u"), prob.query("y"), prob.stats()
    print(f"  rc={rc} nli={s.nli}/{ref.nli} its={s.krylov_its} rel u={_rel(u, ref.u):.2e}", flush=True)
    assert rc == 0 and s.nli == ref.nli
    assert _rel(u, ref.u) <= 1e-6 and _rel(y, ref.y) <= 1e-6


def test_ppi_application_matches_exact_solves():
    """The GPU's P_Pi application (FP64, 8 V-cycles per multigrid solve) against
    the same three-step formula with exact sparse solves: v2 = z-block inverse,
    v1 = L^-1 (Mbar v2 + r_p), v3 = (L + M_r)^-1 L (L^T + M_l)^-1 ((O + Theta_y) v1 - r_y)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.ipm import barrier_diagonals
    from paper_1806_05896_amd import Options, Problem
    data = W.poisson2d_partial(seed=2, N=63)
    opts = IPMOptions(sigma=data.sigma)
    disc = discretize(data)
    st = initial_state(data, opts)
    for _ in range(3):
        st, _ = ipm_step(data, disc, st, opts, st.mu * opts.sigma)
    mu = st.mu * opts.sigma
    n, a = data.n, data.alpha
    ty, tw, tv = barrier_diagonals(data, st)
    Lm = disc.A.tocsc()
    r = np.random.default_rng(5).normal(size=4 * n)
    ry, rw, rv, rp = r[:n], r[n:2 * n], r[2 * n:3 * n], r[3 * n:]
    det = a * (tw + tv) + tw * tv
    vw = ((a + tv) * rw + a * rv) / det
    vv = (a * rw + (a + tw) * rv) / det
    v1 = spla.spsolve(Lm, vw - vv + rp)
    ml = data.obs + ty
    sig = (tw + tv) / det
    s1 = spla.spsolve((Lm.T + sp.diags(ml)).tocsc(), ml * v1 - ry)
    v3 = spla.spsolve((Lm + sp.diags(sig)).tocsc(), Lm @ s1)
    ref = np.concatenate([v1, vw, vv, v3])
    o = Options(sigma=data.sigma, krylov="fgmres", precond="ppi", mg_precision="fp64", vcycles=8)
    with Problem(data) as prob:
        _load_state(prob, st, False)
        prob.newton_setup(mu, o)
        z = prob.apply_precond(torch.tensor(r, device="cuda", dtype=torch.float64), o).cpu().numpy()
    errs = [_rel(z[k * n:(k + 1) * n], ref[k * n:(k + 1) * n]) for k in range(4)]
    print("  block rel errors", [f"{e:.1e}" for e in errs], flush=True)
    assert errs[1] <= 1e-13 and errs[2] <= 1e-13
    assert errs[0] <= 1e-4 and errs[3] <= 1e-4


def test_ppi_batch_equals_solo():
    """Partial-observation problems of different sizes in one batch (the
    multigrid reaction-term slots switch for every instance at once) give each
    instance its solo result bit for bit."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.poisson2d_partial(seed=s, N=N) for s, N in ((0, 31), (1, 63), (2, 127), (3, 63))]
    o = Options(sigma=0.25, krylov="fgmres", precond="ppi")
    solo = []
    for d in datas:
        with Problem(d) as p:
            p.solve(o)
            solo.append((p.query("u"), p.stats().krylov_its))
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        st = b.solve(o)
    for p, (u, its) in zip(probs, solo):
        assert p.stats().krylov_its == its
        np.testing.assert_array_equal(p.query("u"), u)
        p.close()
    assert st == [0, 0, 0, 0]


def test_ppi_newton_direction_full_size():
    """255^2 partial observation: the GPU Newton direction (FGMRES + P_Pi) from a
    mid-solve state solves the oracle's sparse FP64 system to 1e-10 (or the FP64
    attainable-accuracy floor)."""
    from paper_1806_05896_amd import Options, Problem
    data = W.poisson2d_partial(seed=0, N=255)
    opts = Options(sigma=data.sigma, krylov="fgmres", precond="ppi")
    print("[ppi-255] newton direction", flush=True)
    with Problem(data) as prob:
        mu = 1.0
        for _ in range(3):
            mu *= data.sigma
            prob.ipm_step(mu, opts)
        q = prob.query
        st = IPMState(q("y"), q("w"), q("v"), q("p"), q("lam_wa"), q("lam_wb"), q("lam_va"), q("lam_vb"), mu=mu)
        mu *= data.sigma
        info = prob.newton_direction(mu, opts)
        dx = np.concatenate([prob.query(f) for f in ("dy", "dw", "dv", "dp")])
    disc = discretize(data)
    K = newton_matrix(data, disc, st).tocsr()
    b = newton_rhs(data, disc, st, mu)
    res = np.linalg.norm(b - K @ dx) / np.linalg.norm(b)
    floor = 16 * np.finfo(float).eps * np.linalg.norm(abs(K) @ np.abs(dx) + np.abs(b)) / np.linalg.norm(b)
    print(f"  its={info['krylov_its']} rel residual {res:.2e} (floor {floor:.2e})", flush=True)
    assert res <= max(1e-10, floor) * 1.01
