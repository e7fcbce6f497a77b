"""Whole-solve parity at sizes whose oracle runs take minutes: the GPU solve
against the oracle's solution of the same seeded inputs, stored by
tests/golden/make_oracle_solutions.py (which calls only the oracle), with the
FP64-oracle error printed beside each result.

* 2D convection-diffusion (eps = 1/200, wind of Sec. 5.2) on 127^2 with the
  solver of the 255^2 benchmark (FGMRES(30) + P_T, FP32 V-cycles) and with
  MINRES + P_D;
* 3D Poisson (7-point finite differences) on 31^3 with MINRES + P_D and FP32
  V-cycles (the solver of the 127^3 benchmark), the size at which the finest
  3D levels leave the single-workgroup coarse kernel.
Bar: the same number of IPM iterations and rel-L2 <= 1e-6 in u, y and p."""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _digest(p) -> str:
    h = hashlib.sha256()
    for a in (p.y_d, p.u_a, p.u_b, p.y_a, p.y_b):
        if a is not None:
            h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    h.update(np.array([p.alpha, p.beta, p.sigma], dtype=np.float64).tobytes())
    return h.hexdigest()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), np.sqrt(b.size) * 1e-3))


CASES = {
    "convdiff2d_127_seed0": lambda: W.convdiff2d_255(seed=0, N=127),
    "poisson3d_31_seed0": lambda: W.poisson3d_127(seed=0, N=31),
}


@pytest.mark.parametrize("name,krylov,precond", [("convdiff2d_127_seed0", "fgmres", "pt"),
                                                 ("convdiff2d_127_seed0", "minres", "pd"),
                                                 ("poisson3d_31_seed0", "minres", "pd")])
def test_whole_solve_against_stored_oracle(name, krylov, precond):
    from paper_1806_05896_amd import Options, Problem
    g = np.load(os.path.join(GOLDEN, f"{name}_oracle.npz"), allow_pickle=False)
    data = CASES[name]()
    assert str(g["digest"]) == _digest(data), "stored oracle solution is for other inputs"
    print(f"[stored] {name} {krylov} {precond} fp32", flush=True)
    with Problem(data) as prob:
        rc = prob.solve(Options(sigma=data.sigma, krylov=krylov, precond=precond, mg_precision="fp32"))
        u, y, p = prob.query("u"), prob.query("y"), prob.query("p")
        s = prob.stats()
    hist = json.loads(str(g["history"]))
    worst = max(s.hist_krylov_relres[:s.nli]) if s.nli else 0.0
    print(f"  rc={rc} nli={s.nli}/{int(g['nli'])} its={s.krylov_its} worst Krylov relres {worst:.1e}; rel u "
          f"{_rel(u, g['u']):.2e} y {_rel(y, g['y']):.2e} p {_rel(p, g['p']):.2e}; FP64-oracle error u "
          f"{float(g['oracle_error_u']):.2e} (tight run {str(g['tight_rule'])} rule, {int(g['nli_tight'])} its)",
          flush=True)
    assert str(g["status"]) == "converged" and len(hist) == int(g["nli"]) + 1
    assert rc == 0 and s.nli == int(g["nli"])
    assert _rel(u, g["u"]) <= 1e-6 and _rel(y, g["y"]) <= 1e-6 and _rel(p, g["p"]) <= 1e-6
