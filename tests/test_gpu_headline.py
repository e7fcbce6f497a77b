"""The 2D Poisson 511^2 workload exactly as the benchmark runs it: a batch of
eight instances (seeds 0..7) with MINRES + P_D and FP32 V-cycles, whose
launches serve all eight and so take the large-tile multigrid level kernels.

* every member of the batch equals its solo solve bit for bit (a solo
  511^2 solve takes the small tiles: the tile size changes no node's
  arithmetic);
* seed 0 matches the CPU oracle's solution (Algorithm A.1 with SuperLU on the
  eliminated SPD Newton system, tolerance 1e-6 of Sec. 5) to a relative L2
  error of 1e-6 in u, y and p with the same number of IPM iterations; the
  oracle's own error at that tolerance (its distance from the 1e-12 run) is
  printed beside it (its 1e-6 control against its own tight run).  The
  oracle solution is stored by
  tests/golden/make_oracle_solutions.py, which calls only the oracle."""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "poisson2d_511_seed0_oracle.npz")


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


TUNE_CACHE = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1806_05896_amd", "autotune_cache.json")


@pytest.fixture(scope="module")
def batch8():
    """The benchmarked batch, with the multigrid schedule the benchmark takes
    from the autotuner's cache: results of each member, and of each solo solve
    (level-kernel tiles chosen per launch)."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.poisson2d_511(seed=s) for s in range(8)]
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        tuned, _, hit = b.autotune(Options(sigma=datas[0].sigma, mg_precision="fp32"), cache=TUNE_CACHE)
        print(f"[headline] batch of 8 x 511^2, MINRES + P_D, schedule {tuned} (cache hit {hit})", flush=True)
        st = b.solve(tuned)
    opts = [Options(**{**tuned.__dict__, "mg_tile": "auto"}) for d in datas]
    batch = [(st[k], probs[k].query("u"), probs[k].query("y"), probs[k].query("p"), probs[k].stats())
             for k in range(8)]
    for p in probs:
        p.close()
    solo = []
    for k, (d, o) in enumerate(zip(datas, opts)):
        print(f"[headline] solo solve seed {k}", flush=True)
        with Problem(d) as p:
            rc = p.solve(o)
            solo.append((rc, p.query("u"), p.query("y"), p.query("p"), p.stats()))
    return datas, batch, solo, tuned


def test_batch_of_eight_equals_solo_bit_for_bit(batch8):
    datas, batch, solo, _ = batch8
    for k in range(8):
        rb, ub, yb, pb, sb = batch[k]
        rs, us, ys, ps, ss = solo[k]
        print(f"  seed {k}: rc {rb}/{rs} nli {sb.nli}/{ss.nli} its {sb.krylov_its}/{ss.krylov_its} "
              f"max|du| {np.abs(ub - us).max():.1e}", flush=True)
        assert rb == rs == 0
        assert sb.nli == ss.nli and sb.krylov_its == ss.krylov_its
        assert sb.hist_krylov == ss.hist_krylov
        np.testing.assert_array_equal(ub, us)
        np.testing.assert_array_equal(yb, ys)
        np.testing.assert_array_equal(pb, ps)


def test_seed0_matches_the_oracle_at_511(batch8):
    datas, batch, _, _ = batch8
    g = np.load(GOLDEN, allow_pickle=False)
    assert str(g["digest"]) == _digest(datas[0]), "stored oracle solution is for other inputs"
    rc, u, y, p, st = batch[0]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    eu, ey, ep = rel(u, g["u"]), rel(y, g["y"]), rel(p, g["p"])
    hist = json.loads(str(g["history"]))
    print(f"  511^2 seed 0: nli {st.nli} (oracle {int(g['nli'])}); rel L2 u {eu:.2e} y {ey:.2e} p {ep:.2e}; "
          f"FP64-oracle error u {float(g['oracle_error_u']):.2e} y {float(g['oracle_error_y']):.2e} "
          f"(oracle at 1e-6 against its tight run, {str(g['tight_rule'])} rule, {int(g['nli_tight'])} iterations)",
          flush=True)
    for k in range(min(st.nli, len(hist) - 1)):
        print(f"    k={k} mu {st.hist_mu[k]:.3e}/{hist[k]['mu']:.3e} alpha_P {st.hist_alpha_p[k]:.6f}/"
              f"{hist[k]['alpha_P']:.6f} alpha_D {st.hist_alpha_d[k]:.6f}/{hist[k]['alpha_D']:.6f} "
              f"krylov {st.hist_krylov[k]} relres {st.hist_krylov_relres[k]:.1e}", flush=True)
    assert rc == 0 and str(g["status"]) == "converged"
    assert st.nli == int(g["nli"])
    assert np.isfinite(float(g["oracle_error_u"]))
    assert eu <= 1e-6 and ey <= 1e-6 and ep <= 1e-6


@pytest.mark.parametrize("N,count", [(511, 1), (127, 3)])
def test_tile_size_changes_no_result(N, count):
    """The large and the small tiles of the 2D Poisson level kernels give
    bit-identical solves (one 511^2 instance, and a batch at 127^2 where the
    automatic choice would take the small tiles)."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.poisson2d_511(seed=s, N=N) for s in range(count)]
    res = {}
    for tile in ("small", "large"):
        print(f"[tiles] N={N} x{count} {tile}", flush=True)
        probs = [Problem(d) for d in datas]
        with Batch(probs) as b:
            st = b.solve(Options(sigma=datas[0].sigma, mg_tile=tile))
        res[tile] = [(st[k], p.query("u"), p.query("p"), p.stats().krylov_its) for k, p in enumerate(probs)]
        for p in probs:
            p.close()
    for a, c in zip(res["small"], res["large"]):
        assert a[0] == c[0] == 0 and a[3] == c[3]
        np.testing.assert_array_equal(a[1], c[1])
        np.testing.assert_array_equal(a[2], c[2])
