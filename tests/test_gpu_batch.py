"""Batched solves: several unevenly sized problems advanced by the same
kernel launches give each problem the result of its solo solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _mixed(seed=0):
    reqs = W.served_requests(n_requests=12, seed=seed, sizes=(31, 63, 127))
    return [d for _, d in reqs]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_solo(prec):
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = _mixed()
    print("[batch] sizes", [d.N for d in datas], "pdes", [d.pde for d in datas], flush=True)
    opts = [Options(sigma=d.sigma, mg_precision=prec) for d in datas]
    solo = []
    for d, o in zip(datas, opts):
        with Problem(d) as p:
            rc = p.solve(o)
            solo.append((rc, p.query("u"), p.query("y"), p.stats()))
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        st = b.solve(opts)
    for k, (p, (rc, u, y, s)) in enumerate(zip(probs, solo)):
        ub, yb, sb = p.query("u"), p.query("y"), p.stats()
        print(f"  {k}: N={p.N} rc={rc}/{st[k]} nli={s.nli}/{sb.nli} its={s.krylov_its}/{sb.krylov_its} "
              f"max|du|={np.abs(ub - u).max():.1e}", flush=True)
        assert st[k] == rc == 0
        assert sb.nli == s.nli and sb.krylov_its == s.krylov_its
        np.testing.assert_array_equal(ub, u)
        np.testing.assert_array_equal(yb, y)
        p.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_3d_equals_solo(prec):
    """3D finite-difference problems of different sizes in one batch (the fused cube level
    kernels for the 31^3 and 63^3 members, the whole hierarchy in the coarse kernel for the
    15^3 one) give each member its solo result bit for bit."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = [W.poisson3d_127(seed=1, N=31), W.poisson3d_127(seed=2, N=15), W.poisson3d_127(seed=3, N=63)]
    print("[batch3d]", prec, [d.N for d in datas], flush=True)
    opts = [Options(sigma=d.sigma, mg_precision=prec) for d in datas]
    solo = []
    for d, o in zip(datas, opts):
        with Problem(d) as p:
            rc = p.solve(o)
            solo.append((rc, p.query("u"), p.stats()))
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        st = b.solve(opts)
    for k, (p, (rc, u, s)) in enumerate(zip(probs, solo)):
        ub, sb = p.query("u"), p.stats()
        print(f"  {k}: N={p.N} rc={rc}/{st[k]} nli={s.nli}/{sb.nli} its={s.krylov_its}/{sb.krylov_its} "
              f"max|du|={np.abs(ub - u).max():.1e}", flush=True)
        assert st[k] == rc == 0
        assert sb.nli == s.nli and sb.krylov_its == s.krylov_its
        np.testing.assert_array_equal(ub, u)
        p.close()


@pytest.fixture(scope="module")
def mixed_solo():
    from paper_1806_05896_amd import Options, Problem
    datas = _mixed(seed=3)
    opts = [Options(sigma=d.sigma) for d in datas]
    solo = []
    for d, o in zip(datas, opts):
        with Problem(d) as p:
            rc = p.solve(o)
            solo.append((rc, p.query("u"), p.stats()))
    return datas, opts, solo


@pytest.mark.parametrize("lanes", [2, 5, 16])
def test_batch_lanes_equal_solo(lanes, mixed_solo):
    """The instances split into lanes (sub-batches, each on a stream of its own and driven
    by a host thread of its own; 16 is clamped to the batch's 12 instances) give each
    member its solo result bit for bit, and so does the same batch solved again in one lane."""
    from dataclasses import replace

    from paper_1806_05896_amd import Batch, Problem
    datas, opts, solo = mixed_solo
    print(f"[lanes] {lanes} lanes, sizes {[d.N for d in datas]}", flush=True)
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        for ln in (lanes, 1):
            st = b.solve([replace(o, lanes=ln) for o in opts])
            for k, (p, (rc, u, s)) in enumerate(zip(probs, solo)):
                ub, sb = p.query("u"), p.stats()
                print(f"  lanes {ln} member {k}: N={p.N} rc={rc}/{st[k]} its={s.krylov_its}/{sb.krylov_its}",
                      flush=True)
                assert st[k] == rc == 0
                assert sb.nli == s.nli and sb.krylov_its == s.krylov_its
                np.testing.assert_array_equal(ub, u)
    for p in probs:
        p.close()


def test_autotuner_picks_lanes_and_keeps_results(mixed_solo, tmp_path):
    """The autotuner times lane splits too; its pick solves every member to its solo result."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas, opts, solo = mixed_solo
    datas, solo = datas[:4], solo[:4]
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        best, ms, hit = b.autotune(Options(sigma=datas[0].sigma), cache=str(tmp_path / "tune.json"))
        print(f"[lanes] autotuner pick {best} ({ms:.1f} ms, cache hit {hit})", flush=True)
        assert not hit and 1 <= best.lanes <= 4
        best2, _, hit2 = b.autotune(Options(sigma=datas[0].sigma), cache=str(tmp_path / "tune.json"))
        assert hit2 and best2.lanes == best.lanes and best2.nu_pre == best.nu_pre
        st = b.solve([Options(**{**best.__dict__, "sigma": d.sigma}) for d in datas])
    for k, (p, (rc, u, s)) in enumerate(zip(probs, solo)):
        if best.vcycles == 1 and best.nu_pre == 2 and best.mg_precision == "fp32":
            assert st[k] == rc == 0 and p.stats().krylov_its == s.krylov_its
            np.testing.assert_array_equal(p.query("u"), u)
        else:
            assert st[k] == 0
        p.close()


def test_batch_member_limits_do_not_leak():
    """One member with an IPM iteration limit of 2 stops early (ENOTCONVERGED);
    its batch-mates converge exactly as they would alone."""
    from paper_1806_05896_amd import Batch, Options, Problem
    datas = _mixed(seed=1)[:5]
    opts = [Options(sigma=d.sigma) for d in datas]
    opts[2] = Options(sigma=datas[2].sigma, ipm_maxit=2)
    probs = [Problem(d) for d in datas]
    with Batch(probs) as b:
        st = b.solve(opts)
    assert st[2] == 4 and probs[2].stats().nli == 2
    for k in (0, 1, 3, 4):
        with Problem(datas[k]) as p:
            p.solve(opts[k])
            np.testing.assert_array_equal(p.query("u"), probs[k].query("u"))
        assert st[k] == 0
    for p in probs:
        p.close()


def test_poisoned_member_is_isolated():
    """A member whose data overflow in FP64 (desired state of size 1e300, finite
    and accepted at create) fails (EBREAKDOWN or EKRYLOV) with NaN or Inf
    confined to its own iterates; its batch-mates and the requests served beside it in an engine
    group finish exactly as they would alone."""
    from paper_1806_05896_amd import Batch, Engine, Options, Problem
    from paper_1806_05896_amd import _lib as L
    datas = [d for d in _mixed(seed=2) if d.pde == "poisson"][:2]
    bad = datas[0].copy()
    bad.y_d = bad.y_d * 1e300
    members = [datas[0], bad, datas[1]]
    opts = [Options(sigma=d.sigma) for d in members]
    solo = []
    for k in (0, 2):
        with Problem(members[k]) as p:
            rc = p.solve(opts[k])
            solo.append((k, rc, p.query("u"), p.stats().krylov_its))
    probs = [Problem(d) for d in members]
    with Batch(probs) as b:
        st = b.solve(opts)
    print(f"[poison] batch status {st}", flush=True)
    assert st[1] in (L.EBREAKDOWN, L.EKRYLOV)
    for k, rc, u, its in solo:
        assert st[k] == rc == 0 and probs[k].stats().krylov_its == its
        np.testing.assert_array_equal(probs[k].query("u"), u)
    for p in probs:
        p.close()
    probs = [Problem(d) for d in members]
    with Engine(1 << 30, 8) as e:
        tickets = [e.submit(p, o) for p, o in zip(probs, opts)]
        e.run()
        status = [e.poll(t)["status"] for t in tickets]
    print(f"[poison] engine status {status}", flush=True)
    assert status[1] in (L.EBREAKDOWN, L.EKRYLOV)
    for k, rc, u, its in solo:
        assert status[k] == rc == 0
        np.testing.assert_array_equal(probs[k].query("u"), u)
    for p in probs:
        p.close()
