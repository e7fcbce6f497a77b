"""Serving engine: continuous batching with admission by HBM footprint.

Each request's result must be the same alone and in the mix.  The engine
gives every request the arithmetic of its solo solve, so the comparison is
exact (bit-identical iterates, equal iteration counts)."""
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


def _solo(datas, opts):
    from paper_1806_05896_amd import Problem
    out = []
    for d, o in zip(datas, opts):
        with Problem(d) as p:
            rc = p.solve(o)
            out.append((rc, p.query("u"), p.query("y"), p.stats()))
    return out


def _drive(eng, probs, opts, arrive_at_step, check=None):
    """Submit request i at engine step arrive_at_step[i]; step until drained."""
    tickets = [None] * len(probs)
    step = 0
    while True:
        for i, s in enumerate(arrive_at_step):
            if s == step:
                tickets[i] = eng.submit(probs[i], opts[i])
        running, queued = eng.step()
        if check:
            check(eng)
        step += 1
        if running == 0 and queued == 0 and step > max(arrive_at_step):
            return tickets
        assert step < 5000


def test_engine_solo_vs_mix():
    from paper_1806_05896_amd import Engine, Options, Problem
    reqs = W.served_requests(n_requests=10, seed=3, sizes=(31, 63, 127))
    datas = [d for _, d in reqs]
    opts = [Options(sigma=d.sigma, krylov="fgmres" if d.pde == "convdiff" else "minres",
                    precond="pt" if d.pde == "convdiff" else "pd") for d in datas]
    print("[engine] sizes", [d.N for d in datas], "pdes", [d.pde for d in datas], flush=True)
    solo = _solo(datas, opts)
    probs = [Problem(d) for d in datas]
    arrive = [0, 0, 0, 2, 3, 5, 5, 9, 14, 20]
    with Engine(hbm_budget_bytes=1 << 40, max_slots=4) as eng:
        tickets = _drive(eng, probs, opts, arrive,
                         check=lambda e: (e.info()["running"] <= 4) or pytest.fail("slot limit exceeded"))
        for k, (p, t, (rc, u, y, s)) in enumerate(zip(probs, tickets, solo)):
            info = eng.poll(t)
            sb = p.stats()
            print(f"  {k}: N={p.N} {datas[k].pde} rc={rc}/{info['status']} nli={s.nli}/{sb.nli} "
                  f"its={s.krylov_its}/{sb.krylov_its} lat={info['latency_ms']:.1f}ms", flush=True)
            assert info["state"] == 2 and info["status"] == rc == 0
            assert sb.nli == s.nli and sb.krylov_its == s.krylov_its
            np.testing.assert_array_equal(p.query("u"), u)
            np.testing.assert_array_equal(p.query("y"), y)
            eng.release(t)
    for p in probs:
        p.close()


def test_engine_serves_q1_beside_finite_differences():
    """Q1 requests form their own group in the engine; every result equals its
    solo solve bit for bit."""
    from paper_1806_05896_amd import Engine, Options, Problem
    datas = [W.poisson2d_q1(seed=0, N=31), W.poisson2d_small(seed=1, N=31), W.poisson2d_q1(seed=2, N=63),
             W.poisson2d_small(seed=3, N=63)]
    opts = [Options(sigma=d.sigma, krylov="minres", precond="pd") for d in datas]
    solo = _solo(datas, opts)
    probs = [Problem(d) for d in datas]
    with Engine(hbm_budget_bytes=1 << 40, max_slots=4) as eng:
        tickets = _drive(eng, probs, opts, [0, 0, 1, 2])
        for p, t, (rc, u, y, s) in zip(probs, tickets, solo):
            info = eng.poll(t)
            assert info["state"] == 2 and info["status"] == rc == 0
            assert p.stats().nli == s.nli and p.stats().krylov_its == s.krylov_its
            np.testing.assert_array_equal(p.query("u"), u)
            eng.release(t)
    for p in probs:
        p.close()


def test_engine_admission_by_footprint():
    """Budget for the two largest requests: the admitted bytes never exceed
    it, so fewer run than slots allow while others wait, and every request
    completes."""
    from paper_1806_05896_amd import Engine, Options, Problem, footprint_bytes
    reqs = W.served_requests(n_requests=6, seed=4, sizes=(63,))
    datas = [d for _, d in reqs]
    opts = [Options(sigma=d.sigma, krylov="fgmres" if d.pde == "convdiff" else "minres",
                    precond="pt" if d.pde == "convdiff" else "pd") for d in datas]
    fps = [footprint_bytes(2, d.N, d.pde, False, o) for d, o in zip(datas, opts)]
    budget = sorted(fps)[-1] + sorted(fps)[-2]
    probs = [Problem(d) for d in datas]
    seen = []

    fit = max(k for k in range(1, len(fps) + 1) if sum(sorted(fps)[:k]) <= budget)

    def check(e):
        info = e.info()
        seen.append((info["running"], info["queued"]))
        assert info["bytes_in_use"] <= budget and info["peak_bytes"] <= budget

    with Engine(hbm_budget_bytes=budget, max_slots=16) as eng:
        tickets = _drive(eng, probs, opts, [0] * len(probs), check)
        assert 1 <= max(r for r, _ in seen) <= fit < len(probs)
        assert any(q > 0 for _, q in seen)  # the budget, not the slots, held requests back
        for t in tickets:
            assert eng.poll(t)["status"] == 0
    for p in probs:
        p.close()


def test_engine_rejects_oversized_and_isolates_failures():
    from paper_1806_05896_amd import Engine, Options, Problem, footprint_bytes
    from paper_1806_05896_amd import _lib as L
    reqs = W.served_requests(n_requests=4, seed=5, sizes=(31, 63))
    datas = [d for _, d in reqs]
    opts = [Options(sigma=d.sigma, krylov="fgmres" if d.pde == "convdiff" else "minres",
                    precond="pt" if d.pde == "convdiff" else "pd") for d in datas]
    opts[1] = Options(sigma=datas[1].sigma, ipm_maxit=2, krylov=opts[1].krylov, precond=opts[1].precond)
    solo = _solo(datas, opts)
    probs = [Problem(d) for d in datas]
    small = min(footprint_bytes(2, d.N, d.pde, False, o) for d, o in zip(datas, opts))
    with Engine(hbm_budget_bytes=small - 1, max_slots=2) as eng:
        with pytest.raises(L.IpmpdeError) as ei:
            eng.submit(probs[0], opts[0])
        assert ei.value.code == L.ENOMEM
    with Engine(hbm_budget_bytes=1 << 40, max_slots=2) as eng:
        tickets = _drive(eng, probs, opts, [0, 0, 1, 1])
        st = [eng.poll(t)["status"] for t in tickets]
        assert st[1] == L.ENOTCONVERGED and probs[1].stats().nli == 2
        for k in (0, 2, 3):
            assert st[k] == 0
            np.testing.assert_array_equal(probs[k].query("u"), solo[k][1])
        # a finished problem is usable again on its own
        assert probs[0].solve(opts[0]) == 0
        np.testing.assert_array_equal(probs[0].query("u"), solo[0][1])
    for p in probs:
        p.close()
