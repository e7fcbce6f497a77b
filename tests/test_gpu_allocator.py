"""Device memory through PyTorch's caching allocator (ipmpde_set_allocator,
registered by use_torch_allocator): the library takes every device buffer
from the callback and the results equal those of the default hipMalloc path
bit for bit, for a single solve, a batch and a served mix."""
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


def _solo(d, o):
    from paper_1806_05896_amd import Problem
    with Problem(d) as p:
        rc = p.solve(o)
        return rc, p.query("u"), p.query("y"), p.query("p"), p.stats()


def test_solve_through_the_torch_allocator():
    from paper_1806_05896_amd import Options, Problem, use_torch_allocator
    d = W.poisson2d_511(seed=2, N=63)
    o = Options(sigma=d.sigma)
    ref = _solo(d, o)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    use_torch_allocator(True)
    try:
        p = Problem(d)
        held_data = torch.cuda.memory_allocated() - base
        rc = p.solve(o)
        held_solve = torch.cuda.memory_allocated() - base
        got = (rc, p.query("u"), p.query("y"), p.query("p"), p.stats())
        p.close()
        torch.cuda.synchronize()
        left = torch.cuda.memory_allocated() - base
    finally:
        use_torch_allocator(False)
    print(f"[allocator] bytes held through torch: data {held_data}, during solve {held_solve}, after {left}",
          flush=True)
    assert held_data > 0 and held_solve > held_data and left == 0
    assert got[0] == ref[0] == 0
    assert got[4].nli == ref[4].nli and got[4].krylov_its == ref[4].krylov_its
    for a, b in zip(got[1:4], ref[1:4]):
        np.testing.assert_array_equal(a, b)


def test_batch_and_engine_through_the_torch_allocator():
    from paper_1806_05896_amd import Batch, Engine, Options, Problem, use_torch_allocator
    datas = [d for _, d in W.served_requests(n_requests=6, seed=3, sizes=(31, 63))]
    opts = [Options(sigma=d.sigma, krylov="fgmres" if d.pde == "convdiff" else "minres",
                    precond="pt" if d.pde == "convdiff" else "pd") for d in datas]
    refs = [_solo(d, o) for d, o in zip(datas, opts)]
    use_torch_allocator(True)
    try:
        mine = [d for d, o in zip(datas, opts) if o.krylov == "minres"]
        idx = [k for k, o in enumerate(opts) if o.krylov == "minres"]
        probs = [Problem(d) for d in mine]
        with Batch(probs) as b:
            b.solve([opts[k] for k in idx])
        for k, p in zip(idx, probs):
            np.testing.assert_array_equal(p.query("u"), refs[k][1])
            assert p.stats().nli == refs[k][4].nli
            p.close()
        probs = [Problem(d) for d in datas]
        with Engine(1 << 30, 4) as e:
            tickets = [e.submit(p, o) for p, o in zip(probs, opts)]
            e.run()
            for k, t in enumerate(tickets):
                assert e.poll(t)["status"] == refs[k][0] == 0
        for k, p in enumerate(probs):
            np.testing.assert_array_equal(p.query("u"), refs[k][1])
            np.testing.assert_array_equal(p.query("y"), refs[k][2])
            p.close()
    finally:
        use_torch_allocator(False)
