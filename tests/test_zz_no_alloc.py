"""ipmpde_measures_noalloc, the measures entry point that allocates no device
memory (its scratch is a device array of the library), against
ipmpde_measures on the same iterates: equal bit for bit, on two calls in a
row with the second problem smaller than the first, and without a change of
the device's free memory."""
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


def test_measures_noalloc_equals_measures():
    from paper_1806_05896_amd import Options, Problem
    from paper_1806_05896_amd import _lib as L
    cases = [(W.poisson2d_511(seed=1, N=127), 3),      # 16,129 nodes, state bounds
             (W.convdiff2d_255(seed=2, N=31), 2)]      # 961 nodes: the smaller second call
    for d, steps in cases:
        print(f"[noalloc] {d.pde} N={d.N} after {steps} IPM iterations", flush=True)
        with Problem(d) as p:
            with pytest.raises(L.IpmpdeError):       # iterates not set yet
                p.measures_noalloc()
            kry = "fgmres" if d.pde == "convdiff" else "minres"
            rc = p.solve(Options(sigma=d.sigma, ipm_maxit=steps, krylov=kry, precond="pt" if kry == "fgmres" else "pd"))
            assert rc == L.ENOTCONVERGED
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            a = p.measures_noalloc()
            a2 = p.measures_noalloc()
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            b = p.measures()
            print(f"  noalloc {a} measures {b} free memory {free0} -> {free1}", flush=True)
            assert np.array_equal(np.array(a), np.array(b)) and np.array_equal(np.array(a2), np.array(b))
            assert all(np.isfinite(a)) and max(a) > 0
            assert free1 == free0
