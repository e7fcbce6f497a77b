"""Write stored oracle solutions for the GPU parity tests whose oracle runs
take minutes.

Each entry runs only the CPU oracle (Algorithm A.1 with a SuperLU Newton
solve) on seeded inputs from `workloads`, at the paper's tolerance 1e-6
(Sec. 5), and stores u, y, p, the iteration count and history, and the
FP64-oracle error: the distance of the 1e-6 control from the oracle's own
run to the tight tolerances 1e-10 (primal), 1e-11 (dual) and 1e-12
(complementarity), same barrier rule, or the iterate-based rule where the
fixed decrease of Algorithm A.1 loses the interior first.  The primal and
dual measures stop there because they bottom out at their FP64 rounding
floors (at 511^2, where A's diagonal is 4 / h^2 = 1e6: 3.6e-11 and 4e-12).
A digest of the inputs lets a test notice a changed generator.

  poisson2d_511_seed0   the 2D Poisson 511^2 workload, seed 0 (the
                        benchmarked configuration; eliminated SPD Newton
                        system), the paper's barrier rule
  q1_3d_sb15_central    3D Poisson with trilinear Q1 elements on 15^3, seed 0,
                        state bounds [-0.06, 0.06], the iterate-based barrier
                        rule
  q1_3d_sb15_paper      the same instance under the paper's barrier rule
  convdiff2d_127_seed0  the convection-diffusion workload (eps = 1/200) on
                        127^2, seed 0, the paper's barrier rule
  poisson3d_31_seed0    the 3D finite-difference Poisson workload on 31^3,
                        seed 0, the paper's barrier rule

Usage:  python tests/golden/make_oracle_solutions.py [name ...]
"""
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def input_digest(p) -> str:
    h = hashlib.sha256()
    for a in (p.y_d, p.u_a, p.u_b, p.y_a, p.y_b):
        if a is not None:
            h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    h.update(np.array([p.alpha, p.beta, p.sigma], dtype=np.float64).tobytes())
    return h.hexdigest()


def q1_3d_bounded(N):
    d = W.poisson3d_q1(seed=0, N=N)
    d.y_a = np.full(d.n, -0.06)
    d.y_b = np.full(d.n, 0.06)
    return d


CASES = {
    "poisson2d_511_seed0": (lambda: W.poisson2d_511(seed=0),
                            lambda d: oracle.IPMOptions(sigma=d.sigma, newton="schur")),
    "q1_3d_sb15_central": (lambda: q1_3d_bounded(15),
                           lambda d: oracle.IPMOptions(sigma=d.sigma, mu_rule="central")),
    "q1_3d_sb15_paper": (lambda: q1_3d_bounded(15),
                         lambda d: oracle.IPMOptions(sigma=d.sigma)),
    "convdiff2d_127_seed0": (lambda: W.convdiff2d_255(seed=0, N=127),
                             lambda d: oracle.IPMOptions(sigma=d.sigma)),
    "poisson3d_31_seed0": (lambda: W.poisson3d_127(seed=0, N=31),
                           lambda d: oracle.IPMOptions(sigma=d.sigma)),
}


def make(name):
    data_fn, opts_fn = CASES[name]
    p = data_fn()
    opts = opts_fn(p)
    t0 = time.time()
    r = oracle.solve(p, opts)
    print(f"{name}: eps=1e-6 status={r.status} nli={r.nli} ({time.time() - t0:.1f} s)", flush=True)
    tight = dataclasses.replace(opts, eps_p=1e-10, eps_d=1e-11, eps_c=1e-12)
    rt = oracle.solve(p, tight)
    rule = opts.mu_rule
    if rt.status != "converged":
        print(f"  tight run under the {rule} rule: {rt.status} at {rt.nli}; the iterate-based rule instead", flush=True)
        rt = oracle.solve(p, dataclasses.replace(tight, mu_rule="central"))
        rule = "central"
    print(f"  tight run ({rule} rule): status={rt.status} nli={rt.nli} ({time.time() - t0:.1f} s)", flush=True)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), u=r.u, y=r.y, p=r.p, nli=r.nli, status=r.status,
                        nli_tight=rt.nli, tight_status=rt.status, tight_rule=rule,
                        oracle_error_u=rel(r.u, rt.u), oracle_error_y=rel(r.y, rt.y),
                        history=json.dumps(r.history), digest=input_digest(p))
    print(f"  FP64-oracle error u {rel(r.u, rt.u):.3e} y {rel(r.y, rt.y):.3e}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        make(name)
