"""The FP64-oracle error stated beside a whole-solve parity result: the
relative distance of the oracle's control at the paper's tolerance (1e-6,
Sec. 5) from the optimum, estimated by the oracle's own run to 1e-10
(primal), 1e-11 (dual) and 1e-12 (complementarity) -- the first two near
their FP64 rounding floors on fine grids -- under the same barrier rule, or
under the
iterate-based rule where the fixed decrease of Algorithm A.1 loses the
interior first.  It is O(mu / alpha)
and often far above the 1e-6 parity bar, which is why parity is taken on the
IPM trajectory at equal tolerance rather than on the optimum."""
import dataclasses

import numpy as np

import oracle


def fp64_oracle_error(data, opts, ref) -> float:
    tight = dataclasses.replace(opts, eps_p=1e-10, eps_d=1e-11, eps_c=1e-12)
    r = oracle.solve(data, tight)
    if r.status != "converged":
        r = oracle.solve(data, dataclasses.replace(tight, mu_rule="central"))
    if r.status != "converged":
        return float("nan")
    return float(np.linalg.norm(ref.u - r.u) / max(np.linalg.norm(r.u), np.sqrt(r.u.size) * 1e-3))
