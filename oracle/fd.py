"""Finite-difference discretization of the state equation (oracle).

The paper discretizes with Q1 finite elements (Sec. 2 and Sec. 5); this
oracle follows the finite-difference reading used throughout the build:

* grid: N interior points per axis on (0,1)^d, h = 1/(N+1), x_i = i h;
* Poisson (eq. (eq:lap)): (A y)_i = h^-2 (2d y_i - sum of the 2d neighbours);
* convection-diffusion (Sec. 5.2, -eps Lap y + w.grad y = u): A = eps A_Poisson + C
  with first-order upwinding at node values,
      (C y)_i = sum_a [max(w_a,0)(y_i - y_{i-e_a}) + min(w_a,0)(y_{i+e_a} - y_i)] / h,
  wind w = (2 x2 (1 - x1^2), -2 x1 (1 - x2^2));
* unit mass scaling: M = D = D_M = I.  The FEM-style weighting M = h^d I only
  rescales the objective and the constraint by h^d, which leaves the
  minimizer unchanged (Sec. 2, eq. (pb_fe)).

Dirichlet data g (eq. (eq:lap), y = g on the boundary) enters through the
boundary columns of the full operator: A_II y_I = f - A_IB g_B =: f_hat.

Heat equation y_t - Lap y = u + f (Sec. 4.4), all at once: backward Euler
with step tau on nt steps gives the block lower bidiagonal matrix of Sec.
4.4 (M + tau L on the diagonal, -M below it) acting on the states at
t_1..t_nt.  With M = I and the whole constraint divided by tau (the time
counterpart of the unit mass scaling; the objective's rectangle-rule weight
tau is divided out likewise, which again leaves the minimizer unchanged),
the state operator is

    A = blocks I/tau + A_h on the diagonal, -I/tau below it,

A_h the 2D Poisson matrix, and the initial state y0 moves to the right-hand
side of the first step: f_hat_1 = f_1 - A_IB g_B + y0 / tau.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def _wind(x1: np.ndarray, x2: np.ndarray):
    """Wind of the convection-diffusion example, Sec. 5.2."""
    return 2.0 * x2 * (1.0 - x1 * x1), -2.0 * x1 * (1.0 - x2 * x2)


def _all_nodes(dim: int, N: int):
    """Integer index arrays (0..N+1) of all nodes, lexicographic, x1 fastest."""
    idx = np.indices((N + 2,) * dim)  # idx[a] is the index along axis a
    # flatten so that axis 0 (x1) varies fastest
    return [idx[a].transpose(*range(dim)[::-1]).reshape(-1) for a in range(dim)]


def _full_operator(dim: int, N: int, pde: str, eps: float) -> sp.csr_matrix:
    """Rows for interior nodes, columns for all (N+2)^d nodes."""
    h = 1.0 / (N + 1)
    P = N + 2
    ii = _all_nodes(dim, N)
    interior = np.ones(P ** dim, dtype=bool)
    for a in range(dim):
        interior &= (ii[a] >= 1) & (ii[a] <= N)
    rows_full = np.nonzero(interior)[0]          # full index of each interior node
    n = rows_full.size
    row_of = np.arange(n)
    stride = [P ** a for a in range(dim)]

    diff = 1.0 if pde == "poisson" else float(eps)
    R, C, V = [], [], []
    # diffusion part: diff * h^-2 (2d y_i - sum nbrs)
    R.append(row_of); C.append(rows_full); V.append(np.full(n, diff * 2 * dim / h ** 2))
    for a in range(dim):
        for s in (-1, 1):
            R.append(row_of); C.append(rows_full + s * stride[a]); V.append(np.full(n, -diff / h ** 2))
    if pde == "convdiff":
        if dim != 2:
            raise ValueError("convection-diffusion is defined in 2D")
        x1 = ii[0][rows_full] * h
        x2 = ii[1][rows_full] * h
        wind = _wind(x1, x2)
        for a in range(dim):
            wp = np.maximum(wind[a], 0.0) / h
            wm = np.minimum(wind[a], 0.0) / h
            # max(w,0)(y_i - y_{i-e}) + min(w,0)(y_{i+e} - y_i)
            R.append(row_of); C.append(rows_full); V.append(wp - wm)
            R.append(row_of); C.append(rows_full - stride[a]); V.append(-wp)
            R.append(row_of); C.append(rows_full + stride[a]); V.append(wm)
    elif pde != "poisson":
        raise ValueError(f"unknown pde {pde!r}")
    R = np.concatenate(R); C = np.concatenate(C); V = np.concatenate(V)
    full = sp.csr_matrix((V, (R, C)), shape=(n, P ** dim))
    full.sum_duplicates()
    return full, rows_full


@dataclass
class Discretization:
    dim: int
    N: int
    A: sp.csr_matrix       # interior operator A_II (n x n)
    f_hat: np.ndarray      # f - A_IB g_B
    # finite elements (fem.py): tracking mass, control mass (regularization
    # and the coupling L y - M u), L1 quadrature weights; None: unit mass
    Mt: object = None
    Mc: object = None
    dl: object = None

    @property
    def n(self):
        return self.A.shape[0]


def operator_matrix(dim: int, N: int, pde: str = "poisson", eps: float = 1.0) -> sp.csr_matrix:
    """A_II, the interior block of the discrete state operator (Sec. 2, matrix L)."""
    full, rows_full = _full_operator(dim, N, pde, eps)
    return full[:, rows_full].tocsr()


def rhs_offset(dim: int, N: int, pde: str, eps: float, g) -> np.ndarray:
    """-A_IB g_B: the boundary data moved to the right-hand side."""
    full, rows_full = _full_operator(dim, N, pde, eps)
    if g is None:
        return np.zeros(rows_full.size)
    gg = np.array(g, dtype=np.float64, copy=True)
    gg[rows_full] = 0.0  # interior entries of g are ignored
    return -(full @ gg)


def heat_operator(N: int, nt: int, tau: float) -> sp.csr_matrix:
    """All-at-once backward Euler matrix of Sec. 4.4 with M = I, divided by tau."""
    Ah = operator_matrix(2, N, "poisson")
    Id = sp.identity(N * N, format="csr")
    diag_blocks = sp.kron(sp.identity(nt), Id / tau + Ah)
    sub_blocks = sp.kron(sp.eye(nt, k=-1), Id / tau)
    return (diag_blocks - sub_blocks).tocsr()


def discretize_heat(prob) -> Discretization:
    """Heat equation (Sec. 4.4): the operator above and f_hat with the
    boundary data folded into every step and y0 / tau into the first."""
    N, nt, tau = prob.N, prob.nt, prob.tau
    if prob.dim != 2 or nt < 1 or not tau > 0:
        raise ValueError("the heat equation takes dim 2, nt >= 1 and tau > 0")
    A = heat_operator(N, nt, tau)
    n2 = N * N
    f_hat = np.zeros(n2 * nt) if prob.f is None else np.array(prob.f, dtype=np.float64, copy=True)
    step = rhs_offset(2, N, "poisson", 1.0, prob.g)
    f_hat += np.tile(step, nt)
    if prob.y0 is not None:
        f_hat[:n2] += np.asarray(prob.y0, dtype=np.float64) / tau
    return Discretization(2, N, A, f_hat)


def discretize(prob) -> Discretization:
    """Operator and folded right-hand side for a workloads.ProblemData."""
    if prob.pde == "heat":
        return discretize_heat(prob)
    if prob.pde == "poisson_q1":
        from .fem import discretize_q1
        return discretize_q1(prob)
    full, rows_full = _full_operator(prob.dim, prob.N, prob.pde, prob.eps)
    A = full[:, rows_full].tocsr()
    f = np.zeros(rows_full.size) if prob.f is None else np.asarray(prob.f, dtype=np.float64)
    f_hat = f.copy()
    if prob.g is not None:
        gg = np.array(prob.g, dtype=np.float64, copy=True)
        gg[rows_full] = 0.0
        f_hat -= full @ gg
    return Discretization(prob.dim, prob.N, A, f_hat)
