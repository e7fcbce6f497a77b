"""Bilinear (Q1) finite elements on the uniform square grid (oracle).

The paper discretizes with Q1 elements (Sec. 5): state, control and adjoint
are continuous piecewise bilinear on the N x N interior nodes of (0,1)^2,
h = 1/(N+1), with

* L: the stiffness matrix (Sec. 2), entries of the integrals of grad phi_i .
  grad phi_j,
* M: the consistent mass matrix (Sec. 2), entries of the integrals of
  phi_i phi_j,
* D: the lumped mass diag(integral of phi_i) = h^2 I, the weights of the
  nodal quadrature of the L1 term (Sec. 2),

assembled here element by element from the 4 x 4 element matrices of a
square of side h.  Dirichlet data g enter through the boundary columns of L
and the source through M: f_hat = M_II f_I - L_IB g_B (the boundary part of
M f is dropped with f given at interior nodes only).

The problem handed to the interior point method is eq. (pb_fe_lin) divided
by h^2, the lumped mass of a node (the finite-element counterpart of the
unit-mass form of fd.py): L / h^2, M / h^2 (rows summing to 1 away from the
boundary), D / h^2 = I and f_hat / h^2.  The minimizer is unchanged, and the
barrier parameter and the stopping tolerances keep the meaning they have
for the finite-difference problems, independent of the mesh.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fd import Discretization


def _element_matrices(h: float):
    """Stiffness and mass of one square element, local nodes counter-clockwise
    from the lower left corner: (0,0), (1,0), (1,1), (0,1)."""
    Ke = np.array([[4, -1, -2, -1],
                   [-1, 4, -1, -2],
                   [-2, -1, 4, -1],
                   [-1, -2, -1, 4]], dtype=np.float64) / 6.0
    Me = np.array([[4, 2, 1, 2],
                   [2, 4, 2, 1],
                   [1, 2, 4, 2],
                   [2, 1, 2, 4]], dtype=np.float64) * (h * h / 36.0)
    return Ke, Me


def _full_matrices(N: int):
    """L and M over all (N+2)^2 nodes (lexicographic, x1 fastest)."""
    h = 1.0 / (N + 1)
    P = N + 2
    Ke, Me = _element_matrices(h)
    rows, cols, kv, mv = [], [], [], []
    for e2 in range(N + 1):
        for e1 in range(N + 1):
            nodes = [e1 + P * e2, (e1 + 1) + P * e2, (e1 + 1) + P * (e2 + 1), e1 + P * (e2 + 1)]
            for a in range(4):
                for b in range(4):
                    rows.append(nodes[a]); cols.append(nodes[b])
                    kv.append(Ke[a, b]); mv.append(Me[a, b])
    L = sp.csr_matrix((kv, (rows, cols)), shape=(P * P, P * P))
    M = sp.csr_matrix((mv, (rows, cols)), shape=(P * P, P * P))
    L.sum_duplicates(); M.sum_duplicates()
    return L, M


def _interior_index(N: int) -> np.ndarray:
    P = N + 2
    i1, i2 = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1), indexing="xy")
    return (i1 + P * i2).reshape(-1)


def q1_matrices(N: int):
    """(L_II, M_II, D): interior stiffness, consistent mass and lumped mass diagonal."""
    L, M = _full_matrices(N)
    I = _interior_index(N)
    h = 1.0 / (N + 1)
    return L[I][:, I].tocsr(), M[I][:, I].tocsr(), np.full(N * N, h * h)


def discretize_q1(prob) -> Discretization:
    """Q1 discretization of the 2D Poisson problem: A = L, the tracking and
    control masses M, the L1 weights D, f_hat = M f - L_IB g."""
    if prob.dim != 2:
        raise ValueError("the Q1 discretization is built in 2D")
    N = prob.N
    Lf, Mf = _full_matrices(N)
    I = _interior_index(N)
    h = 1.0 / (N + 1)
    L, M = Lf[I][:, I].tocsr(), Mf[I][:, I].tocsr()
    f_hat = np.zeros(N * N) if prob.f is None else M @ np.asarray(prob.f, dtype=np.float64)
    if prob.g is not None:
        gg = np.array(prob.g, dtype=np.float64, copy=True)
        gg[I] = 0.0
        f_hat = f_hat - (Lf @ gg)[I]
    s = 1.0 / (h * h)
    return Discretization(2, N, (L * s).tocsr(), f_hat * s, Mt=(M * s).tocsr(), Mc=(M * s).tocsr(),
                          dl=np.ones(N * N))
