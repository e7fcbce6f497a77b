"""Bilinear / trilinear (Q1) finite elements on the uniform grid (oracle).

The paper discretizes with Q1 elements (Sec. 5): state, control and adjoint
are continuous piecewise bilinear (2D) or trilinear (3D) on the N^d interior
nodes of (0,1)^d, h = 1/(N+1), with

* L: the stiffness matrix (Sec. 2), entries of the integrals of grad phi_i .
  grad phi_j,
* M: the consistent mass matrix (Sec. 2), entries of the integrals of
  phi_i phi_j,
* D: the lumped mass diag(integral of phi_i) = h^d I, the weights of the
  nodal quadrature of the L1 term (Sec. 2),

assembled here element by element from the element matrices of a square
(4 x 4) or cube (8 x 8) of side h.  Dirichlet data g enter through the
boundary columns of L and the source through M: f_hat = M_II f_I - L_IB g_B
(the boundary part of M f is dropped with f given at interior nodes only).

Partial observation (Sec. 4.3): the tracking term integrates over the
observed subdomain only, so its mass is assembled from the observed
elements; `obs` then holds one weight per element ((N+1)^d values, element
numbered by its lower corner, x1 fastest), 1 observed and 0 not.

The problem handed to the interior point method is eq. (pb_fe_lin) divided
by h^d, the lumped mass of a node (the finite-element counterpart of the
unit-mass form of fd.py): L / h^d, M / h^d (rows summing to 1 away from the
boundary), D / h^d = I and f_hat / h^d.  The minimizer is unchanged, and the
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


def _element_matrices_3d(h: float):
    """Stiffness and mass of one cube element.  A trilinear basis function is
    the product of one 1D hat function per axis, so each element integral is
    a product of 1D integrals over [0, h] (stiffness k1 = [[1, -1], [-1, 1]] / h,
    mass m1 = [[2, 1], [1, 2]] h / 6): the mass takes m1 on every axis, the
    stiffness sums, over the axes, k1 on that axis times m1 on the others.
    Local node a = a1 + 2 a2 + 4 a3 sits at the corner (a1, a2, a3) h."""
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * (h / 6.0)
    Ke = np.zeros((8, 8))
    Me = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            ca = [(a >> t) & 1 for t in range(3)]
            cb = [(b >> t) & 1 for t in range(3)]
            m = [m1[ca[t], cb[t]] for t in range(3)]
            k = [k1[ca[t], cb[t]] for t in range(3)]
            Me[a, b] = m[0] * m[1] * m[2]
            Ke[a, b] = k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]
    return Ke, Me


def _full_matrices_3d(N: int):
    """L and M over all (N+2)^3 nodes (lexicographic, x1 fastest)."""
    h = 1.0 / (N + 1)
    P = N + 2
    Ke, Me = _element_matrices_3d(h)
    e = np.arange(N + 1)
    e1, e2, e3 = np.meshgrid(e, e, e, indexing="ij")
    base = (e1 + P * e2 + P * P * e3).reshape(-1)      # lower corner of every element
    off = [(a & 1) + P * ((a >> 1) & 1) + P * P * ((a >> 2) & 1) for a in range(8)]
    rows, cols, kv, mv = [], [], [], []
    for a in range(8):
        for b in range(8):
            rows.append(base + off[a]); cols.append(base + off[b])
            kv.append(np.full(base.size, Ke[a, b])); mv.append(np.full(base.size, Me[a, b]))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    L = sp.csr_matrix((np.concatenate(kv), (rows, cols)), shape=(P ** 3, P ** 3))
    M = sp.csr_matrix((np.concatenate(mv), (rows, cols)), shape=(P ** 3, P ** 3))
    L.sum_duplicates(); M.sum_duplicates()
    return L, M


def _full_matrices(N: int, dim: int = 2):
    """L and M over all (N+2)^d nodes (lexicographic, x1 fastest)."""
    if dim == 3:
        return _full_matrices_3d(N)
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


def _weighted_mass(N: int, dim: int, elem_w) -> sp.csr_matrix:
    """Mass over all (N+2)^d nodes with element e's integrals multiplied by
    elem_w[e] (partial observation, Sec. 4.3: the mass of the observed
    subdomain is assembled from its elements only).  Elements are numbered
    by their lower corner (e1, e2[, e3]) in 0..N, x1 fastest."""
    h = 1.0 / (N + 1)
    P = N + 2
    _, Me = _element_matrices(h) if dim == 2 else _element_matrices_3d(h)
    e = np.arange(N + 1)
    if dim == 2:
        e2, e1 = np.meshgrid(e, e, indexing="ij")
        base = (e1 + P * e2).reshape(-1)
        # local nodes of _element_matrices: (0,0), (1,0), (1,1), (0,1)
        off = [0, 1, 1 + P, P]
    else:
        e3, e2, e1 = np.meshgrid(e, e, e, indexing="ij")
        base = (e1 + P * e2 + P * P * e3).reshape(-1)
        off = [(a & 1) + P * ((a >> 1) & 1) + P * P * ((a >> 2) & 1) for a in range(8)]
    ew = np.asarray(elem_w, dtype=np.float64).reshape(-1)
    if ew.size != base.size:
        raise ValueError("one weight per element, (N+1)^d values")
    k = len(off)
    rows = np.concatenate([base + off[a] for a in range(k) for b in range(k)])
    cols = np.concatenate([base + off[b] for a in range(k) for b in range(k)])
    vals = np.concatenate([Me[a, b] * ew for a in range(k) for b in range(k)])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(P ** dim, P ** dim))
    M.sum_duplicates()
    return M


def _interior_index(N: int, dim: int = 2) -> np.ndarray:
    P = N + 2
    r = np.arange(1, N + 1)
    if dim == 2:
        i1, i2 = np.meshgrid(r, r, indexing="xy")
        return (i1 + P * i2).reshape(-1)
    i3, i2, i1 = np.meshgrid(r, r, r, indexing="ij")
    return (i1 + P * i2 + P * P * i3).reshape(-1)


def q1_matrices(N: int, dim: int = 2):
    """(L_II, M_II, D): interior stiffness, consistent mass and lumped mass diagonal."""
    L, M = _full_matrices(N, dim)
    I = _interior_index(N, dim)
    h = 1.0 / (N + 1)
    return L[I][:, I].tocsr(), M[I][:, I].tocsr(), np.full(N ** dim, h ** dim)


def discretize_q1(prob) -> Discretization:
    """Q1 discretization of the Poisson problem (2D or 3D): A = L, the
    tracking and control masses M, the L1 weights D, f_hat = M f - L_IB g."""
    if prob.dim not in (2, 3):
        raise ValueError("the Q1 discretization is built in 2D and 3D")
    N, dim = prob.N, prob.dim
    Lf, Mf = _full_matrices(N, dim)
    I = _interior_index(N, dim)
    h = 1.0 / (N + 1)
    L, M = Lf[I][:, I].tocsr(), Mf[I][:, I].tocsr()
    n = N ** dim
    f_hat = np.zeros(n) if prob.f is None else M @ np.asarray(prob.f, dtype=np.float64)
    if prob.g is not None:
        gg = np.array(prob.g, dtype=np.float64, copy=True)
        gg[I] = 0.0
        f_hat = f_hat - (Lf @ gg)[I]
    s = 1.0 / h ** dim
    Mt = M
    if getattr(prob, "obs", None) is not None:  # observed elements only (Sec. 4.3)
        Mt = _weighted_mass(N, dim, prob.obs)[I][:, I].tocsr()
    return Discretization(dim, N, (L * s).tocsr(), f_hat * s, Mt=(Mt * s).tocsr(), Mc=(M * s).tocsr(),
                          dl=np.ones(n))
