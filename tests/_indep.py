"""Independent helpers for pinning the oracle: a dense finite-difference
operator built node by node with plain loops, a proximal-gradient (FISTA)
solver for the control-only reduced problem and an exhaustive active-set
solver for tiny problems.  None of this code is shared with oracle/ or with
the GPU library."""
from __future__ import annotations

import itertools
import math

import numpy as np


def wind(x1, x2):
    # wind field of the convection-diffusion example (Sec. 5.2)
    return 2.0 * x2 * (1.0 - x1 ** 2), -2.0 * x1 * (1.0 - x2 ** 2)


def dense_operator(dim, N, pde="poisson", eps=1.0):
    """Interior FD operator as a dense matrix, one node at a time."""
    h = 1.0 / (N + 1)
    n = N ** dim
    A = np.zeros((n, n))

    def idx(c):
        k = 0
        for a in reversed(range(dim)):
            k = k * N + (c[a] - 1)
        return k

    for c in itertools.product(range(1, N + 1), repeat=dim):
        c = tuple(reversed(c))  # iterate with x1 fastest (not required, but tidy)
        i = idx(c)
        d = 1.0 if pde == "poisson" else eps
        A[i, i] += 2 * dim * d / h ** 2
        for a in range(dim):
            for s in (-1, 1):
                nb = list(c); nb[a] += s
                if 1 <= nb[a] <= N:
                    A[i, idx(nb)] -= d / h ** 2
        if pde == "convdiff":
            x = [c[a] * h for a in range(dim)]
            wv = wind(x[0], x[1])
            for a in range(dim):
                # upwind: flow in +e_a uses the backward difference, in -e_a the forward one
                if wv[a] > 0:
                    A[i, i] += wv[a] / h
                    nb = list(c); nb[a] -= 1
                    if nb[a] >= 1:
                        A[i, idx(nb)] -= wv[a] / h
                elif wv[a] < 0:
                    A[i, i] += -wv[a] / h
                    nb = list(c); nb[a] += 1
                    if nb[a] <= N:
                        A[i, idx(nb)] -= -wv[a] / h
    return A


def sine_mode(dim, N, ks):
    h = 1.0 / (N + 1)
    t = np.arange(1, N + 1) * h
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    out = np.ones_like(grids[0])
    for a in range(dim):
        out = out * np.sin(ks[a] * math.pi * grids[a])
    return out.reshape(-1, order="F")


def sine_eigenvalue(dim, N, ks):
    h = 1.0 / (N + 1)
    return sum(4.0 / h ** 2 * math.sin(k * math.pi * h / 2) ** 2 for k in ks)


def fista(A, yd, fhat, alpha, beta, ua, ub, iters=20000, tol=1e-15, obs=None):
    """min_u 1/2 (y - yd)^T O (y - yd) + alpha/2|u|^2 + beta|u|_1 with
    y = A^-1 (u + fhat), ua <= u <= ub, O = diag(obs) (identity if None)."""
    Ainv = np.linalg.inv(A)
    O = np.eye(A.shape[0]) if obs is None else np.diag(obs)
    G = Ainv.T @ O @ Ainv
    L = np.linalg.eigvalsh(G).max() + alpha
    c = Ainv.T @ O @ (Ainv @ fhat - yd)
    u = np.zeros(A.shape[0]); z = u.copy(); t = 1.0
    for _ in range(iters):
        grad = G @ z + c + alpha * z
        q = z - grad / L
        un = np.clip(np.sign(q) * np.maximum(np.abs(q) - beta / L, 0.0), ua, ub)
        tn = 0.5 * (1 + math.sqrt(1 + 4 * t * t))
        z = un + ((t - 1) / tn) * (un - u)
        if np.abs(un - u).max() < tol:
            u = un
            break
        u, t = un, tn
    return u, Ainv @ (u + fhat)


def active_set_qp(A, yd, fhat, alpha, beta, ua, ub, ya=None, yb=None):
    """Exhaustive active-set solution of the tiny QP in (y, u).

    Each node's control is at u_a, free negative, zero, free positive or at
    u_b; each state (with bounds) is at y_a, free or at y_b.  For each
    pattern the equality-constrained QP is solved and the unique pattern
    whose solution is primal and dual feasible is returned."""
    n = A.shape[0]
    u_states = range(5)
    y_states = range(3) if ya is not None else [1]
    best = None
    for up in itertools.product(u_states, repeat=n):
        for yp in itertools.product(y_states, repeat=n):
            # unknowns [y (n), u (n), p (n)]; KKT of the pattern
            K = np.zeros((3 * n, 3 * n)); r = np.zeros(3 * n)
            # state equation: A y - u = fhat
            K[2 * n:, :n] = A; K[2 * n:, n:2 * n] = -np.eye(n); r[2 * n:] = fhat
            for i in range(n):
                # y row: y - yd + A^T p (+ multiplier) = 0, or y fixed
                if yp[i] == 1:
                    K[i, i] = 1.0; K[i, 2 * n:] = A[:, i]; r[i] = yd[i]
                else:
                    K[i, i] = 1.0; r[i] = ya[i] if yp[i] == 0 else yb[i]
                j = n + i
                if up[i] == 0:
                    K[j, j] = 1.0; r[j] = ua[i]
                elif up[i] == 4:
                    K[j, j] = 1.0; r[j] = ub[i]
                elif up[i] == 2:
                    K[j, j] = 1.0; r[j] = 0.0
                else:  # free: alpha u + beta sign - p = 0
                    K[j, j] = alpha; K[j, 2 * n + i] = -1.0
                    r[j] = -beta if up[i] == 3 else beta
            try:
                sol = np.linalg.solve(K, r)
            except np.linalg.LinAlgError:
                continue
            y, u, p = sol[:n], sol[n:2 * n], sol[2 * n:]
            ok = True
            tol = 1e-10
            for i in range(n):
                s = alpha * u[i] - p[i]  # must equal -beta*d|u| - normal cone
                if up[i] == 0:      # at u_a < 0: multiplier s - beta >= 0
                    ok &= s - beta >= -tol
                elif up[i] == 4:    # at u_b > 0: multiplier -(s + beta) >= 0
                    ok &= s + beta <= tol
                elif up[i] == 2:
                    ok &= abs(s) <= beta + tol
                elif up[i] == 1:
                    ok &= u[i] < tol and u[i] > ua[i] - tol
                else:
                    ok &= u[i] > -tol and u[i] < ub[i] + tol
                if ya is not None:
                    g = y[i] - yd[i] + A[:, i] @ p  # = lambda_a - lambda_b
                    if yp[i] == 1:
                        ok &= ya[i] - tol <= y[i] <= yb[i] + tol
                    elif yp[i] == 0:
                        ok &= g >= -tol
                    else:
                        ok &= g <= tol
                if not ok:
                    break
            ok &= np.all(u >= ua - tol) and np.all(u <= ub + tol)
            if ok:
                if best is not None and np.abs(best[1] - u).max() > 1e-8:
                    raise AssertionError("two KKT points found for a strongly convex QP")
                best = (y, u)
    return best


def dense_heat_operator(N, nt, tau):
    """Backward Euler space-time operator (Sec. 4.4, M = I, divided by tau) as
    a dense matrix, one row at a time: row (t, i) carries
    (y[t, i] - y[t-1, i]) / tau + (Poisson stencil of y[t])_i."""
    n2 = N * N
    Ah = dense_operator(2, N, "poisson")
    A = np.zeros((n2 * nt, n2 * nt))
    for t in range(nt):
        for i in range(n2):
            r = t * n2 + i
            A[r, t * n2:(t + 1) * n2] += Ah[i]
            A[r, r] += 1.0 / tau
            if t > 0:
                A[r, r - n2] -= 1.0 / tau
    return A


def dense_q1(N):
    """Q1 stiffness and consistent mass on the interior nodes from their
    nine-point stencils (interior node: 8/3 and -1/3 for the stiffness,
    h^2/36 times 16, 4 (edge neighbours), 1 (corner neighbours) for the mass),
    one row at a time; neighbours on the boundary are dropped."""
    h = 1.0 / (N + 1)
    n = N * N
    K = np.zeros((n, n)); M = np.zeros((n, n))
    for i2 in range(N):
        for i1 in range(N):
            r = i1 + N * i2
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    j1, j2 = i1 + a, i2 + b
                    if not (0 <= j1 < N and 0 <= j2 < N):
                        continue
                    c = j1 + N * j2
                    if a == 0 and b == 0:
                        K[r, c] += 8.0 / 3.0; M[r, c] += 16.0 * h * h / 36.0
                    elif a == 0 or b == 0:
                        K[r, c] -= 1.0 / 3.0; M[r, c] += 4.0 * h * h / 36.0
                    else:
                        K[r, c] -= 1.0 / 3.0; M[r, c] += 1.0 * h * h / 36.0
    return K, M


def dense_q1_3d(N):
    """Trilinear Q1 stiffness and consistent mass on the interior nodes of the
    unit cube from their 27-point stencils, one row at a time (neighbours on
    the boundary dropped).  By the number of nonzero offsets of a neighbour
    (0: the node, 1: a face, 2: an edge, 3: a corner neighbour): stiffness
    h (8/3, 0, -1/6, -1/12), mass h^3/216 (64, 16, 4, 1)."""
    h = 1.0 / (N + 1)
    n = N ** 3
    kw = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}
    mw = {0: 64.0, 1: 16.0, 2: 4.0, 3: 1.0}
    K = np.zeros((n, n)); M = np.zeros((n, n))
    for i3 in range(N):
        for i2 in range(N):
            for i1 in range(N):
                r = i1 + N * (i2 + N * i3)
                for o in itertools.product((-1, 0, 1), repeat=3):
                    j1, j2, j3 = i1 + o[0], i2 + o[1], i3 + o[2]
                    if not (0 <= j1 < N and 0 <= j2 < N and 0 <= j3 < N):
                        continue
                    c = j1 + N * (j2 + N * j3)
                    k = sum(1 for t in o if t != 0)
                    K[r, c] += kw[k] * h
                    M[r, c] += mw[k] * h ** 3 / 216.0
    return K, M


def dense_q1_observed(N, elem_w):
    """2D Q1 mass of the observed elements only: node by node, the sum over
    the (up to) four elements around it of the element's weight times its
    mass stencil, h^2/36 times 4 (the node), 2 (an edge neighbour in that
    element) and 1 (the opposite corner); elements are numbered by their
    lower corner (e1, e2) in 0..N of the (N+2)^2 grid, e1 fastest."""
    h = 1.0 / (N + 1)
    n = N * N
    ew = np.asarray(elem_w).reshape(N + 1, N + 1)  # [e2, e1]
    M = np.zeros((n, n))
    for i2 in range(N):
        for i1 in range(N):
            r = i1 + N * i2
            g1, g2 = i1 + 1, i2 + 1  # position on the (N+2)^2 grid
            for e2 in (g2 - 1, g2):
                for e1 in (g1 - 1, g1):
                    c = ew[e2, e1]
                    if c == 0:
                        continue
                    for n2 in (e2, e2 + 1):
                        for n1 in (e1, e1 + 1):
                            j1, j2 = n1 - 1, n2 - 1
                            if not (0 <= j1 < N and 0 <= j2 < N):
                                continue
                            d = (n1 != g1) + (n2 != g2)
                            M[r, j1 + N * j2] += c * h * h * (4.0, 2.0, 1.0)[d] / 36.0
    return M


def fista_weighted(K, M, dl, yd, fhat, alpha, beta, ua, ub, iters=200000, tol=1e-15, Mt=None):
    """min_u 1/2 (y - yd)^T Mt (y - yd) + alpha/2 u^T M u + beta sum_i dl_i |u_i|
    with K y = M u + fhat and ua <= u <= ub (the finite-element problem;
    Mt = M unless a tracking mass is given), by FISTA on u with a per-node
    weighted soft threshold."""
    Mt = M if Mt is None else Mt
    Kinv = np.linalg.inv(K)
    G = Kinv @ M                       # y = G u + Kinv fhat
    H = G.T @ Mt @ G + alpha * M       # Hessian in u
    c = G.T @ Mt @ (Kinv @ fhat - yd)
    L = np.linalg.eigvalsh(H).max()
    u = np.zeros(K.shape[0]); z = u.copy(); t = 1.0
    for _ in range(iters):
        q = z - (H @ z + c) / L
        un = np.clip(np.sign(q) * np.maximum(np.abs(q) - beta * dl / L, 0.0), ua, ub)
        tn = 0.5 * (1 + math.sqrt(1 + 4 * t * t))
        z = un + ((t - 1) / tn) * (un - u)
        if np.abs(un - u).max() < tol:
            u = un
            break
        u, t = un, tn
    return u, G @ u + Kinv @ fhat
