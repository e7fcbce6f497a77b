"""Interior point path-following loop for the split QP (oracle).

Follows the paper's Sec. 3 and the Appendix (Algorithm A.1) in unit-mass
finite-difference form (M = D = I, L = A, see fd.py):

  minimize   1/2 |y - y_d|^2 + alpha/2 |w - v|^2 + beta 1^T (w + v)
  subject to A y - (w - v) = f_hat,  0 <= w <= u_b,  0 <= v <= -u_a,
             y_a <= y <= y_b (optional)

which is eq. (pb_fe_lin) with z = [w; v], z_a = [max(u_a,0); -min(u_b,0)],
z_b = [max(u_b,0); -min(u_a,0)] (Sec. 2, eq. (split)).  With u_a < 0 < u_b,
z_a = 0 and z_b = [u_b; -u_a].

Each Newton step solves the reduced system eq. (NewtonSystem) directly
(SuperLU), recovers the multiplier steps by eqs. (zupdate1)-(zupdate4), takes
separate primal and dual step lengths scaled by alpha_0 and updates.

Readings taken where the paper is silent, garbled or ambiguous:
  R1  norms in the stopping test (Algorithm A.1): infinity norms of xi_p, xi_d
      (eq. (prdu)) and of the complementarity products of eq. (gap) taken
      with mu = 0 (with mu^k subtracted the central path would satisfy the
      test trivially).  This reproduces NLI = 9 at sigma = 0.2 and a final
      mu of 0.2^9 = 5.1e-7, as Sec. 5.1 reports.
  R2  mu_0 = 1 (Fig. convh starts at mu = 1).
  R3  starting point: box midpoints (y = 0 without state bounds),
      w = z_b,w / 2, v = z_b,v / 2, p = 0 and lambda = mu_0 / gap for every
      finite bound.
  R4  step lengths: alpha_P = alpha_0 min(1, alpha_P^max), same for alpha_D;
      the primal residual then contracts by exactly (1 - alpha_P) per step
      (Fig. convh shows the ratio 0.005 = 1 - 0.995).
  R5  the barrier parameter in the Newton right-hand side is the reduced one,
      sigma mu^k (Algorithm A.1 reduces mu before the solve).
  R6  the last block row of eq. (7by7) and the last block of eq. (gap) carry
      lambda_{z,b}, not lambda_{z,a} (a typo in the printed system).
  R7  primal variables (y, z) move with alpha_P, dual ones (p, lambdas) with
      alpha_D, as Algorithm A.1 states.
  R8  "no state bounds" means the lambda_y blocks are absent and Theta_y = 0.
  R9  partial observation (Sec. 4.3): the tracking term is taken over the
      observed nodes only, 1/2 (y - y_d)^T O (y - y_d) with O = diag(obs)
      (the unit-mass form of the mass matrix of the observation region), so
      O replaces M = I in the (1,1) block and in the first row of eq.
      (prdu); O + Theta_y is singular where a node is unobserved and has no
      state bound, and only the full 4n system is solved directly.

Option beyond the paper (off by default): mu_rule = "central" takes the
barrier target from the current iterate, mu^{k+1} = sigma * (mean of the
complementarity products of eq. (gap) at mu = 0), the duality measure of the
path-following scheme Algorithm A.1 cites, instead of sigma mu^k.  On the
central path (all products equal mu^k) the two coincide; when the step
lengths collapse the fixed geometric decrease runs ahead of the iterate and
the method can stall or lose interiority, which the iterate-based target
avoids.  A breakdown (a bound gap or product that is no longer positive and
finite, or a singular Newton matrix) ends solve() with status "breakdown".
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fd import discretize, Discretization


@dataclass
class IPMOptions:
    sigma: float = 0.2
    alpha0: float = 0.995
    eps_p: float = 1e-6
    eps_d: float = 1e-6
    eps_c: float = 1e-6
    mu0: float = 1.0
    maxit: int = 200
    fixed_nli: int = 0          # > 0: take exactly this many Newton steps
    newton: str = "auto"        # "full" (4n system) | "schur" (eliminated, SPD in dp) | "auto"
    mu_rule: str = "paper"      # "paper": mu^{k+1} = sigma mu^k | "central": sigma * mean product
    mass_scaling: str = "unit"  # "unit": the problem divided by the lumped mass h^d of a node |
                                # "hd": the literal weighting, objective and constraint times h^d


@dataclass
class IPMState:
    y: np.ndarray
    w: np.ndarray
    v: np.ndarray
    p: np.ndarray
    lwa: np.ndarray
    lwb: np.ndarray
    lva: np.ndarray
    lvb: np.ndarray
    lya: Optional[np.ndarray] = None
    lyb: Optional[np.ndarray] = None
    mu: float = 1.0

    def copy(self):
        c = lambda a: None if a is None else a.copy()
        return IPMState(c(self.y), c(self.w), c(self.v), c(self.p), c(self.lwa), c(self.lwb),
                        c(self.lva), c(self.lvb), c(self.lya), c(self.lyb), self.mu)


@dataclass
class IPMResult:
    u: np.ndarray
    y: np.ndarray
    p: np.ndarray
    state: IPMState
    nli: int
    status: str
    history: List[dict] = field(default_factory=list)


class _Bounds:
    """Bounds of the split problem (Sec. 2, z_a and z_b below eq. (split))."""

    def __init__(self, prob):
        ua = np.asarray(prob.u_a, dtype=np.float64)
        ub = np.asarray(prob.u_b, dtype=np.float64)
        self.zaw = np.maximum(ua, 0.0)
        self.zav = -np.minimum(ub, 0.0)
        self.zbw = np.maximum(ub, 0.0)
        self.zbv = -np.minimum(ua, 0.0)
        self.has_y = prob.y_a is not None
        if self.has_y:
            self.ya = np.asarray(prob.y_a, dtype=np.float64)
            self.yb = np.asarray(prob.y_b, dtype=np.float64)


def _obs(prob) -> np.ndarray:
    """Observation weights O (R9): ones when the whole domain is observed."""
    o = getattr(prob, "obs", None)
    return np.ones(prob.n) if o is None else np.asarray(o, dtype=np.float64)


def initial_state(prob, opts: IPMOptions) -> IPMState:
    """Starting point (reading R3)."""
    bd = _Bounds(prob)
    n = prob.n
    mu = opts.mu0
    y = 0.5 * (bd.ya + bd.yb) if bd.has_y else np.zeros(n)
    w = 0.5 * (bd.zaw + bd.zbw)
    v = 0.5 * (bd.zav + bd.zbv)
    st = IPMState(y, w, v, np.zeros(n), mu / (w - bd.zaw), mu / (bd.zbw - w),
                  mu / (v - bd.zav), mu / (bd.zbv - v), mu=mu)
    if bd.has_y:
        st.lya = mu / (y - bd.ya)
        st.lyb = mu / (bd.yb - y)
    return st


def _fem(disc) -> bool:
    """Finite-element masses present (fem.py): M in the tracking term, the
    regularization and the coupling, D in the L1 term (eq. (pb_fe_lin))."""
    return disc.Mc is not None


def residuals(prob, disc: Discretization, st: IPMState):
    """xi_p, xi_d (eq. (prdu)) and the complementarity products (eq. (gap), mu = 0)."""
    bd = _Bounds(prob)
    A, a, b = disc.A, prob.alpha, prob.beta
    u = st.w - st.v
    if _fem(disc):
        Mc, Mu, Mp = disc.Mc, disc.Mc @ u, disc.Mc @ st.p
        xi_p = A @ st.y - Mu - disc.f_hat
        dy = disc.Mt @ (st.y - prob.y_d) + A.T @ st.p
        bd_ = b * disc.dl
        dw = a * Mu + bd_ - Mp - st.lwa + st.lwb
        dv = -a * Mu + bd_ + Mp - st.lva + st.lvb
    else:
        xi_p = A @ st.y - u - disc.f_hat
        dy = _obs(prob) * (st.y - prob.y_d) + A.T @ st.p
        dw = a * u + b - st.p - st.lwa + st.lwb
        dv = -a * u + b + st.p - st.lva + st.lvb
    if bd.has_y:
        dy = dy - st.lya + st.lyb
    prods = [(st.w - bd.zaw) * st.lwa, (bd.zbw - st.w) * st.lwb,
             (st.v - bd.zav) * st.lva, (bd.zbv - st.v) * st.lvb]
    if bd.has_y:
        prods += [(st.y - bd.ya) * st.lya, (bd.yb - st.y) * st.lyb]
    return xi_p, np.concatenate([dy, dw, dv]), np.concatenate(prods)


def measures(prob, disc, st):
    xp, xd, xc = residuals(prob, disc, st)
    return float(np.abs(xp).max()), float(np.abs(xd).max()), float(np.abs(xc).max())


def complementarity_mean(prob, disc, st) -> float:
    """Mean of the complementarity products (eq. (gap) with mu = 0) over every
    finite bound: the duality measure of the iterate."""
    return float(residuals(prob, disc, st)[2].mean())


def next_mu(prob, disc, st, opts: "IPMOptions") -> float:
    """Barrier target of the next Newton step (Algorithm A.1, or the
    iterate-based target of mu_rule = "central")."""
    if opts.mu_rule == "central":
        return opts.sigma * complementarity_mean(prob, disc, st)
    if opts.mu_rule != "paper":
        raise ValueError(opts.mu_rule)
    return opts.sigma * st.mu


def barrier_diagonals(prob, st: IPMState):
    """Theta_y, Theta_w, Theta_v (Sec. 3, below eq. (NewtonSystem))."""
    bd = _Bounds(prob)
    tw = st.lwa / (st.w - bd.zaw) + st.lwb / (bd.zbw - st.w)
    tv = st.lva / (st.v - bd.zav) + st.lvb / (bd.zbv - st.v)
    if bd.has_y:
        ty = st.lya / (st.y - bd.ya) + st.lyb / (bd.yb - st.y)
    else:
        ty = np.zeros_like(st.y)
    return ty, tw, tv


def newton_matrix(prob, disc: Discretization, st: IPMState) -> sp.csc_matrix:
    """The 4n x 4n reduced Newton matrix of eq. (NewtonSystem), unknowns [dy; dw; dv; dp]."""
    n = prob.n
    a = prob.alpha
    ty, tw, tv = barrier_diagonals(prob, st)
    I = sp.identity(n, format="csr")
    Z = None
    A = disc.A
    if _fem(disc):
        M, Mt = disc.Mc, disc.Mt
        return sp.bmat([
            [Mt + sp.diags(ty), Z, Z, A.T],
            [Z, a * M + sp.diags(tw), -a * M, -M],
            [Z, -a * M, a * M + sp.diags(tv), M],
            [A, -M, M, Z],
        ], format="csc")
    K = sp.bmat([
        [sp.diags(_obs(prob) + ty), Z, Z, A.T],
        [Z, sp.diags(a + tw), -a * I, -I],
        [Z, -a * I, sp.diags(a + tv), I],
        [A, -I, I, Z],
    ], format="csc")
    return K


def newton_rhs(prob, disc: Discretization, st: IPMState, mu: float) -> np.ndarray:
    """Right-hand side of eq. (NewtonSystem) with barrier parameter mu."""
    bd = _Bounds(prob)
    A, a, b = disc.A, prob.alpha, prob.beta
    u = st.w - st.v
    if _fem(disc):
        Mu, Mp, bd_ = disc.Mc @ u, disc.Mc @ st.p, b * disc.dl
        ry = disc.Mt @ (st.y - prob.y_d) + A.T @ st.p
        rw = a * Mu + bd_ - Mp
        rv = -a * Mu + bd_ + Mp
        rp = A @ st.y - Mu - disc.f_hat
    else:
        ry = _obs(prob) * (st.y - prob.y_d) + A.T @ st.p
        rw = a * u + b - st.p
        rv = -a * u + b + st.p
        rp = A @ st.y - u - disc.f_hat
    if bd.has_y:
        ry = ry - mu / (st.y - bd.ya) + mu / (bd.yb - st.y)
    rw = rw - mu / (st.w - bd.zaw) + mu / (bd.zbw - st.w)
    rv = rv - mu / (st.v - bd.zav) + mu / (bd.zbv - st.v)
    return -np.concatenate([ry, rw, rv, rp])


def _splu(M, ordering):
    return spla.splu(sp.csc_matrix(M), permc_spec=ordering)


def newton_solve(prob, disc: Discretization, st: IPMState, mu: float, mode: str = "auto"):
    """Direct solution of eq. (NewtonSystem); returns (dy, dw, dv, dp).

    "full": SuperLU on the whole 4n system.
    "schur": exact elimination of dy (diagonal block) and (dw, dv) (per-node
    2x2 blocks), leaving the SPD system (A (I+Theta_y)^-1 A^T + Sigma) dp = r
    with Sigma = (theta_w + theta_v) / (alpha (theta_w + theta_v) + theta_w theta_v),
    the diagonal form that eq. (Schur) takes for M = I."""
    n = prob.n
    ty, tw, tv = barrier_diagonals(prob, st)
    if mode == "auto":
        if prob.pde == "heat":
            mode = "full" if prob.n <= 30000 else "schur"
        else:
            mode = "full" if (prob.dim == 2 and prob.N <= 127) or (prob.dim == 3 and prob.N <= 31) else "schur"
        if _fem(disc) or not np.all(_obs(prob) + ty > 0):
            # non-diagonal masses, or a singular (1,1) block (R9): no per-node elimination
            mode = "full"
    rhs = newton_rhs(prob, disc, st, mu)
    if mode == "full":
        K = newton_matrix(prob, disc, st)
        x = _splu(K, "COLAMD").solve(rhs)
        return x[:n], x[n:2 * n], x[2 * n:3 * n], x[3 * n:]
    if mode != "schur":
        raise ValueError(mode)
    a = prob.alpha
    by, bw, bv, bp = rhs[:n], rhs[n:2 * n], rhs[2 * n:3 * n], rhs[3 * n:]
    A = disc.A
    dyinv = 1.0 / (_obs(prob) + ty)
    det = a * (tw + tv) + tw * tv
    sigma_d = (tw + tv) / det
    S = (A @ sp.diags(dyinv) @ A.T + sp.diags(sigma_d)).tocsc()
    r = A @ (dyinv * by) - (tv * bw - tw * bv) / det - bp
    dp = _splu(S, "MMD_AT_PLUS_A").solve(r)
    dy = dyinv * (by - A.T @ dp)
    cw = bw + dp
    cv = bv - dp
    dw = ((a + tv) * cw + a * cv) / det
    dv = (a * cw + (a + tw) * cv) / det
    return dy, dw, dv, dp


def multiplier_steps(prob, st: IPMState, dy, dw, dv, mu):
    """Eqs. (zupdate1)-(zupdate4): steps of the bound multipliers."""
    bd = _Bounds(prob)
    ga, gb = st.w - bd.zaw, bd.zbw - st.w
    dlwa = -(st.lwa / ga) * dw - st.lwa + mu / ga
    dlwb = (st.lwb / gb) * dw - st.lwb + mu / gb
    ga, gb = st.v - bd.zav, bd.zbv - st.v
    dlva = -(st.lva / ga) * dv - st.lva + mu / ga
    dlvb = (st.lvb / gb) * dv - st.lvb + mu / gb
    out = {"lwa": dlwa, "lwb": dlwb, "lva": dlva, "lvb": dlvb}
    if bd.has_y:
        ga, gb = st.y - bd.ya, bd.yb - st.y
        out["lya"] = -(st.lya / ga) * dy - st.lya + mu / ga
        out["lyb"] = (st.lyb / gb) * dy - st.lyb + mu / gb
    return out


def _max_step(x, dx, lo, hi):
    """Largest a >= 0 with lo <= x + a dx <= hi (lo/hi may be None)."""
    amax = np.inf
    if lo is not None:
        m = dx < 0
        if m.any():
            amax = min(amax, float(np.min((x[m] - lo[m]) / (-dx[m]))))
    if hi is not None:
        m = dx > 0
        if m.any():
            amax = min(amax, float(np.min((hi[m] - x[m]) / dx[m])))
    return amax


def step_lengths(prob, st: IPMState, dy, dw, dv, dl, alpha0):
    """Algorithm A.1: fraction-to-boundary step lengths (reading R4)."""
    bd = _Bounds(prob)
    aP = min(_max_step(st.w, dw, bd.zaw, bd.zbw), _max_step(st.v, dv, bd.zav, bd.zbv))
    if bd.has_y:
        aP = min(aP, _max_step(st.y, dy, bd.ya, bd.yb))
    aD = np.inf
    for k, d in dl.items():
        aD = min(aD, _max_step(getattr(st, k), d, np.zeros_like(d), None))
    return alpha0 * min(1.0, aP), alpha0 * min(1.0, aD)


def ipm_step(prob, disc, st: IPMState, opts: IPMOptions, mu_new: float, mode: str = "auto"):
    """One pass of the loop body of Algorithm A.1 at barrier parameter mu_new."""
    dy, dw, dv, dp = newton_solve(prob, disc, st, mu_new, mode)
    dl = multiplier_steps(prob, st, dy, dw, dv, mu_new)
    aP, aD = step_lengths(prob, st, dy, dw, dv, dl, opts.alpha0)
    nxt = st.copy()
    nxt.y = st.y + aP * dy
    nxt.w = st.w + aP * dw
    nxt.v = st.v + aP * dv
    nxt.p = st.p + aD * dp
    for k, d in dl.items():
        setattr(nxt, k, getattr(st, k) + aD * d)
    nxt.mu = mu_new
    return nxt, {"alpha_P": aP, "alpha_D": aD, "dy": dy, "dw": dw, "dv": dv, "dp": dp}


def hd_weighted(prob, disc: Discretization) -> Discretization:
    """The literal h^d weighting of eq. (pb_fe_lin): every mass, the L1 weights
    and the state equation carry the lumped mass w = h^d of a node (M = D = w I
    for finite differences, w times the scaled masses for Q1), where the unit
    form divides them out."""
    h = 1.0 / (prob.N + 1)
    w = h ** prob.dim
    n = disc.n
    Mt = disc.Mt if disc.Mt is not None else sp.diags(_obs(prob))
    Mc = disc.Mc if disc.Mc is not None else sp.identity(n, format="csr")
    dl = disc.dl if disc.dl is not None else np.ones(n)
    return Discretization(disc.dim, disc.N, (w * disc.A).tocsr(), w * disc.f_hat,
                          Mt=(w * Mt).tocsr(), Mc=(w * Mc).tocsr(), dl=w * np.asarray(dl))


def solve(prob, opts: Optional[IPMOptions] = None) -> IPMResult:
    """Algorithm A.1 (Appendix) on the problem described by a workloads.ProblemData."""
    opts = opts or IPMOptions()
    disc = discretize(prob)
    if opts.mass_scaling == "hd":
        if prob.pde == "heat":
            raise ValueError("the h^d weighting is defined for the stationary problems")
        disc = hd_weighted(prob, disc)
    elif opts.mass_scaling != "unit":
        raise ValueError(opts.mass_scaling)
    st = initial_state(prob, opts)
    hist = []
    status = "maxit"
    k = 0
    while True:
        xp, xd, xc = measures(prob, disc, st)
        rec = {"k": k, "mu": st.mu, "xi_p": xp, "xi_d": xd, "xi_c": xc}
        if opts.fixed_nli > 0:
            if k >= opts.fixed_nli:
                hist.append(rec)
                status = "fixed"
                break
        elif xp <= opts.eps_p and xd <= opts.eps_d and xc <= opts.eps_c:
            hist.append(rec)
            status = "converged"
            break
        if k >= opts.maxit:
            hist.append(rec)
            break
        prods = residuals(prob, disc, st)[2]
        if not (np.isfinite(xp) and np.isfinite(xd) and np.all(np.isfinite(prods)) and prods.min() > 0):
            hist.append(rec)
            status = "breakdown"
            break
        mu_new = next_mu(prob, disc, st, opts)
        try:
            st, info = ipm_step(prob, disc, st, opts, mu_new, opts.newton)
        except RuntimeError:  # singular Newton matrix
            hist.append(rec)
            status = "breakdown"
            break
        rec.update(alpha_P=info["alpha_P"], alpha_D=info["alpha_D"])
        hist.append(rec)
        k += 1
    return IPMResult(st.w - st.v, st.y, st.p, st, k, status, hist)
