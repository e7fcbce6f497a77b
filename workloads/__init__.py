"""Seeded synthetic problem instances for the sparse box-constrained optimal
control problems (Sec. 1, eqs. (pb), (eq:lap), (box), (boxs)).

This module only *generates data*: grids, desired states, bounds and
parameters.  It contains none of the solution method's arithmetic (no
operators, no interior point steps), so that both the CPU oracle and the GPU
path may draw identical inputs from it without sharing any solver code.

Layout convention used by every consumer: a field on the N^d interior nodes
of (0,1)^d is a flat float64 array in lexicographic order with x1 fastest,
node (i1, ..., id) (1-based) at x = (i1 h, ..., id h), h = 1/(N+1).
Boundary data g lives on the (N+2)^d nodes including the boundary, same
ordering with 0-based indices 0..N+1.

Workload recipes (the paper prints no data files; these stand in for its
analytic desired states, Sec. 5):
  * ``poisson2d_small``: N=31, y_d = A sin(pi x1) sin(pi x2), A ~ N(1, 0.1),
    alpha=1e-2, beta=1e-3, u in [-2, 2], no state bounds.
  * ``poisson2d_511``: N=511, y_d = 8 random sine modes, alpha=1e-4,
    beta=1e-3, u in [-5, 5], y in [-0.2, 0.3].
  * ``poisson3d_127``: N=127 in 3D, 8 sine modes, alpha=1e-5,
    beta from {1e-4, 1e-3, 1e-2, 1e-1}, u in [-10, 10].
  * ``convdiff2d_255``: eps=1/200, wind of Sec. 5.2, N=255, 8 sine modes,
    alpha=beta=1e-3, u in [-3, 3].
  * ``served_mix``: a stream of mixed requests (see ``served_requests``).
  * ``poisson2d_q1``: the 511^2 Poisson data with Q1 finite elements
    (pde "poisson_q1": stiffness, consistent and lumped mass).
  * ``poisson3d_q1``: the 127^3 Poisson data of ``poisson3d_127`` with
    trilinear Q1 finite elements.
  * ``poisson3d_q1_partial``: the 3D partial-observation setting of Sec. 5.1
    with trilinear Q1 elements: N=31 (h = 2^-5), observed subdomain
    (0.2,0.4) x (0.4,0.9) x (0,1), alpha=1e-5, beta=1e-3, u in [-2, 1.5],
    no state bounds, sigma=0.25, 8 sine modes for y_d (the paper's desired
    state is not given in closed form).  ``poisson2d_q1_partial``: the 2D
    analogue on the central square (0.25,0.75)^2, N=255.

For Q1 problems ``obs`` holds one weight per element ((N+1)^d values; the
element with lower corner (e1, ...) of the (N+2)^d grid, x1 fastest): 1 if
its centre lies in the observed subdomain, else 0.
  * ``heat2d``: the heat equation on (0,1)^2 x (0,1] (Sec. 5.3), N=63,
    nt=100 backward Euler steps (tau=0.01), y_d = A sin(pi x1) sin(pi x2) at
    every time step, A ~ N(1, 0.1), y(0) = 0, alpha=1e-4, beta=1e-2,
    u in [-15, 15], no state bounds, sigma=0.25.

Heat-equation fields live on the space-time nodes (x_i, t_k), t_k = k tau,
k = 1..nt: nt consecutive blocks of N^2 values (block k-1 holds time t_k),
each in the layout above.  The initial state y0 has N^2 values; g is
time-independent.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CONFIG_IDS = {
    "poisson2d_small": 0,
    "poisson2d_511": 1,
    "poisson3d_127": 2,
    "convdiff2d_255": 3,
    "served_mix": 4,
    "poisson2d_partial": 5,
    "heat2d": 6,
    "poisson2d_q1": 7,
    "poisson3d_q1": 8,
    "poisson3d_q1_partial": 9,
    "poisson2d_q1_partial": 10,
}


@dataclass
class ProblemData:
    """Inputs of one instance, exactly what the C ABI's problem_create takes."""

    dim: int
    N: int
    pde: str  # "poisson" or "convdiff"
    eps: float
    alpha: float
    beta: float
    u_a: np.ndarray
    u_b: np.ndarray
    y_a: Optional[np.ndarray]
    y_b: Optional[np.ndarray]
    y_d: np.ndarray
    f: Optional[np.ndarray] = None
    g: Optional[np.ndarray] = None
    sigma: float = 0.2  # recommended barrier reduction factor for this class
    name: str = ""
    meta: dict = field(default_factory=dict)
    # observation weights (1 where the state is observed, 0 elsewhere); None:
    # the whole domain is observed
    obs: Optional[np.ndarray] = None
    # heat equation (pde "heat", dim 2): nt time steps of length tau, initial
    # state y0 (N^2 values; None: zero); every other field then has nt N^2 values
    nt: int = 1
    tau: float = 0.0
    y0: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.N ** self.dim * self.nt

    @property
    def h(self) -> float:
        return 1.0 / (self.N + 1)

    def copy(self) -> "ProblemData":
        def c(a):
            return None if a is None else np.array(a, dtype=np.float64, copy=True)

        return ProblemData(self.dim, self.N, self.pde, self.eps, self.alpha, self.beta,
                           c(self.u_a), c(self.u_b), c(self.y_a), c(self.y_b), c(self.y_d),
                           c(self.f), c(self.g), self.sigma, self.name, dict(self.meta), c(self.obs),
                           self.nt, self.tau, c(self.y0))


def rng_for(config: str, instance: int = 0, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng([CONFIG_IDS[config], int(instance), int(seed)])


def interior_coords(dim: int, N: int):
    """Coordinates of the interior nodes, each a flat array (x1 fastest)."""
    h = 1.0 / (N + 1)
    t = np.arange(1, N + 1, dtype=np.float64) * h
    grids = np.meshgrid(*([t] * dim), indexing="ij")  # grids[a] varies along axis a
    # lexicographic with x1 fastest: flatten in Fortran order over (i1, ..., id)
    return [g_.reshape(-1, order="F") for g_ in grids]


def all_coords(dim: int, N: int):
    """Coordinates of all (N+2)^d nodes including the boundary (x1 fastest)."""
    h = 1.0 / (N + 1)
    t = np.arange(0, N + 2, dtype=np.float64) * h
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    return [g_.reshape(-1, order="F") for g_ in grids]


def sine_modes(rng: np.random.Generator, dim: int, N: int, n_modes: int = 8, kmax: int = 4):
    """Sum of n_modes products of sines, amplitude U[-1,1], integer freq U{1..kmax} per axis.

    Returns (values on interior nodes, list of (amplitude, freq tuple))."""
    xs = interior_coords(dim, N)
    out = np.zeros(N ** dim)
    modes = []
    for _ in range(n_modes):
        a = rng.uniform(-1.0, 1.0)
        ks = tuple(int(k) for k in rng.integers(1, kmax + 1, size=dim))
        term = np.full(N ** dim, a)
        for ax in range(dim):
            term = term * np.sin(ks[ax] * math.pi * xs[ax])
        out += term
        modes.append((a, ks))
    return out, modes


def _const(n: int, val: float) -> np.ndarray:
    return np.full(n, float(val))


def poisson2d_small(seed: int = 0, N: int = 31, instance: int = 0) -> ProblemData:
    rng = rng_for("poisson2d_small", instance, seed)
    amp = rng.normal(1.0, 0.1)
    x1, x2 = interior_coords(2, N)
    y_d = amp * np.sin(math.pi * x1) * np.sin(math.pi * x2)
    n = N * N
    return ProblemData(2, N, "poisson", 1.0, 1e-2, 1e-3, _const(n, -2.0), _const(n, 2.0),
                       None, None, y_d, None, None, 0.2, "poisson2d_small",
                       {"amplitude": amp, "modes": [(amp, (1, 1))]})


def poisson2d_511(seed: int = 0, N: int = 511, instance: int = 0) -> ProblemData:
    rng = rng_for("poisson2d_511", instance, seed)
    y_d, modes = sine_modes(rng, 2, N)
    n = N * N
    return ProblemData(2, N, "poisson", 1.0, 1e-4, 1e-3, _const(n, -5.0), _const(n, 5.0),
                       _const(n, -0.2), _const(n, 0.3), y_d, None, None, 0.2, "poisson2d_511",
                       {"modes": modes})


def poisson3d_127(seed: int = 0, N: int = 127, beta: float = 1e-3, instance: int = 0) -> ProblemData:
    rng = rng_for("poisson3d_127", instance, seed)
    y_d, modes = sine_modes(rng, 3, N)
    n = N ** 3
    return ProblemData(3, N, "poisson", 1.0, 1e-5, beta, _const(n, -10.0), _const(n, 10.0),
                       None, None, y_d, None, None, 0.2, "poisson3d_127", {"modes": modes})


def convdiff2d_255(seed: int = 0, N: int = 255, eps: float = 1.0 / 200.0, instance: int = 0) -> ProblemData:
    rng = rng_for("convdiff2d_255", instance, seed)
    y_d, modes = sine_modes(rng, 2, N)
    n = N * N
    return ProblemData(2, N, "convdiff", eps, 1e-3, 1e-3, _const(n, -3.0), _const(n, 3.0),
                       None, None, y_d, None, None, 0.4, "convdiff2d_255", {"modes": modes})


def poisson2d_partial(seed: int = 0, N: int = 255, instance: int = 0) -> ProblemData:
    """Partial observation: the state is observed on the central square
    (0.25, 0.75)^2 only (weights 1 there, 0 elsewhere), 8 sine modes for y_d,
    alpha = 1e-4, beta = 1e-3, u in [-5, 5], no state bounds, sigma = 0.25."""
    rng = rng_for("poisson2d_partial", instance, seed)
    y_d, modes = sine_modes(rng, 2, N)
    x1, x2 = interior_coords(2, N)
    obs = ((x1 > 0.25) & (x1 < 0.75) & (x2 > 0.25) & (x2 < 0.75)).astype(np.float64)
    n = N * N
    return ProblemData(2, N, "poisson", 1.0, 1e-4, 1e-3, _const(n, -5.0), _const(n, 5.0), None, None,
                       y_d, None, None, 0.25, "poisson2d_partial", {"modes": modes}, obs)


def heat2d(seed: int = 0, N: int = 63, nt: int = 100, alpha: float = 1e-4, instance: int = 0) -> ProblemData:
    """Heat equation, time-independent desired state A sin(pi x1) sin(pi x2)
    (Sec. 5.3), T = 1 split into nt backward Euler steps, y(0) = 0,
    beta = 1e-2, u in [-15, 15], no state bounds, sigma = 0.25."""
    rng = rng_for("heat2d", instance, seed)
    amp = rng.normal(1.0, 0.1)
    x1, x2 = interior_coords(2, N)
    frame = amp * np.sin(math.pi * x1) * np.sin(math.pi * x2)
    n = N * N * nt
    return ProblemData(2, N, "heat", 1.0, alpha, 1e-2, _const(n, -15.0), _const(n, 15.0), None, None,
                       np.tile(frame, nt), None, None, 0.25, "heat2d", {"amplitude": amp},
                       None, nt, 1.0 / nt, None)


def poisson2d_q1(seed: int = 0, N: int = 511, instance: int = 0) -> ProblemData:
    """The 511^2 Poisson workload (8 sine modes, alpha = 1e-4, beta = 1e-3,
    u in [-5, 5], y in [-0.2, 0.3]) discretized with Q1 finite elements."""
    rng = rng_for("poisson2d_q1", instance, seed)
    y_d, modes = sine_modes(rng, 2, N)
    n = N * N
    return ProblemData(2, N, "poisson_q1", 1.0, 1e-4, 1e-3, _const(n, -5.0), _const(n, 5.0),
                       _const(n, -0.2), _const(n, 0.3), y_d, None, None, 0.2, "poisson2d_q1", {"modes": modes})


def poisson3d_q1(seed: int = 0, N: int = 127, beta: float = 1e-3, instance: int = 0) -> ProblemData:
    """The 127^3 Poisson workload (8 sine modes, alpha = 1e-5, beta = 1e-3,
    u in [-10, 10], no state bounds) discretized with trilinear Q1 elements."""
    rng = rng_for("poisson3d_q1", instance, seed)
    y_d, modes = sine_modes(rng, 3, N)
    n = N ** 3
    return ProblemData(3, N, "poisson_q1", 1.0, 1e-5, beta, _const(n, -10.0), _const(n, 10.0),
                       None, None, y_d, None, None, 0.2, "poisson3d_q1", {"modes": modes})


def element_centres(dim: int, N: int):
    """Centres of the (N+1)^d elements (lower corner e, x1 fastest), each a flat array."""
    h = 1.0 / (N + 1)
    t = (np.arange(N + 1, dtype=np.float64) + 0.5) * h
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    return [g_.reshape(-1, order="F") for g_ in grids]


def poisson3d_q1_partial(seed: int = 0, N: int = 31, instance: int = 0) -> ProblemData:
    rng = rng_for("poisson3d_q1_partial", instance, seed)
    y_d, modes = sine_modes(rng, 3, N)
    c1, c2, c3 = element_centres(3, N)
    obs = ((c1 > 0.2) & (c1 < 0.4) & (c2 > 0.4) & (c2 < 0.9)).astype(np.float64)
    n = N ** 3
    return ProblemData(3, N, "poisson_q1", 1.0, 1e-5, 1e-3, _const(n, -2.0), _const(n, 1.5), None, None,
                       y_d, None, None, 0.25, "poisson3d_q1_partial", {"modes": modes}, obs)


def poisson2d_q1_partial(seed: int = 0, N: int = 255, instance: int = 0) -> ProblemData:
    rng = rng_for("poisson2d_q1_partial", instance, seed)
    y_d, modes = sine_modes(rng, 2, N)
    c1, c2 = element_centres(2, N)
    obs = ((c1 > 0.25) & (c1 < 0.75) & (c2 > 0.25) & (c2 < 0.75)).astype(np.float64)
    n = N * N
    return ProblemData(2, N, "poisson_q1", 1.0, 1e-4, 1e-3, _const(n, -5.0), _const(n, 5.0), None, None,
                       y_d, None, None, 0.25, "poisson2d_q1_partial", {"modes": modes}, obs)


def served_requests(n_requests: int = 256, seed: int = 0, sizes=(31, 63, 127, 255), rate: float = 1.0):
    """Request stream for the serving workload: (arrival_time, ProblemData) pairs.

    Arrivals are a Poisson process of the given rate (requests per unit time);
    each request is 50% Poisson, 25% conv-diff eps=1/50, 25% conv-diff eps=1/200,
    N uniform over ``sizes``, alpha log-U[1e-6,1e-2], beta log-U[1e-5,1e-2],
    u_a = -U[1,10], u_b = U[1,10], no state bounds, 8 sine modes for y_d."""
    rng = rng_for("served_mix", 0, seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        kind = rng.uniform()
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        alpha = 10.0 ** rng.uniform(-6.0, -2.0)
        beta = 10.0 ** rng.uniform(-5.0, -2.0)
        ua = -rng.uniform(1.0, 10.0)
        ub = rng.uniform(1.0, 10.0)
        sub = np.random.default_rng([CONFIG_IDS["served_mix"], r + 1, seed])
        y_d, modes = sine_modes(sub, 2, N)
        n = N * N
        if kind < 0.5:
            pde, eps, sigma = "poisson", 1.0, 0.2
        elif kind < 0.75:
            pde, eps, sigma = "convdiff", 1.0 / 50.0, 0.4
        else:
            pde, eps, sigma = "convdiff", 1.0 / 200.0, 0.4
        out.append((t, ProblemData(2, N, pde, eps, alpha, beta, _const(n, ua), _const(n, ub), None, None,
                                   y_d, None, None, sigma, f"req{r}", {"modes": modes})))
    return out


def by_name(name: str, seed: int = 0, **kw) -> ProblemData:
    return {"poisson2d_small": poisson2d_small, "poisson2d_511": poisson2d_511,
            "poisson3d_127": poisson3d_127, "convdiff2d_255": convdiff2d_255,
            "poisson2d_partial": poisson2d_partial, "heat2d": heat2d, "poisson2d_q1": poisson2d_q1,
            "poisson3d_q1": poisson3d_q1, "poisson3d_q1_partial": poisson3d_q1_partial,
            "poisson2d_q1_partial": poisson2d_q1_partial}[name](seed=seed, **kw)
