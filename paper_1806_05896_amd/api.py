"""Python binding of libipmpde: argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields
from typing import Optional

import numpy as np

from . import _lib as L

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "libipmpde.hip")
_INC = os.path.join(os.path.dirname(_HERE), "include")

# -amdgpu-kernarg-preload-count: the first kernel arguments arrive in SGPRs
# (gfx950), which takes one memory round trip off every launch.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17", "-Wno-unused-value",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-mllvm", "-amdgpu-kernarg-preload-count=8"]


def library_path() -> str:
    return L.LIB_PATH


def build_library(verbose: bool = False) -> str:
    """Compile csrc/libipmpde.hip for gfx950 into the package directory."""
    tmp = L.LIB_PATH + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", _INC, "-o", tmp, _SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    os.replace(tmp, L.LIB_PATH)
    if verbose:
        print(" ".join(cmd))
    return L.LIB_PATH


@dataclass
class Options:
    """Solver options (defaults as in include/ipmpde.h)."""

    sigma: float = 0.2
    alpha0: float = 0.995
    eps_p: float = 1e-6
    eps_d: float = 1e-6
    eps_c: float = 1e-6
    mu0: float = 1.0
    ipm_maxit: int = 200
    fixed_nli: int = 0
    krylov: str = "minres"          # "minres" | "fgmres"
    precond: str = "pd"             # "pd" | "pt" | "ppi" (partial observation, FGMRES)
    restart: int = 30
    krylov_tol: float = 1e-10
    krylov_maxit: int = 500
    vcycles: int = 1
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.0
    mg_precision: str = "fp32"      # "fp32" | "fp64"
    chunk: int = 8
    use_graphs: bool = True
    mu_rule: str = "paper"          # "paper" (sigma mu^k) | "central" (sigma x mean complementarity)
    mass_scaling: str = "unit"      # "unit" (divided by the lumped mass h^d) | "hd" (literal weighting)
    mg_tile: str = "auto"           # "auto" | "small" | "large": tiles of the 2D Poisson level kernels
    lanes: int = 1                  # batches: sub-batches solved concurrently, one stream and host thread each

    _ENUMS = {
        "krylov": {"minres": L.MINRES, "fgmres": L.FGMRES},
        "precond": {"pd": L.PD, "pt": L.PT, "ppi": L.PPI},
        "mg_precision": {"fp64": L.FP64, "fp32": L.FP32},
        "mu_rule": {"paper": L.MU_PAPER, "central": L.MU_CENTRAL},
        "mass_scaling": {"unit": L.MASS_UNIT, "hd": L.MASS_HD},
        "mg_tile": {"auto": L.TILE_AUTO, "small": L.TILE_SMALL, "large": L.TILE_LARGE},
    }

    @classmethod
    def from_c(cls, o: L.COptions) -> "Options":
        kw = {}
        for f in fields(cls):
            v = getattr(o, f.name)
            if f.name in cls._ENUMS:
                v = {c: k for k, c in cls._ENUMS[f.name].items()}[v]
            elif f.name == "use_graphs":
                v = bool(v)
            kw[f.name] = v
        return cls(**kw)

    def to_c(self) -> L.COptions:
        o = L.COptions()
        for f in fields(self):
            v = getattr(self, f.name)
            if f.name == "krylov":
                v = {"minres": L.MINRES, "fgmres": L.FGMRES}[v]
            elif f.name == "precond":
                v = {"pd": L.PD, "pt": L.PT, "ppi": L.PPI}[v]
            elif f.name == "mg_precision":
                v = {"fp64": L.FP64, "fp32": L.FP32}[v]
            elif f.name == "use_graphs":
                v = int(bool(v))
            elif f.name == "mu_rule":
                v = {"paper": L.MU_PAPER, "central": L.MU_CENTRAL}[v]
            elif f.name == "mass_scaling":
                v = {"unit": L.MASS_UNIT, "hd": L.MASS_HD}[v]
            elif f.name == "mg_tile":
                v = {"auto": L.TILE_AUTO, "small": L.TILE_SMALL, "large": L.TILE_LARGE}[v]
            setattr(o, f.name, v)
        return o


@dataclass
class Stats:
    status: int
    nli: int
    krylov_its: int
    krylov_fail: int
    xi_p: float
    xi_d: float
    xi_c: float
    mu: float
    solve_ms: float
    hist_krylov: list
    hist_mu: list
    hist_xi_p: list
    hist_xi_d: list
    hist_xi_c: list
    hist_alpha_p: list
    hist_alpha_d: list
    hist_krylov_relres: list


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, n, name):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != (n,):
        raise ValueError(f"{name} must have {n} entries")
    return a


class Problem:
    """One problem instance resident on the GPU (ipmpde_problem)."""

    def __init__(self, data=None, *, dim=None, N=None, pde="poisson", eps=1.0, alpha=None, beta=None,
                 u_a=None, u_b=None, y_a=None, y_b=None, y_d=None, f=None, g=None, obs=None,
                 nt=1, tau=0.0, y0=None):
        if data is not None:
            dim, N, pde, eps = data.dim, data.N, data.pde, data.eps
            alpha, beta = data.alpha, data.beta
            u_a, u_b, y_a, y_b, y_d, f, g = data.u_a, data.u_b, data.y_a, data.y_b, data.y_d, data.f, data.g
            obs = getattr(data, "obs", None)
            nt, tau, y0 = getattr(data, "nt", 1), getattr(data, "tau", 0.0), getattr(data, "y0", None)
        self._lib = L.load()
        self.dim, self.N = int(dim), int(N)
        self.nt = int(nt) if pde == "heat" else 1
        self.n = self.N ** self.dim * self.nt
        n = self.n
        self._keep = [_f64(u_a, n, "u_a"), _f64(u_b, n, "u_b"), _f64(y_a, n, "y_a"), _f64(y_b, n, "y_b"),
                      _f64(y_d, n, "y_d"), _f64(f, n, "f"), _f64(g, (self.N + 2) ** self.dim, "g")]
        grid = L.Grid(self.dim, self.N)
        h = C.c_void_p()
        if pde == "heat":
            # the heat equation (Sec. 4.4): nt backward Euler steps of length tau
            self._keep.append(_f64(y0, self.N ** self.dim, "y0"))
            L.check(self._lib.ipmpde_heat_create(C.byref(grid), self.nt, float(tau), float(alpha), float(beta),
                                                 *[_ptr(a) for a in self._keep], C.byref(h)))
        else:
            kind = {"poisson": L.POISSON, "convdiff": L.CONVDIFF, "poisson_q1": L.POISSON_Q1}[pde]
            pdes = L.Pde(kind, float(eps))
            L.check(self._lib.ipmpde_problem_create(C.byref(grid), C.byref(pdes), float(alpha), float(beta),
                                                    *[_ptr(a) for a in self._keep], C.byref(h)))
        self._h = h
        self.pde = pde
        self.has_state_bounds = y_a is not None
        self._keep = None
        if obs is not None:
            self.set_observation(obs)

    def set_observation(self, weights):
        """Observation weights (Sec. 4.3); None: the whole domain.  One per
        node (finite differences) or one per element ((N+1)^dim, Q1)."""
        if weights is None:
            L.check(self._lib.ipmpde_set_observation(self._h, None, 0))
            return
        m = (self.N + 1) ** self.dim if self.pde == "poisson_q1" else self.n
        w = _f64(weights, m, "obs")
        L.check(self._lib.ipmpde_set_observation(self._h, _ptr(w), m))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ipmpde_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @staticmethod
    def _opts(opts):
        return C.byref((opts or Options()).to_c())

    def solve(self, opts: Optional[Options] = None, stream=None, raise_on_error=False) -> int:
        rc = self._lib.ipmpde_solve(self._h, self._opts(opts), _stream_handle(stream))
        if raise_on_error:
            L.check(rc)
        elif rc not in (L.OK, L.ENOTCONVERGED, L.EKRYLOV, L.EBREAKDOWN):
            L.check(rc)
        return rc

    def reset(self, opts: Optional[Options] = None, stream=None):
        L.check(self._lib.ipmpde_reset(self._h, self._opts(opts), _stream_handle(stream)))

    def ipm_step(self, mu_new: float, opts: Optional[Options] = None, stream=None):
        aP, aD, rel = C.c_double(), C.c_double(), C.c_double()
        its = C.c_int()
        rc = self._lib.ipmpde_ipm_step(self._h, self._opts(opts), float(mu_new), _stream_handle(stream),
                                       C.byref(aP), C.byref(aD), C.byref(its), C.byref(rel))
        L.check(rc, allow=(L.EKRYLOV,))
        return {"alpha_P": aP.value, "alpha_D": aD.value, "krylov_its": its.value, "relres": rel.value, "rc": rc}

    def newton_direction(self, mu_new: float, opts: Optional[Options] = None, stream=None):
        its, rel = C.c_int(), C.c_double()
        rc = self._lib.ipmpde_newton_direction(self._h, self._opts(opts), float(mu_new), _stream_handle(stream),
                                               C.byref(its), C.byref(rel))
        L.check(rc, allow=(L.EKRYLOV,))
        return {"krylov_its": its.value, "relres": rel.value, "rc": rc}

    def newton_setup(self, mu_new: float, opts: Optional[Options] = None, stream=None):
        L.check(self._lib.ipmpde_newton_setup(self._h, self._opts(opts), float(mu_new), _stream_handle(stream)))

    def measures(self, stream=None):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        L.check(self._lib.ipmpde_measures(self._h, _stream_handle(stream), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def measures_noalloc(self, stream=None):
        """measures() through the entry point that allocates no device memory."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        L.check(self._lib.ipmpde_measures_noalloc(self._h, _stream_handle(stream), C.byref(a), C.byref(b),
                                                  C.byref(c)))
        return a.value, b.value, c.value

    def query(self, field: str) -> np.ndarray:
        out = np.empty(self.n)
        L.check(self._lib.ipmpde_query(self._h, L.FIELDS[field], out.ctypes.data_as(C.c_void_p), self.n))
        return out

    def set_field(self, field: str, values):
        a = _f64(values, self.n, field)
        L.check(self._lib.ipmpde_set_field(self._h, L.FIELDS[field], a.ctypes.data_as(C.c_void_p), self.n))

    def query_rhs(self) -> np.ndarray:
        out = np.empty(4 * self.n)
        L.check(self._lib.ipmpde_query_rhs(self._h, out.ctypes.data_as(C.c_void_p), 4 * self.n))
        return out

    def stats(self) -> Stats:
        s = L.CStats()
        L.check(self._lib.ipmpde_get_stats(self._h, C.byref(s)))
        k = s.hist_len
        return Stats(s.status, s.nli, s.krylov_its, s.krylov_fail, s.xi_p, s.xi_d, s.xi_c, s.mu, s.solve_ms,
                     list(s.hist_krylov[:k]), list(s.hist_mu[:k]), list(s.hist_xi_p[:k]), list(s.hist_xi_d[:k]),
                     list(s.hist_xi_c[:k]), list(s.hist_alpha_p[:k]), list(s.hist_alpha_d[:k]),
                     list(s.hist_krylov_relres[:k]))

    # ---- low-level operators on device tensors (torch.float64 on cuda)
    @staticmethod
    def _dptr(t):
        import torch
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("expected a contiguous float64 CUDA tensor")
        return C.c_void_p(t.data_ptr())

    def apply_operator(self, x, transpose: bool = False, stream=None):
        import torch
        y = torch.empty_like(x)
        L.check(self._lib.ipmpde_apply_operator(self._h, int(transpose), self._dptr(x), self._dptr(y),
                                                _stream_handle(stream)))
        return y

    def apply_saddle(self, x, stream=None):
        import torch
        y = torch.empty_like(x)
        L.check(self._lib.ipmpde_apply_saddle(self._h, self._dptr(x), self._dptr(y), _stream_handle(stream)))
        return y

    def apply_precond(self, x, opts: Optional[Options] = None, stream=None):
        import torch
        y = torch.empty_like(x)
        L.check(self._lib.ipmpde_apply_precond(self._h, self._opts(opts), self._dptr(x), self._dptr(y),
                                               _stream_handle(stream)))
        return y

    def time_kernel(self, kernel: int, reps: int = 50, opts: Optional[Options] = None, stream=None):
        ms, nbytes = C.c_double(), C.c_double()
        L.check(self._lib.ipmpde_time_kernel(self._h, self._opts(opts), int(kernel), int(reps),
                                             _stream_handle(stream), C.byref(ms), C.byref(nbytes)))
        return ms.value, nbytes.value


class Batch:
    """Several problems advanced by the same kernel launches (ipmpde_batch)."""

    def __init__(self, problems):
        self._lib = L.load()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = C.c_void_p()
        L.check(self._lib.ipmpde_batch_create(arr, len(self.problems), C.byref(h)))
        self._h = h

    def solve(self, opts=None, stream=None):
        """opts: None, one Options, or a list with one Options per problem."""
        if opts is None:
            ptr, per = None, 0
        elif isinstance(opts, Options):
            self._opts_keep = opts.to_c()
            ptr, per = C.cast(C.byref(self._opts_keep), C.c_void_p), 0
        else:
            arr = (L.COptions * len(opts))(*[o.to_c() for o in opts])
            self._opts_keep = arr
            ptr, per = C.cast(arr, C.c_void_p), 1
        L.check(self._lib.ipmpde_batch_solve(self._h, ptr, per, _stream_handle(stream)))
        return [p.stats().status for p in self.problems]

    def autotune(self, opts: Optional[Options] = None, cache: Optional[str] = None, tune_precision: bool = False,
                 stream=None):
        """The library's autotuner (ipmpde_batch_autotune): returns (Options with
        the fastest multigrid schedule, its batched solve time in ms, whether
        it came from the cache file)."""
        best = L.COptions()
        ms, hit = C.c_double(), C.c_int()
        path = None if cache is None else os.fsencode(cache)
        L.check(self._lib.ipmpde_batch_autotune(self._h, Problem._opts(opts), L.TUNE_PRECISION if tune_precision else 0,
                                                path, _stream_handle(stream), C.byref(best), C.byref(ms),
                                                C.byref(hit)))
        return Options.from_c(best), ms.value, bool(hit.value)

    def time_kernel(self, kernel: int, reps: int = 50, opts: Optional[Options] = None, stream=None):
        """(avg_ms, bytes) of one launch serving every instance (after a batch solve)."""
        ms, b = C.c_double(), C.c_double()
        L.check(self._lib.ipmpde_batch_time_kernel(self._h, Problem._opts(opts), kernel, reps, _stream_handle(stream),
                                                   C.byref(ms), C.byref(b)))
        return ms.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ipmpde_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Engine:
    """Serving engine (ipmpde_engine): continuous batching of solves with
    admission by HBM footprint.  The Python side only marshals arguments;
    queueing, admission, stepping and retirement run in the library."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.ipmpde_engine_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self._h = h
        self._problems = {}  # ticket -> Problem (kept alive while queued or running)

    def submit(self, problem: "Problem", opts: Optional[Options] = None) -> int:
        t = C.c_uint64()
        o = Problem._opts(opts)
        L.check(self._lib.ipmpde_engine_submit(self._h, problem._h, o, C.byref(t)))
        self._problems[t.value] = problem
        return t.value

    def step(self, stream=None):
        """One IPM iteration of every admitted request; returns (running, queued)."""
        r, q = C.c_int(), C.c_int()
        L.check(self._lib.ipmpde_engine_step(self._h, _stream_handle(stream), C.byref(r), C.byref(q)))
        return r.value, q.value

    def poll(self, ticket: int) -> dict:
        info = L.RequestInfo()
        L.check(self._lib.ipmpde_engine_poll(self._h, C.c_uint64(ticket), C.byref(info)))
        return {k: getattr(info, k) for k, _ in info._fields_}

    def release(self, ticket: int):
        L.check(self._lib.ipmpde_engine_release(self._h, C.c_uint64(ticket)))
        self._problems.pop(ticket, None)

    def info(self) -> dict:
        info = L.EngineInfo()
        L.check(self._lib.ipmpde_engine_get_info(self._h, C.byref(info)))
        return {k: getattr(info, k) for k, _ in info._fields_}

    def run(self, stream=None, max_steps: int = 100000):
        """Step until nothing is queued or running."""
        for _ in range(max_steps):
            r, q = self.step(stream)
            if r == 0 and q == 0:
                return
        raise RuntimeError("engine did not drain")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ipmpde_engine_destroy(self._h)
            self._h = None
            self._problems.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# The registered allocator callbacks; kept referenced while registered (the
# library calls them whenever it allocates or frees device memory).
_allocator_keep = None


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device allocations through PyTorch's caching
    allocator (ipmpde_set_allocator), or back to hipMalloc/hipFree.

    Affects problems, batches and engines created (and workspaces allocated)
    afterwards; memory already held keeps the allocator it came from.  Blocks
    come from the allocator's pool for the current device and stream at the
    time of the call.  The library synchronizes the device before it frees a
    problem's or a batch's memory and frees a served request's workspace only
    after the engine step that retired it has synchronized its stream, so a
    freed block is idle when the caching allocator hands it out again."""
    global _allocator_keep
    lib = L.load()
    if not enable:
        L.check(lib.ipmpde_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None))
        _allocator_keep = None
        return
    import torch

    def _alloc(nbytes, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:  # out of memory: the library reports ENOMEM
            return None

    def _free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))

    keep = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
    L.check(lib.ipmpde_set_allocator(keep[0], keep[1], None))
    _allocator_keep = keep


def footprint_bytes(dim: int, N: int, pde: str = "poisson", has_state_bounds: bool = False,
                    opts: Optional[Options] = None) -> int:
    lib = L.load()
    grid = L.Grid(dim, N)
    p = L.Pde({"poisson": L.POISSON, "convdiff": L.CONVDIFF}[pde], 1.0)
    return int(lib.ipmpde_footprint_bytes(C.byref(grid), C.byref(p), int(has_state_bounds),
                                          C.byref((opts or Options()).to_c())))
