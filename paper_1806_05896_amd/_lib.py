"""ctypes declarations of the libipmpde C ABI (include/ipmpde.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipmpde.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONVERGED, EKRYLOV, EBREAKDOWN = range(7)
POISSON, CONVDIFF, HEAT, POISSON_Q1 = 0, 1, 2, 3
MINRES, FGMRES = 0, 1
PD, PT, PPI = 0, 1, 2
FP64, FP32 = 0, 1
MU_PAPER, MU_CENTRAL = 0, 1
MASS_UNIT, MASS_HD = 0, 1
TILE_AUTO, TILE_SMALL, TILE_LARGE = 0, 1, 2
TUNE_PRECISION = 1
MAX_HIST = 256

FIELDS = {
    "u": 0, "y": 1, "p": 2, "w": 3, "v": 4, "lam_ya": 5, "lam_yb": 6, "lam_wa": 7, "lam_wb": 8,
    "lam_va": 9, "lam_vb": 10, "dy": 11, "dw": 12, "dv": 13, "dp": 14, "theta_y": 15, "theta_w": 16,
    "theta_v": 17, "fhat": 18,
}

ERROR_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
               ENOTCONVERGED: "ENOTCONVERGED", EKRYLOV: "EKRYLOV", EBREAKDOWN: "EBREAKDOWN"}


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int)]


class Pde(C.Structure):
    _fields_ = [("kind", C.c_int), ("eps", C.c_double)]


class COptions(C.Structure):
    _fields_ = [
        ("sigma", C.c_double), ("alpha0", C.c_double), ("eps_p", C.c_double), ("eps_d", C.c_double),
        ("eps_c", C.c_double), ("mu0", C.c_double), ("ipm_maxit", C.c_int), ("fixed_nli", C.c_int),
        ("krylov", C.c_int), ("precond", C.c_int), ("restart", C.c_int), ("krylov_tol", C.c_double),
        ("krylov_maxit", C.c_int), ("vcycles", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int),
        ("omega", C.c_double), ("mg_precision", C.c_int), ("chunk", C.c_int), ("use_graphs", C.c_int),
        ("mu_rule", C.c_int), ("mass_scaling", C.c_int), ("mg_tile", C.c_int), ("lanes", C.c_int),
    ]


class CStats(C.Structure):
    _fields_ = [
        ("status", C.c_int), ("nli", C.c_int), ("krylov_its", C.c_int), ("krylov_fail", C.c_int),
        ("xi_p", C.c_double), ("xi_d", C.c_double), ("xi_c", C.c_double), ("mu", C.c_double),
        ("solve_ms", C.c_double), ("hist_len", C.c_int),
        ("hist_krylov", C.c_int * MAX_HIST),
        ("hist_mu", C.c_double * MAX_HIST),
        ("hist_xi_p", C.c_double * MAX_HIST), ("hist_xi_d", C.c_double * MAX_HIST),
        ("hist_xi_c", C.c_double * MAX_HIST),
        ("hist_alpha_p", C.c_double * MAX_HIST), ("hist_alpha_d", C.c_double * MAX_HIST),
        ("hist_krylov_relres", C.c_double * MAX_HIST),
    ]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("nli", C.c_int), ("krylov_its", C.c_int),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double), ("footprint_bytes", C.c_size_t)]


class EngineInfo(C.Structure):
    _fields_ = [("running", C.c_int), ("queued", C.c_int), ("groups", C.c_int),
                ("bytes_in_use", C.c_size_t), ("peak_bytes", C.c_size_t), ("budget_bytes", C.c_size_t),
                ("steps", C.c_long)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "ipmpde_version": (C.c_char_p, []),
    "ipmpde_last_error": (C.c_char_p, []),
    "ipmpde_default_options": (C.c_int, [C.POINTER(COptions)]),
    "ipmpde_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, C.c_void_p]),
    "ipmpde_problem_create": (C.c_int, [C.POINTER(Grid), C.POINTER(Pde), C.c_double, C.c_double]
                              + [C.c_void_p] * 7 + [C.POINTER(C.c_void_p)]),
    "ipmpde_heat_create": (C.c_int, [C.POINTER(Grid), C.c_int, C.c_double, C.c_double, C.c_double]
                           + [C.c_void_p] * 8 + [C.POINTER(C.c_void_p)]),
    "ipmpde_problem_destroy": (None, [C.c_void_p]),
    "ipmpde_footprint_bytes": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Pde), C.c_int, C.POINTER(COptions)]),
    "ipmpde_solve": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_void_p]),
    "ipmpde_query": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "ipmpde_set_observation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ipmpde_set_field": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "ipmpde_reset": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_void_p]),
    "ipmpde_ipm_step": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_double, C.c_void_p,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int),
                                  C.POINTER(C.c_double)]),
    "ipmpde_newton_direction": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_double, C.c_void_p,
                                          C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "ipmpde_measures": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    "ipmpde_measures_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]),
    "ipmpde_get_stats": (C.c_int, [C.c_void_p, C.POINTER(CStats)]),
    "ipmpde_apply_operator": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ipmpde_apply_saddle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ipmpde_apply_precond": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ipmpde_newton_setup": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_double, C.c_void_p]),
    "ipmpde_query_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ipmpde_time_kernel": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_int, C.c_int, C.c_void_p,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ipmpde_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p)]),
    "ipmpde_batch_destroy": (None, [C.c_void_p]),
    "ipmpde_batch_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "ipmpde_batch_autotune": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_int, C.c_char_p, C.c_void_p,
                                        C.POINTER(COptions), C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "ipmpde_batch_time_kernel": (C.c_int, [C.c_void_p, C.POINTER(COptions), C.c_int, C.c_int, C.c_void_p,
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ipmpde_engine_create": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    "ipmpde_engine_destroy": (None, [C.c_void_p]),
    "ipmpde_engine_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(COptions), C.POINTER(C.c_uint64)]),
    "ipmpde_engine_step": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ipmpde_engine_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(RequestInfo)]),
    "ipmpde_engine_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ipmpde_engine_get_info": (C.c_int, [C.c_void_p, C.POINTER(EngineInfo)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libipmpde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libipmpde is not built ({path} missing); run __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class IpmpdeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, allow=()):
    if code == OK or code in allow:
        return code
    raise IpmpdeError(code, load().ipmpde_last_error().decode())
