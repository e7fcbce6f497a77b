"""The C-ABI library loads and exports every entry point include/ipmpde.h
declares, and host-side validation rejects bad inputs before any device work
(no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1806_05896_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipmpde.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1806_05896_amd.api import build_library
        build_library()
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipmpde_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ipmpde_problem_create", "ipmpde_solve", "ipmpde_query", "ipmpde_get_stats",
                     "ipmpde_problem_destroy", "ipmpde_set_allocator", "ipmpde_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding describes each of them
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_struct_layouts_match_header(lib):
    # the options struct round-trips through the library's default filler
    o = L.COptions()
    assert lib.ipmpde_default_options(C.byref(o)) == L.OK
    assert o.sigma == 0.2 and o.alpha0 == 0.995 and o.krylov_tol == 1e-10
    assert o.nu_pre == 2 and o.nu_post == 2 and o.restart == 30 and o.chunk == 8
    assert o.lanes == 1
    assert lib.ipmpde_version().decode().startswith("libipmpde")


def test_binding_structs_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of the binding's option and statistics structs
    equal those a C compiler gives the header's declarations."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ipmpde.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ipmpde_options), '
                   'offsetof(ipmpde_options, mu_rule), offsetof(ipmpde_options, mass_scaling), '
                   'offsetof(ipmpde_options, mg_tile), offsetof(ipmpde_options, lanes), '
                   'sizeof(ipmpde_stats), offsetof(ipmpde_stats, hist_krylov_relres)); return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(L.COptions), L.COptions.mu_rule.offset, L.COptions.mass_scaling.offset, L.COptions.mg_tile.offset,
            L.COptions.lanes.offset, C.sizeof(L.CStats), L.CStats.hist_krylov_relres.offset]
    assert got == want


def test_default_options_use_the_unit_mass_form(lib):
    o = L.COptions()
    assert lib.ipmpde_default_options(C.byref(o)) == L.OK
    assert o.mass_scaling == L.MASS_UNIT and o.mu0 == 1.0 and o.eps_p == 1e-6


def _create(lib, dim=2, N=7, pde=L.POISSON, eps=1.0, alpha=1e-2, beta=1e-3, ua=-1.0, ub=1.0, ya=None, yb=None,
            yd=None):
    n = N ** dim
    arr = lambda v: None if v is None else np.full(n, v, dtype=np.float64)
    ua_, ub_, ya_, yb_ = arr(ua), arr(ub), arr(ya), arr(yb)
    yd_ = np.zeros(n) if yd is None else yd
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    rc = lib.ipmpde_problem_create(C.byref(L.Grid(dim, N)), C.byref(L.Pde(pde, eps)), alpha, beta, ptr(ua_), ptr(ub_),
                                   ptr(ya_), ptr(yb_), ptr(yd_), None, None, C.byref(h))
    return rc, lib.ipmpde_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(N=8), "2^k - 1"),
    (dict(N=1), "2^k - 1"),
    (dict(dim=4), "dim"),
    (dict(pde=L.CONVDIFF, dim=3), "2D only"),
    (dict(pde=L.CONVDIFF, eps=0.0), "eps"),
    (dict(alpha=0.0), "alpha"),
    (dict(beta=-1.0), "beta"),
    (dict(ua=0.0), "u_a < 0 < u_b"),
    (dict(ub=0.0), "u_a < 0 < u_b"),
    (dict(ya=0.5, yb=0.5), "y_a < y_b"),
    (dict(ya=-0.5), "both"),
    (dict(yd=np.full(49, np.nan)), "NaN"),
])
def test_create_rejects_bad_input_on_the_host(lib, kw, msg):
    rc, err = _create(lib, **kw)
    assert rc == L.EINVAL
    assert msg in err


def test_null_handles_are_rejected(lib):
    assert lib.ipmpde_solve(None, None, None) == L.EINVAL
    assert lib.ipmpde_query(None, 0, None, 0) == L.EINVAL
    s = L.CStats()
    assert lib.ipmpde_get_stats(None, C.byref(s)) == L.EINVAL
    lib.ipmpde_problem_destroy(None)  # no-op


def test_allocator_pair_must_be_complete(lib):
    keep = L.ALLOC_FN(lambda n, ctx: None)
    assert lib.ipmpde_set_allocator(keep, L.FREE_FN(), None) == L.EINVAL
    assert lib.ipmpde_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == L.OK


def test_footprint_grows_with_grid(lib):
    o = L.COptions()
    lib.ipmpde_default_options(C.byref(o))
    f = lambda N: lib.ipmpde_footprint_bytes(C.byref(L.Grid(2, N)), C.byref(L.Pde(L.POISSON, 1.0)), 1, C.byref(o))
    assert f(511) > 3.5 * f(255) > 0


def test_engine_argument_checks(lib):
    h = C.c_void_p()
    assert lib.ipmpde_engine_create(0, 4, C.byref(h)) == L.EINVAL
    assert lib.ipmpde_engine_create(1 << 30, 0, C.byref(h)) == L.EINVAL
    assert lib.ipmpde_engine_create(1 << 30, 5000, C.byref(h)) == L.EINVAL
    assert lib.ipmpde_engine_create(1 << 30, 4, None) == L.EINVAL
    assert lib.ipmpde_engine_create(1 << 30, 4, C.byref(h)) == L.OK and h.value
    info = L.RequestInfo()
    assert lib.ipmpde_engine_poll(h, C.c_uint64(7), C.byref(info)) == L.EINVAL
    assert lib.ipmpde_engine_release(h, C.c_uint64(7)) == L.EINVAL
    ei = L.EngineInfo()
    assert lib.ipmpde_engine_get_info(h, C.byref(ei)) == L.OK
    assert (ei.running, ei.queued, ei.bytes_in_use, ei.budget_bytes) == (0, 0, 0, 1 << 30)
    t = C.c_uint64()
    assert lib.ipmpde_engine_submit(h, None, None, C.byref(t)) == L.EINVAL
    assert lib.ipmpde_engine_step(None, None, None, None) == L.EINVAL
    lib.ipmpde_engine_destroy(h)
    lib.ipmpde_engine_destroy(None)


def test_footprint_counts_fgmres_basis_and_precision(lib):
    o = L.COptions()
    lib.ipmpde_default_options(C.byref(o))
    g, pd = L.Grid(2, 255), L.Pde(L.CONVDIFF, 0.005)
    base = lib.ipmpde_footprint_bytes(C.byref(g), C.byref(pd), 0, C.byref(o))
    o.krylov = L.FGMRES
    fg = lib.ipmpde_footprint_bytes(C.byref(g), C.byref(pd), 0, C.byref(o))
    n4 = 4 * 255 * 255
    assert fg - base == 8 * n4 * (2 * o.restart + 1)
    o.krylov = L.MINRES
    o.mg_precision = L.FP64
    f64 = lib.ipmpde_footprint_bytes(C.byref(g), C.byref(pd), 0, C.byref(o))
    assert f64 > base
    assert lib.ipmpde_footprint_bytes(C.byref(L.Grid(2, 100)), C.byref(pd), 0, None) == 0


@pytest.mark.parametrize("dim,N,nt,tau,msg", [
    (3, 7, 4, 0.25, "2D grid"),
    (2, 8, 4, 0.25, "2^k - 1"),
    (2, 7, 0, 0.25, "nt must be"),
    (2, 7, 70000, 0.25, "nt must be"),
    (2, 7, 4, 0.0, "tau must be positive"),
    (2, 7, 4, float("nan"), "tau must be positive"),
    (2, 2047, 65535, 0.01, "too many space-time nodes"),
])
def test_heat_create_rejects_bad_shapes_on_the_host(lib, dim, N, nt, tau, msg):
    """ipmpde_heat_create validates the grid and the time axis before it
    touches the device."""
    h = C.c_void_p()
    rc = lib.ipmpde_heat_create(C.byref(L.Grid(dim, N)), nt, tau, 1e-2, 1e-3, None, None, None, None, None, None,
                                None, None, C.byref(h))
    assert rc == L.EINVAL
    assert msg in lib.ipmpde_last_error().decode()
    assert not h.value


def test_problem_create_refuses_the_heat_kind(lib):
    h = C.c_void_p()
    rc = lib.ipmpde_problem_create(C.byref(L.Grid(2, 7)), C.byref(L.Pde(L.HEAT, 1.0)), 1e-2, 1e-3, None, None,
                                   None, None, None, None, None, C.byref(h))
    assert rc == L.EINVAL and "ipmpde_heat_create" in lib.ipmpde_last_error().decode()
