"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/cheb.h declares, and rejects invalid plans before any
device call."""
import ctypes
import os

import pytest

from paper_2606_21410_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libchebfft.so is not built (run __graft_entry__.build())")
    return L.load()


def test_exports_every_declared_symbol():
    lib = _lib()
    names = L.declared_functions(os.path.join(ROOT, "include", "cheb.h"))
    assert len(names) >= 14
    debug = L.declared_functions(os.path.join(ROOT, "include", "cheb_debug.h"))
    assert debug == ["cheb_debug_copy", "cheb_debug_gemm"]
    for nm in names + debug:
        assert hasattr(lib, nm), nm


def test_status_strings():
    lib = _lib()
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        s = lib.cheb_status_string(code).decode()
        assert s and s != "unknown status"


def _grid(n=(9, 9, 9), lo=(0, 0, 0), hi=(1, 1, 1), bc=(0, 0, 1, 1, 1, 1), robin=(0.0,) * 6):
    g = L.cheb_grid()
    for a in range(3):
        g.n[a], g.lo[a], g.hi[a] = n[a], lo[a], hi[a]
    for f in range(6):
        g.bc[f] = bc[f]
        g.robin[f] = robin[f]
    return g


@pytest.mark.parametrize("kw,code", [
    (dict(n=(2, 9, 9)), L.CHEB_ERR_INVALID_ARG),
    (dict(n=(9, 514, 9)), L.CHEB_ERR_INVALID_ARG),
    (dict(lo=(0, 1, 0), hi=(1, 1, 1)), L.CHEB_ERR_INVALID_ARG),
    (dict(bc=(0, 0, 2, 1, 1, 1)), L.CHEB_ERR_INVALID_ARG),
    (dict(bc=(1, 1, 1, 1, 1, 1)), L.CHEB_ERR_SINGULAR_BC),
    # Robin coefficient on a Dirichlet face, a non-finite one, and sigma_lo
    # equal to the corner entry D_00 = -(2 N^2 + 1) / 3 of the unit interval
    # at N = 8, which zeroes the end value's coefficient
    (dict(robin=(1.0, 0, 0, 0, 0, 0)), L.CHEB_ERR_INVALID_ARG),
    (dict(robin=(0, 0, float("nan"), 0, 0, 0)), L.CHEB_ERR_INVALID_ARG),
    (dict(robin=(0, 0, -43.0, 0, 0, 0)), L.CHEB_ERR_INVALID_ARG),
])
def test_plan_validation(kw, code):
    lib = _lib()
    g = _grid(**kw)
    h = ctypes.c_void_p()
    rc = lib.cheb_plan_create(ctypes.byref(g), 0, None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert lib.cheb_last_error().decode()


def test_plan_validation_precision_and_nulls():
    lib = _lib()
    g = _grid()
    h = ctypes.c_void_p()
    assert lib.cheb_plan_create(ctypes.byref(g), 7, None, ctypes.byref(h)) == L.CHEB_ERR_INVALID_ARG
    assert lib.cheb_plan_create(None, 0, None, ctypes.byref(h)) == L.CHEB_ERR_INVALID_ARG
    assert lib.cheb_apply(None, None, None, None, 0) == L.CHEB_ERR_INVALID_ARG
    assert lib.cheb_solve(None, None, None, None, None, None, None) == L.CHEB_ERR_INVALID_ARG
    assert lib.cheb_prolong(None, None, None, None, None, None) == L.CHEB_ERR_INVALID_ARG
    assert lib.cheb_plan_destroy(None) == L.CHEB_OK


def test_load_case_packing_matches_generator():
    """The binding's homogenisation load cases pack the same face data and face
    types as the workload generator."""
    import numpy as np
    from paper_2606_21410_amd import workloads as W
    from paper_2606_21410_amd.api import load_case
    n = (5, 7, 6)
    grid = W.Grid(n, (0, 0, 0), (1, 1, 1), W.MIXED_X_BC)
    for a in range(3):
        bc, g = load_case(n, a, device="cpu")
        assert bc == W.load_case_bc(a)
        np.testing.assert_array_equal(g.numpy(), W.load_case_faces(grid, a))


def test_apparent_conductivity_rejects_null_plan():
    import ctypes
    lib = _lib()
    out = (ctypes.c_double * 3)()
    assert lib.cheb_apparent_conductivity(None, None, None, 0, 1.0, out) == L.CHEB_ERR_INVALID_ARG


def test_set_robin_nodes_rejects_null_plan():
    lib = _lib()
    assert lib.cheb_plan_set_robin_nodes(None, None) == L.CHEB_ERR_INVALID_ARG
