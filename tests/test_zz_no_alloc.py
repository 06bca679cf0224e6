"""The allocation-free prolongation entry point (cheb_prolong_noalloc): its
intermediates live in the library's static device scratch instead of the fine
plan's workspace.  Its output must equal the workspace entry point's
(cheb_prolong) on the same inputs, on two calls in a row -- the second on a
smaller grid pair, so it reuses a scratch array that the first call left
dirty -- and it must reject requests beyond the scratch size."""
import ctypes

import numpy as np
import pytest

from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

LO, HI = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)


def _noalloc(lib, pc, pf, uc, uf):
    f = lib.cheb_prolong_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 4
    return f(pc.handle, pf.handle, ctypes.c_void_p(uc.data_ptr()), ctypes.c_void_p(uf.data_ptr()))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_prolong_matches_workspace_entry(prec):
    require_gpu()
    import torch
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import Plan, prolong
    lib = L.load()
    dt = torch.float64 if prec == "f64" else torch.float32
    for nc, nf in (((65, 65, 65), (129, 129, 129)), ((17, 9, 13), (33, 17, 13))):
        log(f"noalloc prolong {prec} {nc} -> {nf}")
        pc = Plan(nc, LO, HI, W.MIXED_X_BC, prec)
        pf = Plan(nf, LO, HI, W.MIXED_X_BC, prec)
        uc = to_dev(W.random_field(nc, 91), dt)
        ref, _ = prolong(pc, pf, uc)
        torch.cuda.synchronize()
        uf = torch.full(nf, float("nan"), dtype=dt, device="cuda")
        torch.cuda.synchronize()
        rc = _noalloc(lib, pc, pf, uc, uf)
        assert rc == 0, lib.cheb_last_error().decode()
        got, want = to_host(uf), to_host(ref)
        log(f"  rel diff {rel_l2(got, want):.2e}")
        assert np.all(np.isfinite(got))
        assert rel_l2(got, want) <= (1e-13 if prec == "f64" else 1e-6)
        np.testing.assert_array_equal(got, want)


def test_noalloc_prolong_rejects_oversize():
    require_gpu()
    import torch
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import Plan
    lib = L.load()
    nc, nf = (200, 200, 200), (385, 385, 385)
    pc = Plan(nc, LO, HI, W.MIXED_X_BC, "f64")
    pf = Plan(nf, LO, HI, W.MIXED_X_BC, "f64")
    uc = torch.zeros(nc, dtype=torch.float64, device="cuda")
    uf = torch.zeros(nf, dtype=torch.float64, device="cuda")
    rc = _noalloc(lib, pc, pf, uc, uf)
    assert rc == -5
    assert "static scratch" in lib.cheb_last_error().decode()
