"""The fast-diagonalisation preconditioner (an extension of the paper's plain
LGMRES): its MFMA contraction kernel, exactness for constant K, and parity of
preconditioned FP64 / mixed / adjoint solves with the oracle."""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(16, 4, 16), (37, 29, 70), (127, 127, 300), (5, 130, 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mfma_gemm_layout(shape, prec):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import debug_gemm
    I, K, C = shape
    r = np.random.default_rng(I * 1000 + K)
    A = r.standard_normal((I, K))
    B = r.standard_normal((K, C))
    dt = torch.float64 if prec == "f64" else torch.float32
    D = to_host(debug_gemm(to_dev(A, dt), to_dev(B, dt)))
    ref = A.astype(np.float32 if prec == "f32" else np.float64).astype(np.float64) @ \
        B.astype(np.float32 if prec == "f32" else np.float64).astype(np.float64)
    assert rel_l2(D, ref) <= (1e-14 if prec == "f64" else 2e-6)


def test_precond_exact_for_constant_K():
    """Constant K: the preconditioner is the exact inverse of the reduced operator,
    so LGMRES converges in one or two applications."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    P = W.manufactured_sincos(17)
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    K = np.full(P.grid.n, 2.5)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64")
    d = lambda a: to_dev(a, torch.float64)
    u, info = plan.solve(d(K), d(P.f), d(P.g), opts=SolveOptions(rtol=1e-12, precond=True))
    log(f"precond const K: {info}")
    assert info["status"] == 0 and info["matvecs"] <= 4
    uref = O.solve(G, K, P.f, P.g)
    assert np.max(np.abs(to_host(u) - uref)) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "mixed", "f32"])
def test_precond_two_phase_33(prec):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    P = W.two_phase_problem(33, seed=1002, n_finest=129)
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    uref = O.solve(G, P.K, P.f, P.g, tol=1e-14)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, prec)
    dt = torch.float32 if prec == "f32" else torch.float64
    rtol = 1e-6 if prec == "f32" else 1e-13
    u, info = plan.solve(to_dev(P.K, dt), to_dev(P.f, dt), to_dev(P.g, dt),
                         opts=SolveOptions(rtol=rtol, precond=True))
    e = rel_l2(to_host(u), uref)
    log(f"precond {prec}: {info} err {e:.3e}")
    assert info["status"] == 0
    assert info["matvecs"] < 400
    assert e <= (1e-3 if prec == "f32" else 1e-9)


def test_precond_adjoint_vs_dense():
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    n = (9, 9, 9)
    bc = W.MIXED_X_BC
    LO, HI = (0, 0, 0), (1, 1, 1)
    G = O.Grid3(n, LO, HI, bc)
    K = W.random_conductivity(n, 51, 0.5)
    f = W.random_field(n, 52)
    g = W.random_faces(W.Grid(n, LO, HI, bc), 53)
    U = O.solve_dense(G, K, f, g)
    t = W.random_field(n, 54)
    _, g_ref = O.adjoint_dense(G, K, U, U - t)
    plan = Plan(n, LO, HI, bc, "f64")
    d = lambda a: to_dev(a, torch.float64)
    _, grad, info = plan.adjoint(d(K), d(U), d(U - t), SolveOptions(rtol=1e-13, precond=True))
    assert info["status"] == 0
    assert rel_l2(to_host(grad), g_ref) <= 1e-9


@pytest.mark.parametrize("shape,bcname", [
    ((33, 49, 65), "DDNNNN"),   # interior sizes 31, 47, 63: contraction widths 32, 48, 64
    ((97, 20, 129), "NDNNDN"),  # 95, 18, 127: widths 96, 32, 128; faces not mirror-symmetric
    ((81, 113, 9), "NNNDNN"),   # 79, 111, 7: widths 80, 112, 16
])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_precond_exact_for_constant_K_shapes(shape, bcname, prec):
    """Constant K on grids whose interior sizes cover every padded width of the
    preconditioner's contraction kernel: the preconditioner is the exact inverse,
    so LGMRES stops after a few applications -- for the forward solve and (FP64)
    for the adjoint solve, which applies the transposed contractions."""
    require_gpu()
    import torch
    from tests.gpu_util import BC_SETS
    from paper_2606_21410_amd.api import Plan, SolveOptions
    bc = BC_SETS[bcname]
    LO, HI = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    K = np.full(shape, 1.7)
    f = W.random_field(shape, 71)
    g = W.random_faces(W.Grid(shape, LO, HI, bc), 72)
    dt = torch.float32 if prec == "f32" else torch.float64
    d = lambda a: to_dev(a, dt)
    plan = Plan(shape, LO, HI, bc, prec)
    rtol = 1e-5 if prec == "f32" else 1e-11
    u, info = plan.solve(d(K), d(f), d(g), opts=SolveOptions(rtol=rtol, precond=True))
    log(f"const K {shape} {bcname} {prec}: {info}")
    assert info["status"] == 0 and info["matvecs"] <= 4
    if prec == "f64":
        r = W.random_field(shape, 73)
        _, _, ainfo = plan.adjoint(d(K), u, d(r), SolveOptions(rtol=1e-11, precond=True))
        log(f"adjoint const K {shape} {bcname}: {ainfo}")
        assert ainfo["status"] == 0 and ainfo["matvecs"] <= 4


@pytest.mark.parametrize("shape,robin", [
    ((34, 66, 98), None),                          # interior sizes 32, 64, 96
    ((130, 97, 129), None),                        # 128, 95, 127
    ((66, 130, 34), (0.0, 0.0, 0.7, 0.7, 0.0, 0.0)),  # Robin pair of equal sigma on the y faces
    ((258, 20, 257), None),                        # 256 and 255 on the generic path's split
])
def test_precond_exact_even_split_widths(shape, robin):
    """Same face type at both ends of every axis, so every axis takes the
    preconditioner's even-odd split contraction, on interior sizes m = 32, 64,
    96 and 128 (no middle node) next to 95 and 127 (a middle node): with
    constant K the preconditioner is the exact inverse, so the forward solve
    (FP64 and FP32) and the adjoint solve, which applies the transposed
    contractions, stop after a few applications."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    D_, N_ = 0, 1
    bc = (D_, D_, N_, N_, D_, D_)
    LO, HI = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    K = np.full(shape, 1.3)
    f = W.random_field(shape, 81)
    g = W.random_faces(W.Grid(shape, LO, HI, bc), 82)
    for prec in ("f64", "f32"):
        dt = torch.float32 if prec == "f32" else torch.float64
        d = lambda a: to_dev(a, dt)
        plan = Plan(shape, LO, HI, bc, prec, robin=robin)
        log(f"even split {shape} robin={robin} {prec}")
        u, info = plan.solve(d(K), d(f), d(g),
                             opts=SolveOptions(rtol=1e-5 if prec == "f32" else 1e-11, precond=True))
        log(f"  forward {info}")
        assert info["status"] == 0 and info["matvecs"] <= 4
        if prec == "f64":
            # the transposed operator's rounding floors the adjoint's relative
            # residual at 1.2e-11 when x has 258 nodes (measured the same with
            # and without the even-odd split of the m > 128 contractions), so
            # that grid's adjoint is held to 1e-10
            artol = 1e-10 if shape[0] > 200 else 1e-11
            r = W.random_field(shape, 83)
            _, _, ainfo = plan.adjoint(d(K), u, d(r), SolveOptions(rtol=artol, maxiter=50, precond=True))
            log(f"  adjoint {ainfo}")
            assert ainfo["status"] == 0 and ainfo["matvecs"] <= 4


@pytest.mark.parametrize("shape,bc,robin", [
    ((17, 17, 17), (0,) * 6, None),                       # interior 15: plain contraction, width 16
    ((33, 49, 65), (0, 0, 1, 1, 1, 1), None),             # 31 / 47 / 63: split, plain, split
    ((97, 20, 129), (1, 0, 1, 1, 0, 1), None),            # faces not mirror-symmetric: plain 96, 32, 128
    ((129, 129, 129), (0,) * 6, None),                    # the 129^3 workload's grid: split width 128
    ((17, 20, 257), (0,) * 6, None),                      # z interior 255: the generic contraction path
    # the generic path's even-odd split (m > 128, ceil(m/2) a multiple of 16)
    # on the x and y sides too, odd and even m, and with a Robin pair
    ((257, 17, 20), (0,) * 6, None),                      # x interior 255 (a middle node)
    ((20, 258, 17), (0, 0, 1, 1, 0, 0), None),            # y interior 256 (no middle node)
    ((17, 20, 226), (0, 0, 0, 0, 1, 1), None),            # z interior 224, halves of 112
    ((20, 17, 257), (0, 0, 0, 0, 1, 1), (0.0, 0.0, 0.0, 0.0, 0.7, 0.7)),  # z 255, Robin pair
    # faces that differ at the two ends of a long axis: the plain (unsplit)
    # contraction past 128 interior nodes, z side and x side
    ((20, 17, 200), (0, 0, 0, 0, 0, 1), None),            # z interior 198, Dirichlet-Neumann
    ((200, 17, 20), (1, 0, 0, 0, 0, 0), None),            # x interior 198, Neumann-Dirichlet
    ((66, 130, 34), (0, 0, 1, 1, 0, 0), (0.0, 0.0, 0.7, 0.7, 0.0, 0.0)),  # Robin pair, even widths
    # y and z axes with one 1-D problem (cubic y-z box), which share their
    # fragment tables
    ((98, 34, 34), (0, 1, 0, 0, 0, 0), "cube"),           # split, width 32
    ((100, 49, 49), (0, 0, 1, 1, 1, 1), "cube"),          # 47: plain, width 48
    ((97, 97, 97), (1, 1, 0, 1, 0, 1), "cube"),           # faces differ: plain, width 96
    ((99, 66, 66), (0, 0, 1, 1, 1, 1), "cube-robin"),     # split, width 64, Robin pairs
    ((129, 129, 129), (0, 0, 1, 1, 1, 1), "cube"),        # the 129^3 workload's faces: split 128
])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_precond_apply_vs_oracle(shape, bc, robin, prec):
    if robin == "cube" or robin == "cube-robin":
        box = ((0.0, 0.0, 0.0), (1.5, 1.0, 1.0))
        robin = (0.0, 0.0, 0.4, 0.4, 0.4, 0.4) if robin == "cube-robin" else None
    else:
        box = ((0.0, -1.0, 0.5), (1.0, 1.0, 2.0))
    _precond_case(shape, bc, robin, prec, box)


def _precond_case(shape, bc, robin, prec, box):
    """cheb_precond_apply against the oracle's fast diagonalisation (itself
    pinned to a direct solve of the constant-coefficient reduced operator),
    element by element on the interior, zero on the boundary.  The 1-D
    eigenvector matrices have condition numbers below 5 on these grids, so the
    apply loses little: FP32 factors and arithmetic emulated on the host stay
    within 5e-7 of the FP64 result, and the oracle's own output leaves a
    relative residual of up to 2e-12 under the constant-coefficient operator
    (the faces that are not mirror-symmetric take a general eigen-solver); the
    bars are 1e-11 (FP64, two independent decompositions) and 4e-6 (FP32).
    The transposed apply is checked by <P^T a, b> = <a, P b>."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    LO, HI = box
    kc = 1.7
    G = O.Grid3(shape, LO, HI, bc, robin)
    F = O.FDM(G, kc)
    r = W.random_field(shape, 91)
    ref = F.solve(r)
    dt = torch.float32 if prec == "f32" else torch.float64
    plan = Plan(shape, LO, HI, bc, "f64" if prec == "f64" else "f32", robin=robin)
    log(f"precond apply {shape} bc={bc} robin={robin} {prec}")
    out = to_host(plan.precond(to_dev(r, dt), kc))
    e = rel_l2(out, ref)
    log(f"  forward rel err {e:.3e}")
    assert e <= (4e-6 if prec == "f32" else 1e-11)
    interior = np.zeros(shape, dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    assert np.all(out[~interior] == 0.0)
    # the transpose: <P^T a, b> = <a, P b> on the interior
    a = W.random_field(shape, 92)
    b = W.random_field(shape, 93)
    pta = to_host(plan.precond(to_dev(a, dt), kc, transpose=True))
    pb = to_host(plan.precond(to_dev(b, dt), kc))
    assert np.all(pta[~interior] == 0.0)
    lhs = float(np.sum(pta[interior] * b[interior]))
    rhs = float(np.sum(a[interior] * pb[interior]))
    scale = np.linalg.norm(pta[interior]) * np.linalg.norm(b[interior])
    log(f"  transpose: <P^T a, b> - <a, P b> = {abs(lhs - rhs) / scale:.3e} (relative)")
    assert abs(lhs - rhs) <= (1e-5 if prec == "f32" else 1e-13) * scale
    # out may alias the input
    rr = to_dev(r, dt)
    plan.precond(rr, kc, out=rr)
    np.testing.assert_array_equal(to_host(rr), out)


def test_precond_apply_rejects_bad_arguments():
    require_gpu()
    import ctypes
    import torch
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import Plan
    plan = Plan((17, 17, 17), (0, 0, 0), (1, 1, 1), (0,) * 6, "f64")
    r = to_dev(W.random_field((17, 17, 17), 94), torch.float64)
    for kc in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(L.ChebError) as ei:
            plan.precond(r, kc)
        assert ei.value.code == L.CHEB_ERR_INVALID_ARG
    p = ctypes.c_void_p(r.data_ptr())
    assert plan.lib.cheb_precond_apply(plan.handle, L.CHEB_MIXED, 1.0, p, p, 0) == L.CHEB_ERR_INVALID_ARG
    assert plan.lib.cheb_precond_apply(plan.handle, L.CHEB_F64, 1.0, p, p, 1) == L.CHEB_ERR_INVALID_ARG
    assert plan.lib.cheb_precond_apply(plan.handle, L.CHEB_F64, 1.0, None, p, 0) == L.CHEB_ERR_INVALID_ARG
