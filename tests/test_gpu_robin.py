"""GPU parity of Robin rows du/dn + sigma u = g (the general linear boundary
operator of Section 2.3.1) against the oracle: the operator in its FULL, REDUCED
and transposed forms on both derivative routes, solves with and without the
preconditioner (including six Robin/Neumann faces, singular without sigma),
the adjoint and Newton on a Robin grid, and the rejections."""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

D_, N_ = O.DIRICHLET, O.NEUMANN
LO, HI = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
ROBIN = {
    "mixed": ((D_, N_, N_, N_, N_, N_), (0.0, 2.5, 0.7, 0.0, 1.3, 4.0)),
    "ydir": ((N_, N_, D_, N_, N_, N_), (3.0, 0.5, 0.0, 0.2, 1.0, 1.0)),
    "allrobin": ((N_,) * 6, (1.0, 2.0, 0.5, 0.5, 3.0, 0.1)),
}
# 129^3 is the metric workload's grid, run in the tile shape and route the bench times
SIZES = [(5, 4, 3), (17, 17, 17), (33, 17, 9), (65, 65, 65), (13, 6, 65), (129, 129, 129)]


def _plan(n, name, prec, route="auto"):
    from paper_2606_21410_amd.api import Plan
    bc, robin = ROBIN[name]
    return Plan(n, LO, HI, bc, prec, route=route, robin=robin), O.Grid3(n, LO, HI, bc, robin)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("name", list(ROBIN))
@pytest.mark.parametrize("route", ["fft", "matrix"])
def test_apply_full_reduced_transpose_f64(n, name, route):
    require_gpu()
    import torch
    d = lambda a: to_dev(a, torch.float64)
    log(f"robin apply n={n} {name} {route}")
    plan, G = _plan(n, name, "f64", route)
    u = W.random_field(n, 400)
    K = W.random_conductivity(n, 401, 0.5)
    for mode, fn in (("full", O.apply_full), ("reduced", O.apply_reduced),
                     ("transpose", O.apply_reduced_transpose)):
        y = to_host(plan.apply(d(K), d(u), mode=mode))
        e = rel_l2(y, fn(G, K, u))
        assert e <= 1e-12, (mode, e)


@pytest.mark.parametrize("n", [(17, 17, 17), (33, 17, 9)])
@pytest.mark.parametrize("name", list(ROBIN))
def test_apply_f32(n, name):
    require_gpu()
    import torch
    plan, G = _plan(n, name, "f32")
    u = W.random_field(n, 410).astype(np.float32).astype(np.float64)
    K = W.random_conductivity(n, 411, 0.5).astype(np.float32).astype(np.float64)
    for mode, fn in (("full", O.apply_full), ("reduced", O.apply_reduced)):
        y = to_host(plan.apply(to_dev(K, torch.float32), to_dev(u, torch.float32), mode=mode))
        assert rel_l2(y, fn(G, K, u)) <= 1e-5, mode


@pytest.mark.parametrize("name", list(ROBIN))
@pytest.mark.parametrize("prec,precond", [("f64", False), ("f64", True), ("mixed", True)])
def test_polynomial_solve_exact(name, prec, precond):
    """Degree-3 polynomial with linear K and Robin data: the discrete solution
    is the polynomial itself."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    bc, robin = ROBIN[name]
    P = W.manufactured_polynomial(9, bc, seed=5, robin=robin)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, bc, prec, robin=robin)
    u, info = plan.solve(d(P.K), d(P.f), d(P.g), opts=SolveOptions(rtol=1e-12, precond=precond))
    err = np.max(np.abs(to_host(u) - P.u_exact)) / np.max(np.abs(P.u_exact))
    log(f"robin poly {name} {prec} precond={precond}: {info['matvecs']} matvecs, err {err:.2e}")
    assert info["rc"] == 0 and err <= 1e-9


@pytest.mark.parametrize("name", list(ROBIN))
def test_heterogeneous_solve_vs_oracle(name):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    n = (17, 17, 17)
    plan, G = _plan(n, name, "f64")
    K = W.random_conductivity(n, 420, 0.5)
    f = W.random_field(n, 421)
    g = W.random_faces(W.Grid(n, LO, HI, G.bc), 422)
    Uo = O.solve_dense(G, K, f, g)
    u, info = plan.solve(d(K), d(f), d(g), opts=SolveOptions(rtol=1e-13, precond=True))
    e = rel_l2(to_host(u), Uo)
    log(f"robin hetero {name}: {info['matvecs']} matvecs, rel {e:.2e}")
    assert info["rc"] == 0 and e <= 1e-9


def test_sincos_large_grid_spectral():
    """65^3 with Robin y and z faces: the error against the analytic field is at
    the solver tolerance (a property that holds at any size)."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    robin = (0.0, 0.0, 1.5, 0.5, 2.0, 0.25)
    P = W.manufactured_sincos(65, robin=robin)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "mixed", robin=robin)
    u, info = plan.solve(d(P.K), d(P.f), d(P.g), opts=SolveOptions(rtol=1e-12, precond=True))
    err = np.max(np.abs(to_host(u) - P.u_exact))
    log(f"robin sincos 65^3: {info['matvecs']} matvecs, err {err:.2e}")
    assert info["rc"] == 0 and err <= 1e-9


def test_adjoint_vs_oracle():
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    n = (9, 11, 7)
    plan, G = _plan(n, "mixed", "f64")
    K = W.random_conductivity(n, 430, 0.4)
    f = W.random_field(n, 431)
    g = W.random_faces(W.Grid(n, LO, HI, G.bc), 432)
    U = O.solve_dense(G, K, f, g)
    dLdU = W.random_field(n, 433)
    lam_o, grad_o = O.adjoint_dense(G, K, U, dLdU)
    lam, grad, info = plan.adjoint(d(K), d(U), d(dLdU), opts=SolveOptions(rtol=1e-13))
    log(f"robin adjoint: {info['matvecs']} matvecs")
    assert info["rc"] == 0
    assert rel_l2(to_host(grad), grad_o) <= 1e-9


def test_newton_on_robin_grid_vs_oracle():
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    n = (13, 11, 9)
    plan, G = _plan(n, "ydir", "f64")
    K0 = W.random_conductivity(n, 440, 0.3)
    f = 0.5 * W.random_field(n, 441)
    g = 0.1 * W.random_faces(W.Grid(n, LO, HI, G.bc), 442)
    To, so, _ = O.newton(G, K0, 0.5, f, g, tol=1e-12)
    u, info = plan.newton(d(K0), d(f), d(g), alpha=0.5, tol=1e-12, max_steps=20,
                          opts=SolveOptions(rtol=1e-13, precond=True))
    assert info["rc"] == 0
    assert rel_l2(to_host(u), To) <= 1e-10


def test_rejections():
    require_gpu()
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import Batch, Plan
    with pytest.raises(L.ChebError):
        Plan((9, 9, 9), bc=(D_, N_, N_, N_, N_, N_), robin=(1.0, 0, 0, 0, 0, 0))
    with pytest.raises(L.ChebError):
        Plan((9, 9, 9), bc=(N_,) * 6)
    Plan((9, 9, 9), bc=(N_,) * 6, robin=(0, 0, 0, 0, 0, 0.5)).close()
    with pytest.raises(L.ChebError):
        Batch([((9, 9, 9), (0, 0, 0), (1, 1, 1), (D_, N_, N_, N_, N_, N_), (0, 1.0, 0, 0, 0, 0))])


@pytest.mark.parametrize("name", ["mixed", "allrobin"])
def test_f32_solve_vs_oracle(name):
    """FP32 plan with Robin rows: the solve against the oracle's dense LU, at
    FP32 accuracy (rtol 1e-5 on the reduced system)."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions
    n = (17, 17, 17)
    plan, G = _plan(n, name, "f32")
    K = W.random_conductivity(n, 450, 0.5)
    f = W.random_field(n, 451)
    g = W.random_faces(W.Grid(n, LO, HI, G.bc), 452)
    Uo = O.solve_dense(G, K, f, g)
    d = lambda a: to_dev(a, torch.float32)
    u, info = plan.solve(d(K), d(f), d(g), opts=SolveOptions(rtol=1e-5, precond=True))
    e = rel_l2(to_host(u), Uo)
    log(f"robin f32 {name}: {info['matvecs']} matvecs, rel {e:.2e}")
    assert info["rc"] == 0 and e <= 1e-3


def test_graph_replay_matches_eager():
    """Reduced applies with Robin rows captured in a HIP graph and replayed three
    times, with eager work in between: every replay equals the eager result."""
    require_gpu()
    import torch
    n = (33, 33, 33)
    plan, G = _plan(n, "allrobin", "f64")
    d = lambda a: to_dev(a, torch.float64)
    K = d(W.random_conductivity(n, 460, 0.5))
    us = [d(W.random_field(n, 461 + i)) for i in range(3)]
    ys = [torch.empty_like(us[0]) for _ in range(3)]
    ref = [to_host(plan.apply(K, u, mode="reduced")) for u in us]
    graph = plan.capture_applies(K, us, ys, "reduced")
    for rep in range(3):
        for y in ys:
            y.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        for y, r in zip(ys, ref):
            assert np.array_equal(to_host(y), r), rep
        plan.apply(K, us[0], mode="full")  # eager work between replays
        torch.cuda.synchronize()
