"""GPU parity of the matrix-core route (dense even-odd contraction on the matrix
cores) of the reduced operator and its transpose, against the CPU oracle and
against the FFT route.

Inputs as in the apply tests: u ~ N(0,1) at every node, K log-normal (sigma 0.5).
Bars: relative L2 error <= 1e-12 in FP64 and <= 1e-5 in FP32; the two routes
agree to <= 1e-13 in FP64.
"""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import BC_SETS, log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5

# every N the matrix route supports (16..128), ragged mixes with FFT-route axes;
# x and y of equal N share one launch (the last three: with another N on z),
# the other mixes take three
SIZES = [(17, 17, 17), (33, 33, 33), (49, 49, 49), (65, 65, 65), (97, 97, 97), (129, 129, 129),
         (33, 24, 65), (129, 17, 49), (13, 97, 33), (65, 65, 33), (33, 33, 129), (17, 17, 97)]
BCS = ["DDNNNN", "NDNNDN", "NNNDNN", "DDDDDD"]


def _case(n, bc, seed, lo=(0.0, -1.0, 0.5), hi=(1.0, 1.0, 2.0)):
    G = O.Grid3(n, lo, hi, bc)
    u = W.random_field(n, seed)
    K = W.random_conductivity(n, seed + 1, 0.5)
    return G, u, K


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bcname", BCS)
def test_matrix_route_f64(n, bcname):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    bc = BC_SETS[bcname]
    log(f"matrix route f64 n={n} bc={bcname}")
    G, u, K = _case(n, bc, 500)
    plan = Plan(n, G.lo, G.hi, bc, "f64", route="matrix")
    Kd, ud = to_dev(K, torch.float64), to_dev(u, torch.float64)
    yr = to_host(plan.apply(Kd, ud, mode="reduced"))
    assert rel_l2(yr, O.apply_reduced(G, K, u)) <= F64_TOL
    assert np.all(yr[~G.interior] == 0.0)
    yt = to_host(plan.apply(Kd, ud, mode="transpose"))
    assert rel_l2(yt, O.apply_reduced_transpose(G, K, u)) <= F64_TOL
    assert np.all(yt[~G.interior] == 0.0)
    # the FFT route of the same plan
    plan.set_route("fft")
    assert rel_l2(to_host(plan.apply(Kd, ud, mode="reduced")), yr) <= 1e-13
    assert rel_l2(to_host(plan.apply(Kd, ud, mode="transpose")), yt) <= 1e-13


@pytest.mark.parametrize("n", [(17, 17, 17), (33, 33, 33), (65, 65, 65), (129, 129, 129), (49, 24, 97),
                               (65, 65, 33)])
@pytest.mark.parametrize("bcname", ["DDNNNN", "NDNNDN"])
def test_matrix_route_f32(n, bcname):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    bc = BC_SETS[bcname]
    log(f"matrix route f32 n={n} bc={bcname}")
    G, u, K = _case(n, bc, 600)
    u32 = u.astype(np.float32).astype(np.float64)
    K32 = K.astype(np.float32).astype(np.float64)
    plan = Plan(n, G.lo, G.hi, bc, "f32", route="matrix")
    Kd, ud = to_dev(K32, torch.float32), to_dev(u32, torch.float32)
    y = to_host(plan.apply(Kd, ud, mode="reduced"))
    assert rel_l2(y, O.apply_reduced(G, K32, u32)) <= F32_TOL
    yt = to_host(plan.apply(Kd, ud, mode="transpose"))
    assert rel_l2(yt, O.apply_reduced_transpose(G, K32, u32)) <= F32_TOL


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_matrix_route_every_tile_shape(shape, prec):
    """Both tile shapes in both precisions, whatever the default or the
    autotuner would pick: two grids whose axes cover every N of the route
    (unit-stride and strided passes, the middle-row sums over 4, 8 and 16
    lanes), reduced operator and transpose, against the oracle."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    dt, tol = (torch.float64, F64_TOL) if prec == "f64" else (torch.float32, F32_TOL)
    for n, bcname in (((129, 33, 97), "NDNNDN"), ((17, 65, 49), "DDNNNN")):
        bc = BC_SETS[bcname]
        log(f"tile shape {shape} {prec} n={n} bc={bcname}")
        G, u, K = _case(n, bc, 800)
        if prec == "f32":
            u = u.astype(np.float32).astype(np.float64)
            K = K.astype(np.float32).astype(np.float64)
        plan = Plan(n, G.lo, G.hi, bc, prec, route="matrix")
        plan.set_tile_shape(shape, prec)
        Kd, ud = to_dev(K, dt), to_dev(u, dt)
        yr = to_host(plan.apply(Kd, ud, mode="reduced"))
        assert rel_l2(yr, O.apply_reduced(G, K, u)) <= tol
        assert np.all(yr[~G.interior] == 0.0)
        yt = to_host(plan.apply(Kd, ud, mode="transpose"))
        assert rel_l2(yt, O.apply_reduced_transpose(G, K, u)) <= tol
        assert np.all(yt[~G.interior] == 0.0)


def test_tile_shape_rejects_bad_arguments():
    require_gpu()
    from paper_2606_21410_amd.api import Plan
    from paper_2606_21410_amd import _lib as L
    plan = Plan((17, 17, 17), (0, 0, 0), (1, 1, 1), BC_SETS["DDNNNN"], "f64")
    for shape, prec in ((2, "f64"), (-1, "f32"), (0, "mixed")):
        with pytest.raises(L.ChebError):
            plan.set_tile_shape(shape, prec)


def test_matrix_route_dot_identity_129():
    """<v, A u> = <A^T v, u> for the matrix route at the benchmark size."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    n = (129, 129, 129)
    bc = BC_SETS["DDNNNN"]
    G, u, K = _case(n, bc, 700)
    v = W.random_field(n, 702)
    u[~G.interior] = 0.0
    v[~G.interior] = 0.0
    plan = Plan(n, G.lo, G.hi, bc, "f64", route="matrix")
    Kd = to_dev(K, torch.float64)
    Au = to_host(plan.apply(Kd, to_dev(u, torch.float64), mode="reduced"))
    Atv = to_host(plan.apply(Kd, to_dev(v, torch.float64), mode="transpose"))
    lhs, rhs = float(np.sum(v * Au)), float(np.sum(Atv * u))
    scale = np.linalg.norm(v) * np.linalg.norm(Au)
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_solve_matrix_route_matches_fft_route():
    """Preconditioned FP64 and mixed solves give the same answer on both routes."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    P = W.two_phase_problem(65, seed=1002, n_finest=129)
    d = lambda a: to_dev(a, torch.float64)
    out = {}
    for route in ("fft", "matrix"):
        for prec in ("f64", "mixed"):
            pl = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, prec, route=route)
            u, info = pl.solve(d(P.K), d(P.f), d(P.g), opts=SolveOptions(rtol=1e-12, precond=True))
            log(f"{route} {prec}: {info}")
            assert info["status"] == 0
            out[(route, prec)] = to_host(u)
    ref = out[("fft", "f64")]
    for k, v in out.items():
        assert rel_l2(v, ref) <= 1e-10, k


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_autotune_then_parity(prec):
    """The autotuner times every route / tile shape, picks one, and the reduced
    operator stays within the parity bar afterwards."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    n = (65, 33, 49)
    bc = BC_SETS["NDNNDN"]
    G, u, K = _case(n, bc, 900)
    plan = Plan(n, G.lo, G.hi, bc, prec)
    rep = plan.autotune(to_dev(K, torch.float64), to_dev(u, torch.float64))
    log(f"autotune {prec}: {rep}")
    for pname, r in rep.items():
        assert r["fft"] > 0 and r["matrix0"] > 0 and r["matrix1"] > 0
        assert r["chosen"] in ("fft", "matrix0", "matrix1")
    if prec == "f32":
        u32 = u.astype(np.float32).astype(np.float64)
        K32 = K.astype(np.float32).astype(np.float64)
        y = to_host(plan.apply(to_dev(K32, torch.float32), to_dev(u32, torch.float32), mode="reduced"))
        assert rel_l2(y, O.apply_reduced(G, K32, u32)) <= F32_TOL
    else:
        y = to_host(plan.apply(to_dev(K, torch.float64), to_dev(u, torch.float64), mode="reduced"))
        assert rel_l2(y, O.apply_reduced(G, K, u)) <= F64_TOL


@pytest.mark.parametrize("route", ["matrix", "fft"])
def test_graph_replay_matches_eager(route):
    """Applies recorded in a HIP graph: every replay (with eager work and
    synchronisations in between) reproduces the eager results exactly."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    n = (33, 33, 33)
    bc = BC_SETS["DDNNNN"]
    G, u, K = _case(n, bc, 1100)
    plan = Plan(n, G.lo, G.hi, bc, "f64", route=route)
    Kd = to_dev(K, torch.float64)
    us = [to_dev(W.random_field(n, 1101 + i), torch.float64) for i in range(3)]
    ys = [torch.empty_like(us[0]) for _ in range(3)]
    eager = [plan.apply(Kd, u_, mode="reduced").clone() for u_ in us]
    graph = plan.capture_applies(Kd, us, ys, "reduced")
    for rep in range(3):
        for y in ys:
            y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), rep
        # eager work on other data between replays
        other = plan.apply(Kd, us[2] * 2.0, mode="transpose")
        torch.cuda.synchronize()
        assert torch.isfinite(other).all()
