"""GPU parity of the Newton path for k = K0 / (1 + alpha T) (Section 3.4):
residual and Jacobian action element by element against the oracle, the
Newton-LGMRES solve against the oracle's Newton iteration and against the
analytic temperature of the manufactured problem, and the hierarchical chain."""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import BC_SETS, log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

THERMAL_BC = (O.DIRICHLET, O.NEUMANN, O.DIRICHLET, O.NEUMANN, O.NEUMANN, O.NEUMANN)
CASES = [((17, 17, 17), THERMAL_BC, (0, 0, 0), (1, 1, 1)),
         ((19, 13, 9), BC_SETS["NDNNDN"], (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)),
         ((33, 17, 65), BC_SETS["DDNNNN"], (0, 0, 0), (1, 2, 1)),
         ((5, 4, 3), BC_SETS["NNNNND"], (0, 0, 0), (1, 1, 1)),
         ((129, 129, 129), THERMAL_BC, (0, 0, 0), (1, 1, 1)),
         # x and y share a launch (their own tables and c_a), z another N
         ((33, 33, 65), BC_SETS["NDNNDN"], (0.0, -1.0, 0.5), (1.0, 1.0, 2.0))]


def _state(n, seed):
    """A full nodal state with 1 + 0.5 T > 0.4 everywhere, and a random K0."""
    T = 0.4 * np.tanh(W.random_field(n, seed))
    return T, W.random_conductivity(n, seed + 1)


@pytest.mark.parametrize("n", [(33, 33, 33), (65, 65, 33), (129, 129, 129)])
def test_jacobian_forms_agree(n):
    """The Jacobian action in its three forms on one plan: the k' terms in the
    matrix-core apply's flux epilogues (tile shape 1, x and y in one launch),
    one matrix-core derivative pass per axis (tile shape 0), and the FFT
    route's derivative passes; all against the oracle's Jacobian."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    d = lambda a: to_dev(a, torch.float64)
    bc = BC_SETS["NDNNDN"]
    lo, hi = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    G = O.Grid3(n, lo, hi, bc)
    T, K0 = _state(n, 41)
    v = W.random_field(n, 44)
    y_o = O.newton_jacobian(G, K0, 0.5, T, v)
    scale = np.max(np.abs(y_o))
    plan = Plan(n, lo, hi, bc, "f64")
    ys = {}
    for name, setup in (("fused", lambda: plan.set_tile_shape(1, "f64")),
                        ("passes", lambda: plan.set_tile_shape(0, "f64")),
                        ("fft", lambda: plan.set_route("fft"))):
        setup()
        log(f"jacobian form {name} n={n}")
        ys[name] = to_host(plan.newton_jacobian(d(K0), d(T), d(v), 0.5))
        assert np.max(np.abs(ys[name] - y_o)) <= 1e-12 * scale
        assert np.all(ys[name][~G.interior] == 0.0)
    for name in ("passes", "fft"):
        assert np.max(np.abs(ys[name] - ys["fused"])) <= 1e-13 * scale


@pytest.mark.parametrize("n,bc,lo,hi", CASES)
def test_residual_and_jacobian_vs_oracle(n, bc, lo, hi):
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan
    d = lambda a: to_dev(a, torch.float64)
    G = O.Grid3(n, lo, hi, bc)
    T, K0 = _state(n, 31)
    f = W.random_field(n, 33)
    v = W.random_field(n, 34)  # boundary values must be ignored
    alpha = 0.5
    plan = Plan(n, lo, hi, bc, "f64")
    r = to_host(plan.newton_residual(d(K0), d(T), d(f), alpha))
    y = to_host(plan.newton_jacobian(d(K0), d(T), d(v), alpha))
    r_o = O.newton_residual(G, K0, alpha, T, f)
    y_o = O.newton_jacobian(G, K0, alpha, T, v)
    er = np.max(np.abs(r - r_o)) / np.max(np.abs(r_o))
    ey = np.max(np.abs(y - y_o)) / np.max(np.abs(y_o))
    log(f"newton n={n}: residual {er:.2e} jacobian {ey:.2e}")
    assert er <= 1e-12 and ey <= 1e-12
    assert np.all(r[~G.interior] == 0.0) and np.all(y[~G.interior] == 0.0)


@pytest.mark.parametrize("prec,precond", [("f64", False), ("f64", True), ("mixed", True)])
def test_thermal_newton_vs_oracle_and_exact(prec, precond):
    """Section 3.4 problem at N = 16 from T_0 = lift(0, g)."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    P = W.thermal_nonlinear(17)
    G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
    To, so, its = O.newton(G, P.K, 0.5, P.f, P.g, tol=1e-12)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, prec)
    u, info = plan.newton(d(P.K), d(P.f), d(P.g), alpha=0.5, tol=1e-12, max_steps=20,
                          opts=SolveOptions(rtol=1e-13, precond=precond, history_len=32))
    uh = to_host(u)
    log(f"newton {prec} precond={precond}: {info['newton_steps']} steps {info['mv_per_step']} "
        f"(oracle {so} {its}); history {info.get('history')}")
    assert info["rc"] == 0
    assert info["newton_steps"] <= so + 1
    assert rel_l2(uh, To) <= 1e-10
    assert np.max(np.abs(uh - P.u_exact)) <= 2.0 * 6.270730e-9


def test_random_problem_newton_vs_oracle():
    """Ragged grid, random K0, mixed faces, small random data."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    n, bc, lo, hi = (13, 17, 11), BC_SETS["NDNNDN"], (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    G = O.Grid3(n, lo, hi, bc)
    grid = W.Grid(n, lo, hi, bc)
    K0 = W.random_conductivity(n, 51, 0.3)
    f = 0.5 * W.random_field(n, 52)
    g = 0.1 * W.random_faces(grid, 53)
    To, so, its = O.newton(G, K0, 0.5, f, g, tol=1e-12)
    plan = Plan(n, lo, hi, bc, "f64")
    u, info = plan.newton(d(K0), d(f), d(g), alpha=0.5, tol=1e-12, max_steps=20,
                          opts=SolveOptions(rtol=1e-13, precond=True))
    log(f"random newton: {info['newton_steps']} steps {info['mv_per_step']} (oracle {so})")
    assert info["rc"] == 0
    assert rel_l2(to_host(u), To) <= 1e-10


def test_alpha_zero_matches_linear_solve():
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    P = W.two_phase_problem(17, seed=1003, volume_fraction=0.3, contrast=10.0)
    plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64")
    opts = SolveOptions(rtol=1e-13, precond=True)
    u_lin, _ = plan.solve(d(P.K), d(P.f), d(P.g), opts=opts)
    u, info = plan.newton(d(P.K), d(P.f), d(P.g), alpha=0.0, tol=1e-11, max_steps=5, opts=opts)
    assert info["rc"] == 0 and info["newton_steps"] == 1
    assert rel_l2(to_host(u), to_host(u_lin)) <= 1e-11


def test_hierarchical_thermal_chain():
    """N = 8 -> 16 -> 32 -> 64 -> 128 with prolonged warm starts (the
    refinement of Section 3.4): the error against the analytic T falls to the
    solver tolerance, Newton needs at most one update past N = 16, and e_ref
    decays."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions, prolong
    d = lambda a: to_dev(a, torch.float64)
    opts = SolveOptions(rtol=1e-10, precond=True)
    prev, errs, erefs = None, {}, {}
    for N in (8, 16, 32, 64, 128):
        P = W.thermal_nonlinear(N + 1)
        plan = Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, "f64")
        u0 = prolong(prev[0], plan, prev[1])[0] if prev else None
        u, info = plan.newton(d(P.K), d(P.f), d(P.g), alpha=0.5, u0=u0, tol=1e-9, max_steps=20,
                              opts=opts)
        assert info["rc"] == 0
        errs[N] = float(np.max(np.abs(to_host(u) - P.u_exact)))
        if prev:
            erefs[N] = prolong(prev[0], plan, prev[1], uf_solved=u)[1]
        log(f"thermal N={N}: newton {info['newton_steps']} {info['mv_per_step']} err {errs[N]:.3e} "
            f"e_ref {erefs.get(N, float('nan')):.3e}")
        if N >= 32:
            assert info["newton_steps"] <= 1
        prev = (plan, u)
    assert 0.5 * 4.903119e-4 <= errs[8] <= 2.0 * 4.903119e-4
    assert errs[16] <= 2.0 * 6.270730e-9
    assert errs[32] <= 2e-9 and errs[64] <= 2e-9 and errs[128] <= 2e-9
    assert erefs[32] < erefs[16] and erefs[64] < erefs[32]


def test_newton_rejects_bad_inputs():
    require_gpu()
    import torch
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import Plan
    d = lambda a: to_dev(a, torch.float64)
    n = (9, 9, 9)
    plan = Plan(n, (0, 0, 0), (1, 1, 1), THERMAL_BC, "f64")
    T = np.full(n, -3.0)  # 1 + 0.5 T < 0: no positive conductivity
    with pytest.raises(L.ChebError):
        plan.newton_residual(d(np.ones(n)), d(T), d(np.zeros(n)), 0.5)
    p32 = Plan(n, (0, 0, 0), (1, 1, 1), THERMAL_BC, "f32")
    with pytest.raises(L.ChebError):
        p32.newton_residual(d(np.ones(n)), d(np.zeros(n)), d(np.zeros(n)), 0.5)
