"""GPU parity of the batched solver (cheb_batch_*) and of the homogenisation
driver: every system of a batch against the single-system solver and against
the oracle's exact solution; apparent conductivities against the oracle."""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

BOX = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))


def _systems(sizes, seed0):
    """Log-normal microstructures (sigma 1, l 0.2) with the three load cases each."""
    out = []
    for i, n in enumerate(sizes):
        nn = (n, n, n)
        grid = W.Grid(nn, BOX[0], BOX[1], W.MIXED_X_BC)
        K = W.lognormal_conductivity(grid, 1004 + seed0 + i, 1.0, 0.2)
        for a in range(3):
            g = W.Grid(nn, BOX[0], BOX[1], W.load_case_bc(a))
            out.append((nn, W.load_case_bc(a), K, np.zeros(nn), W.load_case_faces(g, a)))
    return out


def _batch_solve(systems, prec, opts):
    import torch
    from paper_2606_21410_amd.api import Batch
    d = lambda a: to_dev(a, torch.float64)
    B = Batch([(n, BOX[0], BOX[1], bc) for n, bc, _, _, _ in systems], prec)
    us, infos = B.solve([d(s[2]) for s in systems], [d(s[3]) for s in systems], [d(s[4]) for s in systems],
                        opts=opts)
    return [to_host(u) for u in us], infos


def test_batch_matches_single_solves_f64():
    """Mixed sizes (matrix-core groups 17^3 and 33^3, FFT-route 25^3), three load
    cases each: every batched solution equals the single-system solve up to the
    solver tolerance.  Both stop at relative residual 1e-12; the plain reduced
    system of these log-normal fields (sigma 1) has an effective condition
    number up to ~1e4 at 33^3, so two such solves may differ by ~2e-8.  The
    batched and single solvers reduce in different orders, so their restarted
    Krylov paths drift apart at rounding level; over the ~10^4 matvecs of these
    unpreconditioned solves that moves the count by several per cent."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Plan, SolveOptions
    systems = _systems([17, 25, 33], 0)
    opts = SolveOptions(rtol=1e-12, maxiter=20000)
    us, infos = _batch_solve(systems, "f64", opts)
    d = lambda a: to_dev(a, torch.float64)
    for (n, bc, K, f, g), u, info in zip(systems, us, infos):
        assert info["status"] == 0, info
        pl = Plan(n, BOX[0], BOX[1], bc, "f64")
        us_, inf1 = pl.solve(d(K), d(f), d(g), opts=opts)
        e = rel_l2(u, to_host(us_))
        log(f"n={n[0]} bc={bc}: batch mv {info['matvecs']} single mv {inf1['matvecs']} diff {e:.2e}")
        assert e <= 1e-7
        assert abs(info["matvecs"] - inf1["matvecs"]) <= 0.10 * inf1["matvecs"] + 5


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_shared_K_equals_separate_copies(prec):
    """The three load cases of a microstructure given one K tensor share one
    packed copy (their tiles read the same conductivity lines); the results,
    statuses and matvec counts are those of the same batch given three
    separate copies of K, bit for bit (matrix-core groups 17^3 and 33^3 and
    the FFT-route 25^3)."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Batch, SolveOptions
    d = lambda a: to_dev(a, torch.float64)
    systems = _systems([17, 25, 33], 7)
    opts = SolveOptions(rtol=1e-10, maxiter=4000, precond=True)
    grids = [(n, BOX[0], BOX[1], bc) for n, bc, _, _, _ in systems]
    Ks_shared = []
    for i in range(0, len(systems), 3):
        Kt = d(systems[i][2])
        Ks_shared += [Kt, Kt, Kt]
    Ks_sep = [d(s[2]) for s in systems]
    fs = [d(s[3]) for s in systems]
    gs = [d(s[4]) for s in systems]
    B = Batch(grids, prec)
    u1, i1 = B.solve(Ks_shared, fs, gs, opts=opts)
    u2, i2 = B.solve(Ks_sep, fs, gs, opts=opts)
    u3, i3 = B.solve(Ks_shared, fs, gs, opts=opts)
    for a, b, c, ia, ib, ic in zip(u1, u2, u3, i1, i2, i3):
        assert ia["status"] == 0 and ia["matvecs"] == ib["matvecs"] == ic["matvecs"]
        np.testing.assert_array_equal(to_host(a), to_host(b))
        np.testing.assert_array_equal(to_host(a), to_host(c))


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_batch_precond_vs_oracle(prec):
    """Preconditioned batched solves (FP64, and FP32 inner / FP64 refinement)
    reach the oracle's exact solutions to 1e-8."""
    require_gpu()
    from paper_2606_21410_amd.api import SolveOptions
    systems = _systems([17, 33], 10)
    us, infos = _batch_solve(systems, prec, SolveOptions(rtol=1e-11, maxiter=4000, precond=True))
    for (n, bc, K, f, g), u, info in zip(systems, us, infos):
        G = O.Grid3(n, BOX[0], BOX[1], bc)
        ref = O.solve(G, K, f, g, tol=1e-14)
        e = rel_l2(u, ref)
        log(f"{prec} n={n[0]} bc={bc}: {info['matvecs']} mv ({info['matvecs_f32']} f32), err {e:.2e}")
        assert info["status"] == 0, info
        assert e <= 1e-8


def test_batch_statuses_and_errors():
    require_gpu()
    import torch
    from paper_2606_21410_amd._lib import ChebError
    from paper_2606_21410_amd.api import SolveOptions
    systems = _systems([17], 20)
    us, infos = _batch_solve(systems, "f64", SolveOptions(rtol=1e-14, maxiter=5))
    assert all(i["status"] == 1 for i in infos)
    assert all(np.all(np.isfinite(u)) for u in us)
    bad = list(systems)
    K = bad[1][2].copy()
    K[3, 3, 3] = -1.0
    bad[1] = (bad[1][0], bad[1][1], K, bad[1][3], bad[1][4])
    with pytest.raises(ChebError) as ei:
        _batch_solve(bad, "f64", SolveOptions(rtol=1e-10))
    assert ei.value.code == -3


def test_homogenize_vs_oracle():
    """Apparent conductivity tensors of two microstructures (17^3, 33^3) from
    one batch of six systems, against the oracle's solves and Clenshaw-Curtis
    flux averages; constant K gives K_app = K_c I."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions, homogenize
    Ks = []
    for i, n in enumerate((17, 33)):
        grid = W.Grid((n, n, n), BOX[0], BOX[1], W.MIXED_X_BC)
        Ks.append(W.lognormal_conductivity(grid, 1004 + 30 + i, 1.0, 0.2))
    Ks.append(np.full((9, 9, 9), 2.5))
    Kapp, infos, _ = homogenize([to_dev(K, torch.float64) for K in Ks], precision="mixed",
                                opts=SolveOptions(rtol=1e-12, maxiter=4000, precond=True))
    for K, Ka in zip(Ks, Kapp):
        n = K.shape
        ref = np.zeros((3, 3))
        for a in range(3):
            bc = W.load_case_bc(a)
            G = O.Grid3(n, BOX[0], BOX[1], bc)
            U = O.solve(G, K, np.zeros(n), W.load_case_faces(W.Grid(n, BOX[0], BOX[1], bc), a), tol=1e-14)
            ref[:, a] = O.flux_average(G, K, U) / 1.0
        log(f"K_app n={n[0]}: {np.array(Ka)} ref {ref}")
        np.testing.assert_allclose(np.array(Ka), ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())
    np.testing.assert_allclose(np.array(Kapp[2]), 2.5 * np.eye(3), atol=1e-10)


def test_batch_autotuned_tile_shapes():
    """The batch times both tile shapes of every matrix-core size group on its
    first solve in each precision and keeps the faster; the choice is reported
    and the solves with it match the oracle (the other tests run with it too)."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import Batch, SolveOptions
    systems = _systems([17, 33], 40)
    d = lambda a: to_dev(a, torch.float64)
    B = Batch([(n, BOX[0], BOX[1], bc) for n, bc, _, _, _ in systems], "mixed")
    assert all(t["shape"] == -1 for t in B.tile_shapes("f64"))
    us, infos = B.solve([d(s[2]) for s in systems], [d(s[3]) for s in systems], [d(s[4]) for s in systems],
                        opts=SolveOptions(rtol=1e-11, maxiter=4000, precond=True))
    for prec in ("f64", "f32"):
        shapes = B.tile_shapes(prec)
        log(f"tuned {prec}: {shapes}")
        assert sorted(t["n"] for t in shapes) == [17, 33]
        for t in shapes:
            assert t["shape"] in (0, 1) and t["us_shape0"] > 0 and t["us_shape1"] > 0
            best = min(t["us_shape0"], t["us_shape1"])
            assert (t["us_shape0"], t["us_shape1"])[t["shape"]] == best
    for (n, bc, K, f, g), u, info in zip(systems, us, infos):
        assert info["status"] == 0
        ref = O.solve(O.Grid3(n, BOX[0], BOX[1], bc), K, f, g, tol=1e-14)
        assert rel_l2(to_host(u), ref) <= 1e-8
