"""The 1-D and 2-D front-ends (api.solve_1d, api.solve_2d): problems of lower
dimension solved by the 3-D kernels on a grid extended by axes of three nodes
with zero-flux faces and data constant along them.  Checked against the
oracle (the paper's 1-D example; the 3-D oracle on the embedded 2-D arrays)
and against analytic solutions."""
import math

import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [16, 32])
def test_solve_1d_paper_example(N):
    """u'' = exp(4x) on [-1, 1], u(+-1) = 0 (Section 3.1): the front-end's
    solution equals the oracle's 1-D collocation solution and, at N = 32, the
    exact solution to the spectral error of that N."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions, solve_1d
    x, f, ue = W.poisson1d_exp4x(N)
    u, info = solve_1d(torch.ones(N + 1, dtype=torch.float64), torch.from_numpy(f), [0.0, 0.0],
                       opts=SolveOptions(rtol=1e-14, maxiter=2000, precond=True))
    u = to_host(u)
    uo = O.solve_1d_dirichlet(N, f)
    e_or, e_ex = rel_l2(u, uo), np.max(np.abs(u - ue))
    log(f"1-D N={N}: {info['matvecs']} matvecs, rel diff to oracle {e_or:.2e}, max error to exact {e_ex:.2e}")
    assert info["status"] == 0
    assert e_or <= 1e-11
    if N == 32:
        assert e_ex <= 1e-12


def _manufactured_2d(n0, n1):
    """u = cos(pi x / 2) e^y on (0,1) x (0,2), K = 1 + 0.3 x + 0.2 y^2,
    f = div(K grad u); Dirichlet x faces, Neumann y faces (outward u_y)."""
    x = W.cgl_coords(n0, 0.0, 1.0)
    y = W.cgl_coords(n1, 0.0, 2.0)
    X, Y = np.meshgrid(x, y, indexing="ij")
    c, s, e = np.cos(math.pi * X / 2), np.sin(math.pi * X / 2), np.exp(Y)
    u = c * e
    K = 1.0 + 0.3 * X + 0.2 * Y ** 2
    ux, uy = -math.pi / 2 * s * e, c * e
    lap = (1.0 - (math.pi / 2) ** 2) * u
    f = K * lap + 0.3 * ux + 0.4 * Y * uy
    g = [u[0, :], u[-1, :], -uy[:, 0], uy[:, -1]]
    return X, Y, u, K, f, g


def test_solve_2d_manufactured():
    """Variable K, Dirichlet x faces, Neumann y faces: spectral accuracy to the
    analytic solution."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions, solve_2d
    bc = (W.DIRICHLET, W.DIRICHLET, W.NEUMANN, W.NEUMANN)
    errs = {}
    for n0, n1 in ((9, 11), (17, 21)):
        X, Y, ue, K, f, g = _manufactured_2d(n0, n1)
        u, info = solve_2d(torch.from_numpy(K), torch.from_numpy(f), [torch.from_numpy(np.ascontiguousarray(v)) for v in g],
                           lo=(0.0, 0.0), hi=(1.0, 2.0), bc=bc, opts=SolveOptions(rtol=1e-14, maxiter=5000, precond=True))
        errs[n0] = np.max(np.abs(to_host(u) - ue)) / np.max(np.abs(ue))
        log(f"2-D {n0}x{n1}: {info['matvecs']} matvecs, max rel error {errs[n0]:.2e}")
        assert info["status"] == 0
    assert errs[17] <= 1e-10
    assert errs[17] < 1e-2 * errs[9]


def test_solve_2d_matches_3d_oracle_on_embedding():
    """The front-end solves exactly the embedded 3-D collocation system: its
    result equals the 3-D oracle's solution of the extended arrays, which is
    constant along the added axis."""
    require_gpu()
    import torch
    from paper_2606_21410_amd.api import SolveOptions, solve_2d
    n0, n1 = 9, 11
    X, Y, ue, K, f, g = _manufactured_2d(n0, n1)
    bc = (W.DIRICHLET, W.DIRICHLET, W.NEUMANN, W.NEUMANN)
    u, info = solve_2d(torch.from_numpy(K), torch.from_numpy(f), [torch.from_numpy(np.ascontiguousarray(v)) for v in g],
                       lo=(0.0, 0.0), hi=(1.0, 2.0), bc=bc, opts=SolveOptions(rtol=1e-14, maxiter=5000, precond=True))
    G = O.Grid3((n0, n1, 3), (0.0, 0.0, 0.0), (1.0, 2.0, 1.0), bc + (W.NEUMANN, W.NEUMANN))
    gw = W.Grid(G.n, G.lo, G.hi, G.bc)
    faces = [np.repeat(g[0][:, None], 3, 1), np.repeat(g[1][:, None], 3, 1),
             np.repeat(g[2][:, None], 3, 1), np.repeat(g[3][:, None], 3, 1),
             np.zeros(gw.face_shape(4)), np.zeros(gw.face_shape(5))]
    U3 = O.solve_dense(G, np.repeat(K[:, :, None], 3, 2), np.repeat(f[:, :, None], 3, 2), W.pack_faces(faces))
    log(f"embedding: oracle z-variation {np.max(np.abs(U3 - U3[:, :, :1])):.1e}")
    assert np.max(np.abs(U3 - U3[:, :, :1])) <= 1e-12 * np.max(np.abs(U3))
    assert rel_l2(to_host(u), U3[:, :, 0]) <= 1e-11


@pytest.mark.parametrize("sig", [(0.5, 2.0), (3.0, 0.0)])
def test_solve_1d_robin_polynomial(sig):
    """u = x^3 + x on [-1, 1] with K = 1 (u'' = 6x) and Robin rows at both ends
    (-u'(-1) + s_lo u(-1) = g_lo, u'(1) + s_hi u(1) = g_hi): a cubic is exact
    at any N >= 3, so the collocation solution is the cubic itself."""
    require_gpu()
    import torch
    from paper_2606_21410_amd import _lib as L
    from paper_2606_21410_amd.api import SolveOptions, solve_1d
    N = 12
    x = W.cgl_coords(N + 1, -1.0, 1.0)
    ue = x ** 3 + x
    glo = -(3.0 + 1.0) + sig[0] * (-2.0)
    ghi = (3.0 + 1.0) + sig[1] * 2.0
    u, info = solve_1d(torch.ones(N + 1, dtype=torch.float64), torch.from_numpy(6.0 * x), [glo, ghi],
                       bc=(L.CHEB_NEUMANN, L.CHEB_NEUMANN), robin=sig,
                       opts=SolveOptions(rtol=1e-14, maxiter=2000, precond=True))
    err = np.max(np.abs(to_host(u) - ue))
    log(f"1-D Robin {sig}: {info['matvecs']} matvecs, max error {err:.2e}")
    assert info["status"] == 0 and err <= 1e-12
