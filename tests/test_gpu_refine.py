"""Hierarchical refinement with its stopping rule (cheb_refine; Section 2.3.3,
Algorithm 4): the refinement indicator of each solved level against the
oracle's barycentric prolongation of the GPU's own level solutions, the level
at which the refinement stops for a given tolerance, and the levels past it
being the prolongation alone."""
import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W
from tests.gpu_util import log, rel_l2, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _levels(problems, prec="f64"):
    from paper_2606_21410_amd.api import Plan
    plans = [Plan(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc, prec) for P in problems]
    import torch
    d = lambda a: to_dev(a, torch.float64)
    return plans, [d(P.K) for P in problems], [d(P.f) for P in problems], [d(P.g) for P in problems]


@pytest.mark.parametrize("make,ns,opts_kw", [
    (lambda n: W.manufactured_sincos(n), (9, 17, 33, 65), dict(rtol=1e-12, precond=True)),
    (lambda n: W.two_phase_problem(n, seed=1002, n_finest=129), (17, 33, 65, 129), dict(rtol=1e-12, precond=True)),
])
def test_refinement_stop(make, ns, opts_kw):
    require_gpu()
    from paper_2606_21410_amd.api import SolveOptions, prolong, refine
    problems = [make(n) for n in ns]
    plans, Ks, fs, gs = _levels(problems)
    opts = SolveOptions(maxiter=5000, **opts_kw)
    # tol = 0: every level is solved; its indicators set the expected stop
    log(f"refine {ns}: every level")
    us, e_full, solved, infos = refine(plans, Ks, fs, gs, 0.0, opts)
    assert solved == [1] * len(ns)
    uh = [to_host(u) for u in us]
    for l in range(1, len(ns)):
        G = problems[l].grid
        ref = O.e_ref(uh[l], O.prolong(uh[l - 1], G.lo, G.hi, G.n))
        log(f"  level {ns[l]}: e_ref {e_full[l]:.3e} (oracle prolongation {ref:.3e}), {infos[l]['matvecs']} matvecs")
        assert abs(e_full[l] - ref) <= 1e-10 * max(ref, 1e-300) + 1e-15
        assert infos[l]["status"] == 0
    assert np.isnan(e_full[0])
    # a tolerance between the indicators of levels 1 and 2: levels 0..2 are
    # solved, the finer ones are the prolongation of level 2
    tol = float(np.sqrt(e_full[1] * e_full[2]))
    assert e_full[2] <= tol < e_full[1]
    log(f"refine {ns}: tol {tol:.3e}")
    us2, e2, solved2, infos2 = refine(plans, Ks, fs, gs, tol, opts)
    assert solved2 == [1, 1, 1] + [0] * (len(ns) - 3)
    assert e2[1] == e_full[1] and e2[2] == e_full[2]
    for l in range(3, len(ns)):
        assert np.isnan(e2[l]) and infos2[l]["matvecs"] == 0
        want, _ = prolong(plans[l - 1], plans[l], us2[l - 1])
        np.testing.assert_array_equal(to_host(us2[l]), to_host(want))
        # the prolongation alone stays within the indicator's size of the solve
        d = rel_l2(to_host(us2[l]), uh[l])
        log(f"  level {ns[l]} interpolated: {d:.3e} from the solved level")
        assert d <= 10.0 * tol


def test_refine_rejects_bad_levels():
    require_gpu()
    import torch
    from paper_2606_21410_amd._lib import ChebError
    from paper_2606_21410_amd.api import Plan, SolveOptions, refine
    a = W.manufactured_sincos(17)
    b = W.manufactured_sincos(9)
    plans, Ks, fs, gs = _levels([a, b])
    with pytest.raises(ChebError) as ei:
        refine(plans, Ks, fs, gs, 1e-6, SolveOptions())
    assert ei.value.code == -1
