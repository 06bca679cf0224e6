"""The spherical-inclusion workload of Section 3.3 (centred sphere or corner
eighth-spheres, contrast sweep, Maxwell comparison): CPU pins for the Maxwell
estimate (oracle and the workload module's copy used by the benchmark), the
inclusion sampler, and symmetries of the oracle solution."""
import math

import numpy as np
import pytest

from oracle import cheb_oracle as O
from paper_2606_21410_amd import workloads as W

PHI = 4.0 / 3.0 * math.pi * 0.2 ** 3  # the paper's phi = 0.03351


def _hashin_shtrikman_matrix_ref(phi, ki, km):
    """Hashin-Shtrikman bound with the matrix as reference medium (3D):
    km + phi / (1/(ki - km) + (1 - phi)/(3 km)); Maxwell's dilute formula is
    algebraically the same expression."""
    return km + phi / (1.0 / (ki - km) + (1.0 - phi) / (3.0 * km))


@pytest.mark.parametrize("fn", [O.maxwell_estimate, W.maxwell_keff])
def test_maxwell_closed_forms(fn):
    km = 1.7
    for phi in (1e-3, PHI, 0.2, 0.45):
        for ki in (1e-4, 0.3, 2.5, 10.0, 1e4):
            assert abs(fn(phi, ki, km) - _hashin_shtrikman_matrix_ref(phi, ki, km)) <= 1e-13 * km
        # perfectly conducting and insulating spheres
        assert abs(fn(phi, 1e14, km) - km * (1 + 2 * phi) / (1 - phi)) <= 1e-10 * km
        assert abs(fn(phi, 0.0, km) - km * (2 - 2 * phi) / (2 + phi)) <= 1e-13 * km
    # no inclusion, or no contrast
    assert fn(0.0, 10.0, km) == pytest.approx(km, abs=1e-15)
    assert fn(0.3, km, km) == pytest.approx(km, abs=1e-15)
    # dilute slope dK/dphi at phi -> 0: 3 km (ki - km) / (ki + 2 km)
    for ki in (0.1, 10.0):
        h = 1e-7
        slope = (fn(h, ki, km) - km) / h
        assert abs(slope - 3 * km * (ki - km) / (ki + 2 * km)) <= 1e-5 * abs(slope)


@pytest.mark.parametrize("layout", ["center", "corner"])
def test_inclusion_volume_fraction_converges(layout):
    """The Clenshaw-Curtis volume of the sharply sampled inclusion tends to
    4 pi R^3 / 3 (both layouts hold one sphere's volume)."""
    errs = []
    for n in (33, 65, 129):
        g = W.Grid((n, n, n), (0.0,) * 3, (1.0,) * 3, W.MIXED_X_BC)
        chi = (W.inclusion_conductivity(g, 2.0, layout) > 1.5).astype(float)
        G = O.Grid3(g.n, g.lo, g.hi, g.bc)
        errs.append(abs(O.volume_average(G, chi) - PHI))
    assert errs[-1] < 0.1 * PHI
    assert errs[-1] < errs[0]


@pytest.mark.parametrize("layout", ["center", "corner"])
def test_inclusion_oracle_symmetry_and_unit_contrast(layout):
    """Both layouts are mirror-symmetric about the three mid-planes and the
    data u = -g / +g is odd in x, so the discrete solution is odd in x - 1/2
    and even in y - 1/2, z - 1/2 (the CGL nodes are symmetric).  At contrast 1
    the solution is linear and K_num = k_m exactly.  Dense direct solves, so the
    symmetry holds to rounding (times the condition number)."""
    n = 9
    for c in (1e-3, 1.0, 1e3):
        P = W.inclusion_problem(n, c, layout)
        G = O.Grid3(P.grid.n, P.grid.lo, P.grid.hi, P.grid.bc)
        U = O.solve_dense(G, P.K, P.f, P.g)
        # rounding of the direct solve grows with the condition number, which
        # the contrast multiplies
        tol = 1e-11 * max(c, 1.0 / c) * np.max(np.abs(U))
        assert np.max(np.abs(U + U[::-1, :, :])) <= tol
        assert np.max(np.abs(U - U[:, ::-1, :])) <= tol
        assert np.max(np.abs(U - U[:, :, ::-1])) <= tol
        if c == 1.0:
            assert abs(O.effective_conductivity(G, P.K, U, 0, P.meta["G"]) - 1.0) <= 1e-11
