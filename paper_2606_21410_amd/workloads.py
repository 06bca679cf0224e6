"""Seeded synthetic inputs for the Chebyshev-collocation diffusion solver.

This module only *produces inputs*: sampling coordinates, analytic manufactured
fields and their boundary data, random two-phase microstructures and log-normal
conductivity fields, random test vectors.  It contains none of the solver's
arithmetic (no differentiation, no transforms, no boundary elimination), so the
GPU path and the CPU oracle can both consume its arrays without sharing method
code.  Every generator takes an explicit seed.

Conventions shared by both sides of the boundary:
  * arrays are C-contiguous ``[i][j][k]`` with ``i`` along x (slowest) and ``k``
    along z (fastest);
  * node coordinates are the Chebyshev-Gauss-Lobatto points in *ascending*
    order, affinely mapped to ``[lo, hi]`` (Section 2.2, affine map);
  * faces are numbered x_lo, x_hi, y_lo, y_hi, z_lo, z_hi; a face array of axis
    ``a`` is indexed by the two remaining axes in increasing order;
  * Neumann data are the outward normal derivative du/dn.

Workload recipes (sphere microstructure, log-normal fields) follow the
configurations of the paper's heterogeneous examples (Section 3.3) with the
sizes stated in the accompanying design notes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DIRICHLET = 0
NEUMANN = 1
FACE_NAMES = ("x_lo", "x_hi", "y_lo", "y_hi", "z_lo", "z_hi")


def rng(*seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(seed)))


def cgl_coords(n: int, lo: float, hi: float) -> np.ndarray:
    """Ascending Chebyshev-Gauss-Lobatto coordinates on [lo, hi] (n = N+1 points).

    Uses -cos(pi j/N) = sin(pi (2j-N)/(2N)) so the set is exactly symmetric.
    """
    N = n - 1
    j = np.arange(n, dtype=np.float64)
    t = np.sin(np.pi * (2.0 * j - N) / (2.0 * N))
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * t


@dataclass
class Grid:
    n: tuple[int, int, int]
    lo: tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: tuple[float, float, float] = (1.0, 1.0, 1.0)
    bc: tuple[int, int, int, int, int, int] = (DIRICHLET,) * 6
    # sigma of the Neumann row du/dn + sigma u = g per face (0: plain Neumann)
    robin: tuple[float, float, float, float, float, float] = (0.0,) * 6
    # per-node part of sigma (packed faces like g, added to robin[f]); None: none
    robin_nodes: np.ndarray | None = None

    def coords(self):
        return [cgl_coords(self.n[a], self.lo[a], self.hi[a]) for a in range(3)]

    def mesh(self):
        x, y, z = self.coords()
        return np.meshgrid(x, y, z, indexing="ij")

    def face_shape(self, f: int):
        a = f // 2
        return tuple(self.n[b] for b in range(3) if b != a)

    def face_size(self, f: int):
        s = self.face_shape(f)
        return s[0] * s[1]


def pack_faces(faces) -> np.ndarray:
    """Concatenate six face arrays (x_lo..z_hi) into the flat g_faces buffer."""
    return np.concatenate([np.ascontiguousarray(f, dtype=np.float64).ravel() for f in faces])


def unpack_faces(grid: Grid, g: np.ndarray):
    out, off = [], 0
    for f in range(6):
        s = grid.face_shape(f)
        m = s[0] * s[1]
        out.append(np.asarray(g[off:off + m]).reshape(s))
        off += m
    return out


def face_coords(grid: Grid, f: int):
    """Meshgrid of the physical coordinates of face f (2-D arrays)."""
    c = grid.coords()
    a, side = divmod(f, 2)
    val = grid.lo[a] if side == 0 else grid.hi[a]
    others = [b for b in range(3) if b != a]
    P, Q = np.meshgrid(c[others[0]], c[others[1]], indexing="ij")
    xyz = [None, None, None]
    xyz[a] = np.full(P.shape, val)
    xyz[others[0]] = P
    xyz[others[1]] = Q
    return xyz


# ----------------------------------------------------------------------------
# Manufactured problems (analytic fields, their sources and face data)
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    grid: Grid
    K: np.ndarray
    f: np.ndarray
    g: np.ndarray          # packed faces
    u_exact: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def _faces_from(grid: Grid, value_fn, grad_fn):
    faces = []
    for f in range(6):
        a, side = divmod(f, 2)
        X, Y, Z = face_coords(grid, f)
        if grid.bc[f] == DIRICHLET:
            faces.append(value_fn(X, Y, Z))
        else:
            sgn = -1.0 if side == 0 else 1.0
            data = sgn * grad_fn(X, Y, Z)[a]
            sig = grid.robin[f]
            if grid.robin_nodes is not None:
                sig = sig + unpack_faces(grid, grid.robin_nodes)[f]
            if np.any(sig != 0.0):
                data = data + sig * value_fn(X, Y, Z)
            faces.append(data)
    return pack_faces(faces)


def random_robin_nodes(grid: Grid, seed: int, lo: float = 0.2, hi: float = 2.0) -> np.ndarray:
    """Per-node Robin coefficients (packed faces): uniform in [lo, hi] on the
    Neumann faces, 0 on the Dirichlet faces."""
    r = rng(seed)
    faces = []
    for f in range(6):
        s = grid.face_shape(f)
        faces.append(r.uniform(lo, hi, size=s) if grid.bc[f] == NEUMANN else np.zeros(s))
    return pack_faces(faces)


def manufactured_sincos(n: int = 17, robin=(0.0,) * 6) -> Problem:
    """Homogeneous Poisson on [-1,1]^3: u = sin(pi x) cos(pi y) exp(z), K = 1.

    Dirichlet on the x faces, Neumann (outward du/dn, plus robin[f] u where
    robin[f] is nonzero) on the y and z faces.
    """
    grid = Grid((n, n, n), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0),
                (DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN), tuple(float(v) for v in robin))
    pi = math.pi

    def u(X, Y, Z):
        return np.sin(pi * X) * np.cos(pi * Y) * np.exp(Z)

    def grad(X, Y, Z):
        return (pi * np.cos(pi * X) * np.cos(pi * Y) * np.exp(Z),
                -pi * np.sin(pi * X) * np.sin(pi * Y) * np.exp(Z),
                np.sin(pi * X) * np.cos(pi * Y) * np.exp(Z))

    X, Y, Z = grid.mesh()
    ue = u(X, Y, Z)
    f = (1.0 - 2.0 * pi * pi) * ue
    return Problem(grid, np.ones_like(ue), f, _faces_from(grid, u, grad), ue,
                   {"name": "sincos-poisson"})


def manufactured_paper3d(n: int) -> Problem:
    """The paper's 3-D Poisson example on (0,1)^3 (Section 3.2):
    u = exp(x+y+z) + x^2 + 2y - z^2, Laplacian 3 exp(x+y+z); Dirichlet on
    x=0, x=1, z=0 and Neumann on y=0, y=1, z=1."""
    grid = Grid((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                (DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, DIRICHLET, NEUMANN))

    def u(X, Y, Z):
        return np.exp(X + Y + Z) + X ** 2 + 2 * Y - Z ** 2

    def grad(X, Y, Z):
        e = np.exp(X + Y + Z)
        return (e + 2 * X, e + 2.0, e - 2 * Z)

    X, Y, Z = grid.mesh()
    ue = u(X, Y, Z)
    f = 3.0 * np.exp(X + Y + Z)
    return Problem(grid, np.ones_like(ue), f, _faces_from(grid, u, grad), ue,
                   {"name": "paper-3d-poisson"})


def thermal_nonlinear(n: int, alpha: float = 0.5, flux_form: bool = False) -> Problem:
    """The nonlinear thermal example of Section 3.4 on (0,1)^3, written for
    div(k(T) grad T) = f with k(T) = K0 / (1 + alpha T), K0 = 1:
    Phi = sin(pi x) sin(pi y) sin(pi z), T = (exp(alpha Phi) - 1) / alpha, so
    k(T) grad T = grad Phi and f = Laplacian(Phi) = -3 pi^2 Phi.  Dirichlet on
    x=0 and y=0; on x=1, y=1, z=0 and z=1 the prescribed outward flux
    h = k(T) dT/dn = dPhi/dn.

    flux_form False: the Neumann rows read dT/dn = h.  Phi = 0 on every face,
    so there T = 0, k = 1 and the exact solution satisfies them.
    flux_form True: the rows are the flux condition itself, k(T) dT/dn = h.
    With 1/k = (1 + alpha T)/K0 it is linear in T: dT/dn - (alpha h/K0) T = h/K0,
    a Robin row with the per-node coefficient -alpha h/K0 (grid.robin_nodes)
    and data h/K0 (the same data here, K0 = 1)."""
    grid = Grid((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                (DIRICHLET, NEUMANN, DIRICHLET, NEUMANN, NEUMANN, NEUMANN))
    pi = math.pi

    def phi(X, Y, Z):
        return np.sin(pi * X) * np.sin(pi * Y) * np.sin(pi * Z)

    def u(X, Y, Z):
        return np.expm1(alpha * phi(X, Y, Z)) / alpha

    def grad(X, Y, Z):
        e = np.exp(alpha * phi(X, Y, Z))
        sx, sy, sz = np.sin(pi * X), np.sin(pi * Y), np.sin(pi * Z)
        return (e * pi * np.cos(pi * X) * sy * sz,
                e * pi * sx * np.cos(pi * Y) * sz,
                e * pi * sx * sy * np.cos(pi * Z))

    X, Y, Z = grid.mesh()
    ue = u(X, Y, Z)
    f = -3.0 * pi * pi * phi(X, Y, Z)
    g = _faces_from(grid, u, grad)
    if flux_form:
        # sigma = -alpha h / K0 on the Neumann faces (K0 = 1); T = 0 there, so
        # the data h/K0 of the Robin rows is g as formed above
        grid.robin_nodes = pack_faces([-alpha * F if grid.bc[f_] == NEUMANN else np.zeros_like(F)
                                       for f_, F in enumerate(unpack_faces(grid, g))])
    return Problem(grid, np.ones_like(ue), f, g, ue,
                   {"name": "thermal-nonlinear-flux" if flux_form else "thermal-nonlinear", "alpha": alpha})


def manufactured_polynomial(n: int, bc, seed: int = 7, deg_u: int = 3,
                            lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), robin=(0.0,) * 6,
                            robin_nodes=None) -> Problem:
    """Random separable-sum polynomial u with polynomial K (degree 1); the
    discrete operator is exact for it when deg u + deg K - 1 <= N.  Neumann faces
    with a nonzero coefficient (robin[f] plus the face's entries of the packed
    per-node array robin_nodes) carry the data du/dn + sigma u."""
    r = rng(seed)
    grid = Grid((n, n, n), tuple(lo), tuple(hi), tuple(bc), tuple(float(v) for v in robin),
                None if robin_nodes is None else np.asarray(robin_nodes, dtype=np.float64))
    cu = r.normal(size=(deg_u + 1, deg_u + 1, deg_u + 1)) / 4
    ck = r.uniform(0.1, 0.3, size=3)

    def u(X, Y, Z):
        s = np.zeros_like(X)
        for p in range(deg_u + 1):
            for q in range(deg_u + 1 - p):
                for s_ in range(deg_u + 1 - p - q):
                    s = s + cu[p, q, s_] * X ** p * Y ** q * Z ** s_
        return s

    def grad(X, Y, Z):
        gx = np.zeros_like(X); gy = np.zeros_like(X); gz = np.zeros_like(X)
        for p in range(deg_u + 1):
            for q in range(deg_u + 1 - p):
                for s_ in range(deg_u + 1 - p - q):
                    c = cu[p, q, s_]
                    if p: gx = gx + c * p * X ** (p - 1) * Y ** q * Z ** s_
                    if q: gy = gy + c * q * X ** p * Y ** (q - 1) * Z ** s_
                    if s_: gz = gz + c * s_ * X ** p * Y ** q * Z ** (s_ - 1)
        return gx, gy, gz

    def kfun(X, Y, Z):
        return 1.0 + ck[0] * X + ck[1] * Y + ck[2] * Z

    def lap_flux(X, Y, Z):
        # div(K grad u) = K lap u + grad K . grad u, evaluated analytically
        gx, gy, gz = grad(X, Y, Z)
        lap = np.zeros_like(X)
        for p in range(deg_u + 1):
            for q in range(deg_u + 1 - p):
                for s_ in range(deg_u + 1 - p - q):
                    c = cu[p, q, s_]
                    if p >= 2: lap = lap + c * p * (p - 1) * X ** (p - 2) * Y ** q * Z ** s_
                    if q >= 2: lap = lap + c * q * (q - 1) * X ** p * Y ** (q - 2) * Z ** s_
                    if s_ >= 2: lap = lap + c * s_ * (s_ - 1) * X ** p * Y ** q * Z ** (s_ - 2)
        return kfun(X, Y, Z) * lap + ck[0] * gx + ck[1] * gy + ck[2] * gz

    X, Y, Z = grid.mesh()
    return Problem(grid, kfun(X, Y, Z), lap_flux(X, Y, Z), _faces_from(grid, u, grad),
                   u(X, Y, Z), {"name": "polynomial"})


def poisson1d_exp4x(N: int):
    """The paper's 1-D example (Section 3.1): u'' = exp(4x) on [-1,1],
    u(-1) = u(1) = 0, exact u = (exp(4x) - sinh(4) x - cosh(4)) / 16."""
    x = cgl_coords(N + 1, -1.0, 1.0)
    f = np.exp(4 * x)
    ue = (np.exp(4 * x) - math.sinh(4.0) * x - math.cosh(4.0)) / 16.0
    return x, f, ue


# ----------------------------------------------------------------------------
# Heterogeneous microstructures
# ----------------------------------------------------------------------------

def rsa_spheres(seed: int, radius: float = 0.15, volume_fraction: float = 0.2,
                lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_tries: int = 200000):
    """Random sequential addition of non-overlapping spheres: centres uniform in
    the box, a candidate is rejected when closer than 2R to an accepted centre;
    spheres may be clipped by the faces.  Count = round(vf * vol / (4 pi R^3/3))."""
    r = rng(seed)
    vol = float(np.prod(np.subtract(hi, lo)))
    count = int(round(volume_fraction * vol / (4.0 / 3.0 * math.pi * radius ** 3)))
    centres = []
    tries = 0
    while len(centres) < count and tries < max_tries:
        c = r.uniform(lo, hi)
        tries += 1
        if all(np.sum((c - p) ** 2) >= (2 * radius) ** 2 for p in centres):
            centres.append(c)
    if len(centres) < count:
        raise RuntimeError("RSA could not place all spheres")
    return np.array(centres)


def sphere_conductivity(grid: Grid, centres: np.ndarray, radius: float, k_inc: float,
                        k_mat: float = 1.0, width: float | None = None,
                        n_finest: int | None = None) -> np.ndarray:
    """K = K_m + (K_i - K_m) max_s chi_s, chi_s = (1 - tanh((d_s - R)/w))/2 with
    w = 2 h and h = L / N of the finest grid of the configuration."""
    if width is None:
        nf = n_finest if n_finest is not None else grid.n[0]
        width = 2.0 * (grid.hi[0] - grid.lo[0]) / (nf - 1)
    xs = grid.coords()
    chi = np.zeros(grid.n)
    # tanh(t) rounds to 1 in FP64 for t > 19.1, so chi_s is exactly 0 farther
    # than R + 20 w from the centre: each sphere only touches the nodes of its
    # bounding box (the same values as evaluating it everywhere)
    reach = radius + 20.0 * width
    for c in centres:
        sl = []
        for a in range(3):
            i0 = int(np.searchsorted(xs[a], c[a] - reach, side="left"))
            i1 = int(np.searchsorted(xs[a], c[a] + reach, side="right"))
            sl.append(slice(i0, i1))
        if any(s_.stop <= s_.start for s_ in sl):
            continue
        dx = (xs[0][sl[0]] - c[0]) ** 2
        dy = (xs[1][sl[1]] - c[1]) ** 2
        dz = (xs[2][sl[2]] - c[2]) ** 2
        d = np.sqrt(dx[:, None, None] + dy[None, :, None] + dz[None, None, :])
        blk = chi[sl[0], sl[1], sl[2]]
        np.maximum(blk, 0.5 * (1.0 - np.tanh((d - radius) / width)), out=blk)
    return k_mat + (k_inc - k_mat) * chi


def gaussian_field_rff(grid: Grid, seed: int, corr_len: float, n_features: int = 2048,
                       chunk: int = 16) -> np.ndarray:
    """Zero-mean unit-variance Gaussian field with covariance exp(-r^2/(2 l^2)),
    by random Fourier features: g(x) = sqrt(2/M) sum_m cos(w_m . x + phi_m),
    w ~ N(0, I/l^2), phi ~ U(0, 2 pi).  Grid-independent for a given seed (an
    int, or a tuple such as (1004, s) for structure s of a family)."""
    r = rng(*seed) if isinstance(seed, tuple) else rng(seed)
    w = r.normal(size=(n_features, 3)) / corr_len
    phi = r.uniform(0.0, 2.0 * math.pi, size=n_features)
    x, y, z = grid.coords()
    ex = np.exp(1j * (np.outer(w[:, 0], x) + phi[:, None]))     # (M, nx)
    ey = np.exp(1j * np.outer(w[:, 1], y))                      # (M, ny)
    ez = np.exp(1j * np.outer(w[:, 2], z))                      # (M, nz)
    out = np.empty(grid.n, dtype=np.float64)
    for i0 in range(0, grid.n[0], chunk):
        i1 = min(grid.n[0], i0 + chunk)
        t = ex[:, i0:i1, None] * ey[:, None, :]                 # (M, ci, ny)
        t = t.reshape(n_features, -1).T                          # (ci*ny, M)
        out[i0:i1] = np.real(t @ ez).reshape(i1 - i0, grid.n[1], grid.n[2])
    return out * math.sqrt(2.0 / n_features)


def lognormal_conductivity(grid: Grid, seed: int, sigma: float = 1.0,
                           corr_len: float = 0.2) -> np.ndarray:
    return np.exp(sigma * gaussian_field_rff(grid, seed, corr_len))


# ----------------------------------------------------------------------------
# Configurations
# ----------------------------------------------------------------------------

def dirichlet_x_faces(grid: Grid, left: float, right: float) -> np.ndarray:
    """u = left on x_lo, u = right on x_hi, zero flux on the other faces."""
    faces = []
    for f in range(6):
        s = grid.face_shape(f)
        if f == 0:
            faces.append(np.full(s, left))
        elif f == 1:
            faces.append(np.full(s, right))
        else:
            faces.append(np.zeros(s))
    return pack_faces(faces)


def load_case_faces(grid: Grid, axis: int) -> np.ndarray:
    """Unit mean gradient along `axis`: u = 0 on the lo face, u = 1 on the hi face,
    zero flux elsewhere (the other four faces are Neumann)."""
    faces = []
    for f in range(6):
        s = grid.face_shape(f)
        faces.append(np.full(s, 1.0) if f == 2 * axis + 1 else np.zeros(s))
    return pack_faces(faces)


def load_case_bc(axis: int):
    bc = [NEUMANN] * 6
    bc[2 * axis] = DIRICHLET
    bc[2 * axis + 1] = DIRICHLET
    return tuple(bc)


MIXED_X_BC = (DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN)


def two_phase_problem(n: int, seed: int = 1002, volume_fraction: float = 0.2,
                      contrast: float = 10.0, n_finest: int | None = None,
                      radius: float = 0.15) -> Problem:
    """Seeded spherical inclusions in (0,1)^3, u = -1 at x=0, +1 at x=1, zero flux
    elsewhere, f = 0 (heterogeneous two-phase workload)."""
    grid = Grid((n, n, n), (0.0,) * 3, (1.0,) * 3, MIXED_X_BC)
    centres = rsa_spheres(seed, radius, volume_fraction)
    K = sphere_conductivity(grid, centres, radius, contrast, 1.0, n_finest=n_finest or n)
    f = np.zeros(grid.n)
    return Problem(grid, K, f, dirichlet_x_faces(grid, -1.0, 1.0), None,
                   {"name": "two-phase", "seed": seed, "vf": volume_fraction,
                    "contrast": contrast, "spheres": len(centres)})


def maxwell_keff(phi: float, k_inc: float, k_mat: float = 1.0) -> float:
    """Maxwell's dilute estimate of the effective conductivity of spheres of
    conductivity k_inc at volume fraction phi in a matrix k_mat (Section 3.3)."""
    d = k_inc - k_mat
    return k_mat * (2.0 * k_mat + k_inc + 2.0 * phi * d) / (2.0 * k_mat + k_inc - phi * d)


def inclusion_conductivity(grid: Grid, contrast: float, layout: str = "center",
                           radius: float = 0.2, k_mat: float = 1.0) -> np.ndarray:
    """Two-phase field sampled sharply at the nodes (Section 3.3): k_mat * contrast
    inside the inclusion, k_mat outside.  layout 'center': one sphere of radius R
    at the box centre; 'corner': the sphere's eighths at the eight box corners
    (the same volume, so the same volume fraction 4 pi R^3 / 3 in the unit box)."""
    X, Y, Z = grid.mesh()
    lo, hi = np.array(grid.lo), np.array(grid.hi)
    if layout == "center":
        c = 0.5 * (lo + hi)
        inside = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= radius ** 2
    elif layout == "corner":
        inside = np.zeros(grid.n, dtype=bool)
        for cx in (lo[0], hi[0]):
            for cy in (lo[1], hi[1]):
                for cz in (lo[2], hi[2]):
                    inside |= (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 <= radius ** 2
    else:
        raise ValueError("layout must be 'center' or 'corner'")
    return np.where(inside, k_mat * contrast, k_mat)


def inclusion_problem(n: int, contrast: float, layout: str = "center", radius: float = 0.2,
                      g: float = 1.0) -> Problem:
    """The spherical-inclusion homogenisation problem of Section 3.3 in (0,1)^3:
    u = -g at x = 0, u = +g at x = 1, zero flux elsewhere, f = 0; the imposed
    mean gradient is G = 2 g / L_x."""
    grid = Grid((n, n, n), (0.0,) * 3, (1.0,) * 3, MIXED_X_BC)
    K = inclusion_conductivity(grid, contrast, layout, radius)
    f = np.zeros(grid.n)
    phi = 4.0 / 3.0 * math.pi * radius ** 3
    return Problem(grid, K, f, dirichlet_x_faces(grid, -g, g), None,
                   {"name": "inclusion", "layout": layout, "contrast": contrast, "radius": radius,
                    "phi": phi, "G": 2.0 * g / (grid.hi[0] - grid.lo[0])})


def random_field(shape, seed: int, dtype=np.float64) -> np.ndarray:
    return rng(seed).standard_normal(size=shape).astype(dtype)


def random_conductivity(shape, seed: int, sigma: float = 0.5) -> np.ndarray:
    """Point-wise log-normal conductivity (iid), a rough stress input for parity."""
    return np.exp(sigma * rng(seed).standard_normal(size=shape))


def random_faces(grid: Grid, seed: int) -> np.ndarray:
    r = rng(seed)
    return pack_faces([r.standard_normal(grid.face_shape(f)) for f in range(6)])
