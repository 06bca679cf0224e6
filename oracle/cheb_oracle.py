"""Plain FP64 CPU oracle for the Chebyshev-collocation diffusion solver.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path: there is no FFT, no DCT and no derivative-coefficient
recurrence here.  Everything is the plain definition, written out:

* nodal Chebyshev differentiation matrices D (Section 2, D_jm = l'_m(x_j)),
  applied along an axis with ``np.tensordot`` (Section 2, separable
  derivatives / Kronecker form);
* the collocation operator sum_a D_a (K * D_a u) at interior nodes (Algorithm 3,
  and its 3-D flux form in Section 3.3), with one boundary-condition row per
  boundary node (Section 2.3.1);
* boundary elimination x_r = G x_k + H g, reduced operator A_kk + A_kr G and
  reduced right-hand side f_k - A_kr H g (Section 2.3.1), realised as a lift of
  interior values to the full state;
* direct solves (dense LU for small grids, fast diagonalisation for constant K,
  GMRES preconditioned by fast diagonalisation otherwise);
* modal prolongation evaluated as barycentric Lagrange interpolation of the
  degree-N interpolant (Section 2.3.3: the zero-padded series *is* that
  interpolant) and the refinement indicator e_ref;
* Clenshaw-Curtis volume averages and the effective conductivity (Section 3.3);
* the adjoint of the reduced system and dL/dlog K;
* Picard (lagged-coefficient) iteration for K = K0 (1 + u^2/2);
* Newton's method for k = K0 / (1 + alpha T) (Section 3.4): residual, the
  reduced Jacobian action and the outer loop;
* Robin rows du/dn + sigma u = g with sigma per face plus a per-node part
  (Section 2.3.1's general linear row; the flux condition of Section 3.4 is
  such a row with a node-dependent sigma).

Readings of the paper that this oracle fixes (edge/corner ownership, Neumann
datum = outward du/dn, operator sign div(K grad u) = f, ascending node order)
are listed in the design notes; the GPU path implements the same readings.

Parity pins live in tests/test_oracle_*.py.  Functions whose only check is
another oracle function say "parity unpinned" in their docstring.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

DIRICHLET = 0
NEUMANN = 1


# -----------------------------------------------------------------------------
# Nodes and differentiation matrices  (Section 2; Section 2.2 affine map)
# -----------------------------------------------------------------------------

def nodes(N: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Ascending CGL nodes t_j = -cos(pi j / N) mapped to [lo, hi]."""
    j = np.arange(N + 1, dtype=np.float64)
    t = np.sin(np.pi * (2.0 * j - N) / (2.0 * N))
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * t


def diff_matrix(N: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Nodal differentiation matrix D_ij = l'_j(x_i) on ascending CGL nodes.

    Off-diagonal entries (cbar_i / cbar_j) (-1)^(i+j) / (t_i - t_j), cbar = 2 at
    the two end nodes and 1 elsewhere (Trefethen, Spectral Methods in MATLAB,
    ch. 6).  Node differences are formed as 2 sin(pi(i+j)/2N) sin(pi(i-j)/2N)
    to avoid cancellation; the diagonal is minus the off-diagonal row sum (so
    D applied to a constant is exactly zero).  Scaled by 2/(hi-lo) for the
    affine map.
    """
    if N < 1:
        raise ValueError("N >= 1 required")
    i = np.arange(N + 1)
    I, J = np.meshgrid(i, i, indexing="ij")
    diff = 2.0 * np.sin(np.pi * (I + J) / (2.0 * N)) * np.sin(np.pi * (I - J) / (2.0 * N))
    cbar = np.ones(N + 1)
    cbar[0] = cbar[N] = 2.0
    sign = np.where((I + J) % 2 == 0, 1.0, -1.0)
    D = np.zeros((N + 1, N + 1))
    off = I != J
    D[off] = (cbar[I[off]] / cbar[J[off]]) * sign[off] / diff[off]
    D[i, i] = -np.sum(D, axis=1)
    return D * (2.0 / (hi - lo))


def deriv(D: np.ndarray, U: np.ndarray, axis: int) -> np.ndarray:
    """(D along `axis`) U, i.e. [dU/dx_a]_{..p..} = sum_m D_pm U_{..m..}."""
    return np.moveaxis(np.tensordot(D, U, axes=(1, axis)), 0, axis)


def deriv_t(D: np.ndarray, U: np.ndarray, axis: int) -> np.ndarray:
    """(D^T along `axis`) U."""
    return np.moveaxis(np.tensordot(D.T, U, axes=(1, axis)), 0, axis)


class Grid3:
    """Tensor CGL grid with per-face boundary types (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi)."""

    def __init__(self, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(DIRICHLET,) * 6, robin=None,
                 robin_nodes=None):
        self.n = tuple(int(v) for v in n)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.bc = tuple(int(v) for v in bc)
        # sigma of the row du/dn + sigma u = g on each Neumann face (0: plain Neumann)
        self.robin = tuple(float(v) for v in (robin if robin is not None else (0.0,) * 6))
        if any(self.robin[f] != 0.0 and self.bc[f] == DIRICHLET for f in range(6)):
            raise ValueError("a Robin coefficient needs a Neumann face")
        if any(v < 3 for v in self.n):
            raise ValueError("at least 3 nodes per axis")
        # a per-node part of sigma (packed faces, the layout of g), added to
        # robin[f] at each node of face f; a coefficient that varies along the
        # face is the general linear row of Section 2.3.1 with node-dependent
        # coefficients (the flux row of Section 3.4 is one)
        self.robin_nodes = None
        if robin_nodes is not None:
            faces = [np.array(F, dtype=np.float64) for F in self.unpack_faces(np.asarray(robin_nodes))]
            if any(self.bc[f] == DIRICHLET and np.any(faces[f] != 0.0) for f in range(6)):
                raise ValueError("a Robin coefficient needs a Neumann face")
            self.robin_nodes = faces
        self.D = [diff_matrix(self.n[a] - 1, self.lo[a], self.hi[a]) for a in range(3)]
        self.x = [nodes(self.n[a] - 1, self.lo[a], self.hi[a]) for a in range(3)]
        self.owner = owner_map(self.n, self.bc)

    @property
    def interior(self):
        return self.owner < 0

    def face_shape(self, f):
        a = f // 2
        return tuple(self.n[b] for b in range(3) if b != a)

    def sigma(self, f):
        """Robin coefficient at every node of face f (array of the face's shape)."""
        s = np.full(self.face_shape(f), self.robin[f])
        if self.robin_nodes is not None:
            s = s + self.robin_nodes[f]
        return s

    def sigma_mean(self):
        """Mean Robin coefficient of each face (the constant-coefficient
        operator that preconditions a node-dependent one uses these)."""
        return tuple(float(np.mean(self.sigma(f))) for f in range(6))

    def sigma_uniform(self):
        return all(np.all(self.sigma(f) == self.robin[f]) for f in range(6))

    def unpack_faces(self, g):
        out, off = [], 0
        for f in range(6):
            s = self.face_shape(f)
            m = s[0] * s[1]
            out.append(np.asarray(g[off:off + m]).reshape(s))
            off += m
        return out


def face_mask(n, f):
    """Boolean mask of the nodes lying on face f."""
    a, side = divmod(f, 2)
    idx = np.arange(n[a])
    on = idx == (0 if side == 0 else n[a] - 1)
    shape = [1, 1, 1]
    shape[a] = n[a]
    return np.broadcast_to(on.reshape(shape), n)


def owner_map(n, bc) -> np.ndarray:
    """Face that owns each boundary node's equation (-1 for interior nodes).

    Reading of the paper (silent on edges/corners, Section 2.3.1): a node on a
    Dirichlet face is owned by the Dirichlet face of lowest axis; a node on
    Neumann faces only is owned by the Neumann face of lowest axis.
    """
    own = np.full(n, -1, dtype=np.int64)
    for kind in (DIRICHLET, NEUMANN):
        for f in range(6):
            if bc[f] != kind:
                continue
            m = face_mask(n, f) & (own < 0)
            own[m] = f
    return own


# -----------------------------------------------------------------------------
# Collocation operator and boundary rows (Algorithm 3; Section 2.3.1)
# -----------------------------------------------------------------------------

def interior_operator(G: Grid3, K: np.ndarray, U: np.ndarray) -> np.ndarray:
    """sum_a D_a (K * D_a U) evaluated at every node."""
    return sum(deriv(G.D[a], K * deriv(G.D[a], U, a), a) for a in range(3))


def end_block(G: Grid3, a: int):
    """Coefficients of the two end values in the boundary rows of each pencil
    along axis a, written as  m00 U_0 + m0N U_N = -g_lo - s_0,
    mN0 U_0 + mNN U_N = g_hi - s_N  with s the rows' sums over the inner nodes.
    The lo row is -(D U)_0 + sigma_lo U_0 = g_lo, the hi row
    (D U)_N + sigma_hi U_N = g_hi (the general linear row a u + b du/dn = g of
    Section 2.3.1 with b != 0, divided by b; sigma = 0 is the Neumann row).
    m00 and mNN are arrays over the pencils (the face's shape: sigma may vary
    from node to node), m0N and mN0 scalars."""
    D = G.D[a]
    N = G.n[a] - 1
    return (D[0, 0] - G.sigma(2 * a), D[0, N], D[N, 0], D[N, N] + G.sigma(2 * a + 1))


def _blocks(m00, m0N, mN0, mNN):
    """Stack of 2 x 2 end blocks [[m00, m0N], [mN0, mNN]], one per pencil."""
    M = np.empty(m00.shape + (2, 2))
    M[..., 0, 0] = m00
    M[..., 0, 1] = m0N
    M[..., 1, 0] = mN0
    M[..., 1, 1] = mNN
    return M


def bc_rows(G: Grid3, U: np.ndarray) -> np.ndarray:
    """Value of each node's boundary row: U (Dirichlet) or outward du/dn + sigma U
    (Neumann/Robin: -D_a U on the lo face, +D_a U on the hi face).  Interior: 0."""
    y = np.zeros_like(U)
    for f in range(6):
        a, side = divmod(f, 2)
        m = G.owner == f
        if not m.any():
            continue
        if G.bc[f] == DIRICHLET:
            y[m] = U[m]
        else:
            d = deriv(G.D[a], U, a)
            sig = np.broadcast_to(np.expand_dims(G.sigma(f), a), G.n)
            y[m] = (d if side == 1 else -d)[m] + sig[m] * U[m]
    return y


def apply_full(G: Grid3, K: np.ndarray, U: np.ndarray) -> np.ndarray:
    """A_full U: interior rows of the collocation operator, boundary rows of B."""
    y = interior_operator(G, K, U)
    y[~G.interior] = 0.0
    return y + bc_rows(G, U)


def face_values(G: Grid3, g) -> np.ndarray:
    """Scatter packed face data onto the nodes each face owns (zero elsewhere)."""
    faces = G.unpack_faces(g)
    out = np.zeros(G.n, dtype=np.result_type(faces[0], np.float64))
    for f in range(6):
        a = f // 2
        m = G.owner == f
        if m.any():
            full = np.broadcast_to(np.expand_dims(faces[f], a), G.n)
            out[m] = full[m]
    return out


def lift(G: Grid3, x: np.ndarray, g=None) -> np.ndarray:
    """Full nodal state from interior values x and face data g (Section 2.3.1,
    x_r = G x_k + H g).

    Order: Dirichlet-owned nodes take their data; then the Neumann-owned nodes
    of the z faces, the y faces and the x faces, each pencil along that axis
    solving its one or two Neumann rows (a 1x1 or 2x2 block of B_r) with every
    other value of the pencil already known.  Unknown boundary values start as
    NaN so that an ordering mistake cannot pass silently.
    """
    U = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    U[~G.interior] = np.nan
    gv = face_values(G, g) if g is not None else np.zeros(G.n)
    for f in range(6):
        if G.bc[f] == DIRICHLET:
            m = G.owner == f
            U[m] = gv[m]
    for a in (2, 1, 0):
        flo, fhi = 2 * a, 2 * a + 1
        own_lo = np.moveaxis(G.owner, a, -1)[..., 0] == flo
        own_hi = np.moveaxis(G.owner, a, -1)[..., -1] == fhi
        nlo = own_lo & (G.bc[flo] == NEUMANN)
        nhi = own_hi & (G.bc[fhi] == NEUMANN)
        if not (nlo.any() or nhi.any()):
            continue
        D = G.D[a]
        N = G.n[a] - 1
        Um = np.moveaxis(U, a, -1)          # view: pencils along a are the last axis
        gm = np.moveaxis(gv, a, -1)
        glo = gm[..., 0]
        ghi = gm[..., -1]
        inner = Um[..., 1:N]
        both = nlo & nhi
        lo_only = nlo & ~nhi
        hi_only = nhi & ~nlo
        m00, m0N, mN0, mNN = end_block(G, a)
        if both.any():
            s0 = inner[both] @ D[0, 1:N]
            sN = inner[both] @ D[N, 1:N]
            M = _blocks(m00[both], m0N, mN0, mNN[both])
            rhs = np.stack([-glo[both] - s0, ghi[both] - sN], axis=-1)
            sol = np.linalg.solve(M, rhs[..., None])[..., 0]
            Um[..., 0][both] = sol[:, 0]
            Um[..., N][both] = sol[:, 1]
        if lo_only.any():
            s0 = Um[lo_only][:, 1:] @ D[0, 1:]
            Um[..., 0][lo_only] = (-glo[lo_only] - s0) / m00[lo_only]
        if hi_only.any():
            sN = Um[hi_only][:, :N] @ D[N, :N]
            Um[..., N][hi_only] = (ghi[hi_only] - sN) / mNN[hi_only]
    if np.isnan(U).any():
        raise AssertionError("lift left boundary values undetermined")
    return U


def lift_transpose(G: Grid3, z: np.ndarray) -> np.ndarray:
    """Transpose of the homogeneous lift, returned on the interior (boundary 0).

    The lift is a product of steps, each overwriting the Neumann-owned end
    values of pencils along one axis with a linear function of that pencil's
    other values.  Its transpose runs the steps in reverse order (x, y, z); a
    step's transpose adds the end value, mapped back by the transposed 1x1/2x2
    solve, onto the other values of the pencil and clears the end.  Dirichlet
    values of a homogeneous lift are zero, so their transpose clears them.
    """
    W = np.array(z, copy=True)
    for a in (0, 1, 2):
        flo, fhi = 2 * a, 2 * a + 1
        own_lo = np.moveaxis(G.owner, a, -1)[..., 0] == flo
        own_hi = np.moveaxis(G.owner, a, -1)[..., -1] == fhi
        nlo = own_lo & (G.bc[flo] == NEUMANN)
        nhi = own_hi & (G.bc[fhi] == NEUMANN)
        if not (nlo.any() or nhi.any()):
            continue
        D = G.D[a]
        N = G.n[a] - 1
        Wm = np.moveaxis(W, a, -1)
        both = nlo & nhi
        lo_only = nlo & ~nhi
        hi_only = nhi & ~nlo
        m00, m0N, mN0, mNN = end_block(G, a)
        if both.any():
            MT = np.swapaxes(_blocks(m00[both], m0N, mN0, mNN[both]), -1, -2)
            # forward: [U0, UN] = M^{-1} [-s0, -sN] (+ data), s = D_{end, 1:N} . inner
            zl = Wm[..., 0][both]
            zh = Wm[..., N][both]
            mu = np.linalg.solve(MT, np.stack([zl, zh], axis=-1)[..., None])[..., 0]
            blk = Wm[both]
            blk[:, 1:N] -= np.outer(mu[:, 0], D[0, 1:N]) + np.outer(mu[:, 1], D[N, 1:N])
            blk[:, 0] = 0.0
            blk[:, N] = 0.0
            Wm[both] = blk
        if lo_only.any():
            blk = Wm[lo_only]
            mu = blk[:, 0] / m00[lo_only]
            blk[:, 1:] -= np.outer(mu, D[0, 1:])
            blk[:, 0] = 0.0
            Wm[lo_only] = blk
        if hi_only.any():
            blk = Wm[hi_only]
            mu = blk[:, N] / mNN[hi_only]
            blk[:, :N] -= np.outer(mu, D[N, :N])
            blk[:, N] = 0.0
            Wm[hi_only] = blk
    W[~G.interior] = 0.0
    return W


def apply_reduced(G: Grid3, K: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Reduced operator (A_kk + A_kr G) x on the interior; boundary entries 0."""
    U = lift(G, np.where(G.interior, x, 0.0), None)
    y = interior_operator(G, K, U)
    y[~G.interior] = 0.0
    return y


def apply_reduced_transpose(G: Grid3, K: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Transpose of the reduced operator: lift^T [sum_a D_a^T (K * D_a^T v~)],
    v~ = v on interior rows and 0 on boundary rows."""
    vt = np.where(G.interior, v, 0.0)
    w = sum(deriv_t(G.D[a], K * deriv_t(G.D[a], vt, a), a) for a in range(3))
    return lift_transpose(G, w)


def reduced_rhs(G: Grid3, K, f, g) -> np.ndarray:
    """f~ = f_k - A_kr H g: interior rows of A applied to the lift of (0, g)."""
    U0 = lift(G, np.zeros(G.n), g)
    r = f - interior_operator(G, K, U0)
    r[~G.interior] = 0.0
    return r


# -----------------------------------------------------------------------------
# Dense assembly and direct solve (small grids)
# -----------------------------------------------------------------------------

def axis_operator_sparse(G: Grid3, a: int):
    mats = [sp.identity(G.n[b], format="csr") for b in range(3)]
    mats[a] = sp.csr_matrix(G.D[a])
    return sp.kron(sp.kron(mats[0], mats[1]), mats[2], format="csr")


def assemble_full(G: Grid3, K: np.ndarray) -> np.ndarray:
    """Dense A_full: interior collocation rows and owned boundary rows."""
    Kd = sp.diags(K.ravel())
    Da = [axis_operator_sparse(G, a) for a in range(3)]
    A = (Da[0] @ Kd @ Da[0] + Da[1] @ Kd @ Da[1] + Da[2] @ Kd @ Da[2]).toarray()
    own = G.owner.ravel()
    for f in range(6):
        rows = np.nonzero(own == f)[0]
        if rows.size == 0:
            continue
        a, side = divmod(f, 2)
        if G.bc[f] == DIRICHLET:
            A[rows, :] = 0.0
            A[rows, rows] = 1.0
        else:
            A[rows, :] = (Da[a][rows, :].toarray()) * (1.0 if side == 1 else -1.0)
            A[rows, rows] += np.broadcast_to(np.expand_dims(G.sigma(f), a), G.n).ravel()[rows]
    return A


def full_rhs(G: Grid3, f, g) -> np.ndarray:
    F = np.where(G.interior, f, 0.0) + face_values(G, g)
    return F


def solve_dense(G: Grid3, K, f, g) -> np.ndarray:
    """Exact solution of [interior rows; owned BC rows] U = [f; g] by LU."""
    A = assemble_full(G, K)
    F = full_rhs(G, f, g).ravel()
    return sla.lu_solve(sla.lu_factor(A), F).reshape(G.n)


def assemble_reduced(G: Grid3, K) -> np.ndarray:
    """Dense reduced matrix on the interior unknowns (columns by lifting unit vectors)."""
    idx = np.nonzero(G.interior.ravel())[0]
    cols = []
    for j in idx:
        e = np.zeros(G.n)
        e.ravel()[j] = 1.0
        cols.append(apply_reduced(G, K, e).ravel()[idx])
    return np.array(cols).T


# -----------------------------------------------------------------------------
# Fast diagonalisation (constant K) and FDM-preconditioned GMRES (variable K)
# -----------------------------------------------------------------------------

def reduced_1d(D: np.ndarray, bclo: int, bchi: int, slo: float = 0.0, shi: float = 0.0) -> np.ndarray:
    """1-D reduced second-derivative operator R D D L on the N-1 interior nodes,
    L the homogeneous lift of one pencil (Robin coefficients slo, shi on
    Neumann ends)."""
    N = D.shape[0] - 1
    L = np.zeros((N + 1, N - 1))
    L[1:N, :] = np.eye(N - 1)
    m00, mNN = D[0, 0] - slo, D[N, N] + shi
    if bclo == NEUMANN and bchi == NEUMANN:
        M = np.array([[m00, D[0, N]], [D[N, 0], mNN]])
        E = -np.linalg.solve(M, np.stack([D[0, 1:N], D[N, 1:N]]))
        L[0, :] = E[0]
        L[N, :] = E[1]
    elif bclo == NEUMANN:
        L[0, :] = -D[0, 1:N] / m00
    elif bchi == NEUMANN:
        L[N, :] = -D[N, 1:N] / mNN
    return (D @ D @ L)[1:N, :]


class FDM:
    """Exact inverse of the constant-coefficient reduced operator Kc * (A_x + A_y + A_z)
    (Kronecker sum of 1-D reduced operators) by eigendecomposition of each.
    Robin coefficients that vary along a face enter through their face means:
    the inverse is then exact only for its own constant-coefficient operator
    (a preconditioner for the node-dependent one)."""

    def __init__(self, G: Grid3, Kc: float = 1.0):
        sm = G.sigma_mean()
        if all(b == NEUMANN for b in G.bc) and not any(sm):
            raise ValueError("all-Neumann problem is singular")
        self.G = G
        self.Kc = float(Kc)
        self.V, self.Vi, self.lam = [], [], []
        for a in range(3):
            A1 = reduced_1d(G.D[a], G.bc[2 * a], G.bc[2 * a + 1], sm[2 * a], sm[2 * a + 1])
            w, V = np.linalg.eig(A1)
            if np.max(np.abs(w.imag)) > 1e-8 * np.max(np.abs(w)):
                raise AssertionError("complex eigenvalues in 1-D reduced operator")
            w, V = w.real, V.real
            self.V.append(V)
            self.Vi.append(np.linalg.inv(V))
            self.lam.append(w)
        l0, l1, l2 = self.lam
        self.den = self.Kc * (l0[:, None, None] + l1[None, :, None] + l2[None, None, :])

    def solve_interior(self, r_int: np.ndarray) -> np.ndarray:
        t = r_int
        for a in range(3):
            t = deriv(self.Vi[a], t, a)
        t = t / self.den
        for a in range(3):
            t = deriv(self.V[a], t, a)
        return t

    def solve(self, r: np.ndarray) -> np.ndarray:
        """Apply the inverse to a full-size array (interior used, boundary -> 0)."""
        out = np.zeros(self.G.n, dtype=np.result_type(r, np.float64))
        out[1:-1, 1:-1, 1:-1] = self.solve_interior(r[1:-1, 1:-1, 1:-1])
        return out


def gmres(matvec, b, precond=None, x0=None, tol=1e-13, restart=60, maxiter=4000):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt (plain
    textbook algorithm, Saad, Iterative Methods, Alg. 9.5).  Vectors are flat."""
    n = b.size
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros(n, dtype=b.dtype) if x0 is None else x0.astype(b.dtype).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    its = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while beta > tol * bnorm and its < maxiter:
        V = np.zeros((restart + 1, n), dtype=b.dtype)
        Z = np.zeros((restart, n), dtype=b.dtype)
        H = np.zeros((restart + 1, restart), dtype=b.dtype)
        V[0] = r / beta
        g = np.zeros(restart + 1, dtype=b.dtype)
        g[0] = beta
        k_used = 0
        for k in range(restart):
            Z[k] = M(V[k])
            w = matvec(Z[k])
            its += 1
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w) if np.iscomplexobj(w) else V[i] @ w
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            k_used = k + 1
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], g[:k + 2], rcond=None)
            res = np.linalg.norm(g[:k + 2] - H[:k + 2, :k + 1] @ y)
            if res <= tol * bnorm or H[k + 1, k] == 0:
                break
        y, *_ = np.linalg.lstsq(H[:k_used + 1, :k_used], g[:k_used + 1], rcond=None)
        x = x + Z[:k_used].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, its, beta / bnorm


def solve_interior_system(G: Grid3, K, rhs_int_full, tol=1e-13, x0=None, Kc=None,
                          restart=60, maxiter=4000):
    """Solve (reduced operator) x = rhs on the interior.  Constant K: FDM
    directly.  Variable K: GMRES right-preconditioned by FDM at mean(K)."""
    K = np.asarray(K)
    kmin, kmax = float(K.min()), float(K.max())
    if kmax - kmin <= 1e-15 * max(abs(kmax), 1.0) and G.sigma_uniform():
        return FDM(G, kmax).solve(rhs_int_full), 0, 0.0
    fdm = FDM(G, float(np.mean(K)) if Kc is None else Kc)
    mask = G.interior

    def mv(v):
        return apply_reduced(G, K, v.reshape(G.n)).ravel()

    def pc(v):
        return fdm.solve(v.reshape(G.n)).ravel()

    b = np.where(mask, rhs_int_full, 0.0).ravel()
    x, its, rel = gmres(mv, b, pc, None if x0 is None else np.where(mask, x0, 0.0).ravel(),
                        tol=tol, restart=restart, maxiter=maxiter)
    return x.reshape(G.n), its, rel


def solve(G: Grid3, K, f, g, tol=1e-13, method="auto", **kw):
    """Full-state solution of the collocation system (Algorithm 2 endpoint)."""
    if method == "dense" or (method == "auto" and np.prod(G.n) <= 17 ** 3 and
                             not np.allclose(K, K.flat[0])):
        return solve_dense(G, K, f, g)
    rt = reduced_rhs(G, K, f, g)
    x, _, _ = solve_interior_system(G, K, rt, tol=tol, **kw)
    return lift(G, x, g)


# -----------------------------------------------------------------------------
# One-dimensional solve (Section 3.1 example), dense
# -----------------------------------------------------------------------------

def solve_1d_dirichlet(N: int, f: np.ndarray, ulo: float = 0.0, uhi: float = 0.0,
                       lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    D = diff_matrix(N, lo, hi)
    A = D @ D
    A[0, :] = 0.0
    A[0, 0] = 1.0
    A[N, :] = 0.0
    A[N, N] = 1.0
    F = f.astype(np.float64).copy()
    F[0] = ulo
    F[N] = uhi
    return np.linalg.solve(A, F)


# -----------------------------------------------------------------------------
# Prolongation and refinement indicator (Section 2.3.3)
# -----------------------------------------------------------------------------

def barycentric_matrix(xc: np.ndarray, xf: np.ndarray) -> np.ndarray:
    """Rows evaluate the CGL interpolant through nodes xc at points xf
    (Berrut & Trefethen 2004, second barycentric form, w_j = (-1)^j delta_j)."""
    Nc = xc.size - 1
    w = np.where(np.arange(Nc + 1) % 2 == 0, 1.0, -1.0)
    w[0] *= 0.5
    w[Nc] *= 0.5
    P = np.zeros((xf.size, xc.size))
    for r, x in enumerate(xf):
        d = x - xc
        hit = np.nonzero(d == 0.0)[0]
        if hit.size:
            P[r, hit[0]] = 1.0
            continue
        t = w / d
        P[r] = t / t.sum()
    return P


def prolong(Uc: np.ndarray, lo, hi, n_fine) -> np.ndarray:
    """Evaluate the tensor interpolant of Uc at the fine CGL grid (the exact
    embedding of P_N in P_Nf obtained by zero-padding the modal coefficients)."""
    U = Uc
    for a in range(3):
        xc = nodes(Uc.shape[a] - 1, lo[a], hi[a])
        xf = nodes(n_fine[a] - 1, lo[a], hi[a])
        U = deriv(barycentric_matrix(xc, xf), U, a)
    return U


def e_ref(U_fine_solved: np.ndarray, U_prolonged: np.ndarray) -> float:
    return float(np.linalg.norm(U_fine_solved - U_prolonged) / np.linalg.norm(U_fine_solved))


# -----------------------------------------------------------------------------
# Quadrature and effective conductivity (Section 3.3)
# -----------------------------------------------------------------------------

def cc_weights(N: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Clenshaw-Curtis weights on the ascending CGL nodes: the unique weights
    integrating T_0..T_N exactly (int T_k = 2/(1-k^2) for even k, 0 for odd k),
    from the Chebyshev-Vandermonde system."""
    t = nodes(N)
    k = np.arange(N + 1)
    V = np.cos(np.outer(np.arccos(np.clip(t, -1.0, 1.0)), k))   # V_jk = T_k(t_j)
    mom = np.where(k % 2 == 0, 2.0 / (1.0 - k.astype(float) ** 2 + (k % 2)), 0.0)
    w = np.linalg.solve(V.T, mom)
    return w * (hi - lo) / 2.0


def volume_average(G: Grid3, F: np.ndarray) -> float:
    w = [cc_weights(G.n[a] - 1, G.lo[a], G.hi[a]) for a in range(3)]
    vol = np.prod([G.hi[a] - G.lo[a] for a in range(3)])
    return float(np.einsum("i,j,k,ijk->", w[0], w[1], w[2], F) / vol)


def flux_average(G: Grid3, K, U) -> np.ndarray:
    """<K dU/dx_b> for b = 0,1,2 (volume averages of -q_b)."""
    return np.array([volume_average(G, K * deriv(G.D[b], U, b)) for b in range(3)])


def effective_conductivity(G: Grid3, K, U, axis: int, gradient: float) -> float:
    """K_num = -<q_a>/G = <K du/dx_a>/G for the load along `axis`."""
    return float(flux_average(G, K, U)[axis] / gradient)


def maxwell_estimate(phi, k_i, k_m):
    """Dilute Maxwell estimate of the effective conductivity (Section 3.3)."""
    return k_m * (2 * k_m + k_i + 2 * phi * (k_i - k_m)) / (2 * k_m + k_i - phi * (k_i - k_m))


# -----------------------------------------------------------------------------
# Adjoint sensitivity of L = 1/2 ||u - u_target||^2 with respect to log K
# -----------------------------------------------------------------------------

def gradient_logK(G: Grid3, K, U, lam) -> np.ndarray:
    """dL/dlogK_j = -K_j sum_a (D_a U)_j (D_a^T lam~)_j, lam~ = lam on interior
    rows, 0 on boundary rows (boundary rows do not depend on K)."""
    lt = np.where(G.interior, lam, 0.0)
    s = sum(deriv(G.D[a], U, a) * deriv_t(G.D[a], lt, a) for a in range(3))
    return -K * s


def adjoint_dense(G: Grid3, K, U, dLdU):
    """lam = A_full^{-T} dL/dU with the assembled matrix; returns (lam, grad)."""
    A = assemble_full(G, K)
    lam = sla.lu_solve(sla.lu_factor(A.T), dLdU.ravel()).reshape(G.n)
    return lam, gradient_logK(G, K, U, lam)


def adjoint_reduced(G: Grid3, K, U, dLdU, tol=1e-13):
    """Same adjoint through the reduced system: (reduced)^T lam_k = r_k + G^T r_r,
    solved by GMRES on the transposed reduced operator.  parity unpinned beyond
    its agreement with adjoint_dense on small grids."""
    rhs = lift_transpose(G, dLdU)
    fdm = FDM(G, float(np.mean(K)))

    def mv(v):
        return apply_reduced_transpose(G, K, v.reshape(G.n)).ravel()

    def pc(v):
        # transpose of the FDM inverse (1-D factors transposed)
        t = v.reshape(G.n)[1:-1, 1:-1, 1:-1]
        for a in range(3):
            t = deriv(fdm.V[a].T, t, a)
        t = t / fdm.den
        for a in range(3):
            t = deriv(fdm.Vi[a].T, t, a)
        out = np.zeros(G.n)
        out[1:-1, 1:-1, 1:-1] = t
        return out.ravel()

    lam, its, rel = gmres(mv, rhs.ravel(), pc, tol=tol)
    lam = lam.reshape(G.n)
    return lam, gradient_logK(G, K, U, lam)


# -----------------------------------------------------------------------------
# Picard iteration for K(x, u) = K0(x) (1 + u^2/2)  (Section 2.3, Picard form)
# -----------------------------------------------------------------------------

def picard(G: Grid3, K0, f, g, tol=1e-10, max_steps=100, U0=None, lin_tol=1e-13):
    """Lagged-coefficient Picard: solve div(K0 (1 + u_m^2/2) grad u_{m+1}) = f
    until ||u_{m+1} - u_m|| / ||u_{m+1}|| <= tol.  Each linear solve starts its
    GMRES from the previous iterate (the solution of each linear system does not
    depend on the starting guess).  Returns (U, steps)."""
    U = np.zeros(G.n) if U0 is None else U0.copy()
    for step in range(1, max_steps + 1):
        K = K0 * (1.0 + 0.5 * U * U)
        Un = solve(G, K, f, g, tol=lin_tol, x0=U)
        rel = np.linalg.norm(Un - U) / max(np.linalg.norm(Un), 1e-300)
        U = Un
        if rel <= tol:
            return U, step
    return U, max_steps


def picard_closed_form_1d(x: np.ndarray, L: float = 1.0) -> np.ndarray:
    """Exact solution for constant K0 with u = -1 at x = 0, u = +1 at x = L and
    zero flux elsewhere: the Kirchhoff variable u + u^3/6 is linear in x, so u
    is the real root of u^3/6 + u = Phi(x), Phi from -7/6 to 7/6 (Cardano)."""
    phi = -7.0 / 6.0 + (7.0 / 3.0) * (x / L)
    q = 3.0 * phi
    s = np.sqrt(q * q + 8.0)
    return np.cbrt(q + s) + np.cbrt(q - s)


# -----------------------------------------------------------------------------
# Newton iteration for k(x, T) = K0(x) / (1 + alpha T)  (Section 3.4)
# -----------------------------------------------------------------------------

def newton_conductivity(K0, alpha: float, T):
    """k = K0 / (1 + alpha T) and its derivative in T, k' = -alpha K0 / (1 + alpha T)^2
    (the reciprocal law of Section 3.4, alpha = 0.5 and K0 = 1 there)."""
    d = 1.0 + alpha * T
    return K0 / d, -alpha * K0 / (d * d)


def newton_residual(G: Grid3, K0, alpha: float, T, f) -> np.ndarray:
    """Interior rows of R(T) = sum_a D_a (k(T) D_a T) - f (Section 3.4 residual,
    written for div(k grad T) = f); boundary entries 0.  T is a full state that
    satisfies its boundary rows (T = lift(x, g)), so those rows have no residual."""
    k, _ = newton_conductivity(K0, alpha, T)
    r = interior_operator(G, k, T) - f
    r[~G.interior] = 0.0
    return r


def newton_jacobian(G: Grid3, K0, alpha: float, T, v) -> np.ndarray:
    """Action of the reduced Jacobian of newton_residual at T on interior values v
    (Section 3.4 Jacobian action): with V = lift(v, 0),
    sum_a D_a (k(T) D_a V + k'(T) V D_a T) on interior rows, 0 on boundary rows."""
    k, dk = newton_conductivity(K0, alpha, T)
    V = lift(G, np.where(G.interior, v, 0.0), None)
    y = sum(deriv(G.D[a], k * deriv(G.D[a], V, a) + dk * V * deriv(G.D[a], T, a), a)
            for a in range(3))
    y[~G.interior] = 0.0
    return y


def newton(G: Grid3, K0, alpha: float, f, g, tol=1e-10, max_steps=50, U0=None, lin_tol=1e-13):
    """Newton's method on the reduced system (Section 2.3 Newton form, Section 3.4):
    T_m = lift(x_m, g); stop once ||R(T_m)|| <= tol r_ref, r_ref = ||R(lift(0, g))||
    (the paper states no stopping rule; this one judges warm and cold starts on
    the same scale); otherwise solve J(T_m) dx = -R(T_m) by GMRES (preconditioned
    by the constant-coefficient inverse at the mean of k(T_m)) to the relative
    residual lin_tol -- an exact Newton step up to that tolerance -- and set
    x_{m+1} = x_m + dx.  Returns (T, steps, gmres iterations per step)."""
    K0 = np.broadcast_to(np.asarray(K0, dtype=np.float64), G.n)
    rref = float(np.linalg.norm(newton_residual(G, K0, alpha, lift(G, np.zeros(G.n), g), f)))
    x = np.zeros(G.n) if U0 is None else np.where(G.interior, U0, 0.0)
    T = lift(G, x, g)
    its = []
    for step in range(max_steps + 1):
        R = newton_residual(G, K0, alpha, T, f)
        rn = float(np.linalg.norm(R))
        if rn <= tol * rref or step == max_steps:
            return T, step, its
        k, _ = newton_conductivity(K0, alpha, T)
        if not np.all(k > 0):
            raise ValueError("Newton iterate left the range where 1 + alpha T > 0")
        fdm = FDM(G, float(np.mean(k)))
        Tm = T

        def mv(v):
            return newton_jacobian(G, K0, alpha, Tm, v.reshape(G.n)).ravel()

        def pc(v):
            return fdm.solve(v.reshape(G.n)).ravel()

        dx, it, _ = gmres(mv, (-R).ravel(), pc, tol=lin_tol)
        its.append(it)
        x = x + np.where(G.interior, dx.reshape(G.n), 0.0)
        T = lift(G, x, g)
    return T, max_steps, its
