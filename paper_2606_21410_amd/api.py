"""Torch-facing wrappers of the C ABI (argument marshalling only).

PyTorch provides device memory and the stream; every step of the solver runs in
the HIP kernels of libchebfft.so.  Names follow the C calls: ``Plan.apply`` is
``cheb_apply``, ``Plan.solve`` is ``cheb_solve`` and so on.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

_PREC = {"f64": L.CHEB_F64, "f32": L.CHEB_F32, "mixed": L.CHEB_MIXED}
_MODE = {"full": L.CHEB_APPLY_FULL, "reduced": L.CHEB_APPLY_REDUCED,
         "transpose": L.CHEB_APPLY_REDUCED | L.CHEB_APPLY_TRANSPOSE}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class SolveOptions:
    rtol: float = 1e-10
    atol: float = 0.0
    maxiter: int = 10000
    inner_m: int = 30
    outer_k: int = 3
    ir_inner_rtol: float = 1e-3
    ir_max_outer: int = 50
    history_len: int = 0
    precond: bool = False   # fast-diagonalisation right preconditioner (extension)

    def to_c(self, warm: bool):
        o = L.cheb_solve_opts()
        o.rtol, o.atol, o.maxiter = self.rtol, self.atol, self.maxiter
        o.inner_m, o.outer_k = self.inner_m, (self.outer_k if self.outer_k > 0 else -1)
        o.ir_inner_rtol, o.ir_max_outer = self.ir_inner_rtol, self.ir_max_outer
        o.flags = (1 if warm else 0) | (2 if self.precond else 0)
        hist = None
        if self.history_len > 0:
            hist = (ctypes.c_double * self.history_len)()
            o.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
            o.history_len = self.history_len
        return o, hist


_ROUTE = {"auto": L.CHEB_ROUTE_AUTO, "fft": L.CHEB_ROUTE_FFT, "matrix": L.CHEB_ROUTE_MATRIX}


class Plan:
    """One grid: sizes, box, face types, precision ('f64', 'f32', 'mixed').

    ``robin``: six coefficients sigma, one per face; a Neumann face with sigma != 0
    carries the Robin row du/dn + sigma u = g (cheb_grid.robin).
    ``robin_nodes``: optional per-node part of sigma (packed faces, the layout of
    g; see set_robin_nodes)."""

    def __init__(self, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(0,) * 6, precision="f64",
                 device="cuda", route: str = "auto", robin=None, robin_nodes=None):
        self.lib = L.load()
        self.n = tuple(int(v) for v in n)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.bc = tuple(int(v) for v in bc)
        self.robin = tuple(float(v) for v in (robin if robin is not None else (0.0,) * 6))
        self.precision = precision
        self.device = torch.device(device)
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        g = L.cheb_grid()
        for a in range(3):
            g.n[a], g.lo[a], g.hi[a] = self.n[a], self.lo[a], self.hi[a]
        for f in range(6):
            g.bc[f] = self.bc[f]
            g.robin[f] = self.robin[f]
        self._h = ctypes.c_void_p()
        stream = _stream_handle(self.device) if self.device.type == "cuda" else 0
        L.check(self.lib.cheb_plan_create(ctypes.byref(g), _PREC[precision], ctypes.c_void_p(stream),
                                          ctypes.byref(self._h)))
        self._ws = None
        self._ws_bytes = 0
        self.set_route(route)
        self.robin_nodes = None
        if robin_nodes is not None:
            self.set_robin_nodes(robin_nodes)

    def set_robin_nodes(self, sigma_faces):
        """Robin coefficients that vary from node to node (cheb_plan_set_robin_nodes):
        ``sigma_faces`` holds, in the packed face layout of g, the per-node part
        added to ``robin[f]`` on each face (0 on Dirichlet faces); None removes
        it.  The flux condition k(T) dT/dn = h of k = K0 / (1 + alpha T) is the
        row with sigma = -alpha h / K0 and data h / K0."""
        if sigma_faces is None:
            L.check(self.lib.cheb_plan_set_robin_nodes(self._h, None))
            self.robin_nodes = None
            return
        t = torch.as_tensor(sigma_faces, dtype=torch.float64).to(self.device).contiguous()
        want = sum(self.n[b] * self.n[c] for b, c in ((1, 2), (1, 2), (0, 2), (0, 2), (0, 1), (0, 1)))
        if t.numel() != want:
            raise ValueError(f"robin_nodes: expected {want} packed face entries, got {t.numel()}")
        self._sync_stream()
        L.check(self.lib.cheb_plan_set_robin_nodes(self._h, ctypes.c_void_p(t.data_ptr())))
        self.robin_nodes = t

    def set_route(self, route: str):
        """'auto', 'fft' or 'matrix': how the reduced operator evaluates the per-axis derivatives."""
        L.check(self.lib.cheb_plan_set_route(self._h, _ROUTE[route]))
        self.route = route

    def set_tile_shape(self, shape: int, precision: str = "f64"):
        """Tile shape of the matrix-core route for the passes that run in
        ``precision`` ('f64' or 'f32'): 0 = 8-wave workgroups with the fragment
        table in LDS, 1 = 4-wave workgroups with register fragments."""
        L.check(self.lib.cheb_plan_set_tile_shape(self._h, _PREC[precision], int(shape)))

    def capture_applies(self, K, us, ys, mode: str = "reduced"):
        """Record one operator application per (u, y) pair into a HIP graph
        (torch.cuda.CUDAGraph; the applies launch only kernels, no memsets or
        allocations).  Returns the graph; ``graph.replay()`` runs all of them."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            for u, y in zip(us, ys):
                self.apply(K, u, y, mode)  # first launches set up per-kernel state outside the capture
        torch.cuda.current_stream(self.device).wait_stream(side)
        torch.cuda.synchronize(self.device)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for u, y in zip(us, ys):
                self.apply(K, u, y, mode)
        return graph

    def autotune(self, K=None, u=None):
        """Time the FFT route and the matrix-core tile shapes of the reduced
        operator (per precision the plan computes in) and keep the fastest for
        route 'auto'.  Returns {precision: {"fft": us, "matrix0": us,
        "matrix1": us, "chosen": name}}."""
        out = {}
        precs = {"f64": [("f64", torch.float64)], "f32": [("f32", torch.float32)],
                 "mixed": [("f64", torch.float64), ("f32", torch.float32)]}[self.precision]
        names = ["fft", "matrix0", "matrix1"]
        for pname, dt in precs:
            Kt = (K if K is not None else torch.ones(self.n, device=self.device, dtype=torch.float64)).to(dt)
            ut = (u if u is not None else torch.randn(self.n, device=self.device, dtype=torch.float64)).to(dt)
            Kt, ut = Kt.contiguous(), ut.contiguous()
            yt = torch.empty_like(ut)
            rep = (ctypes.c_double * 4)()
            self._sync_stream()
            L.check(self.lib.cheb_plan_autotune(self._h, _PREC[pname], ctypes.c_void_p(Kt.data_ptr()),
                                                ctypes.c_void_p(ut.data_ptr()), ctypes.c_void_p(yt.data_ptr()),
                                                rep, 4))
            out[pname] = {names[i]: rep[i] for i in range(3)}
            out[pname]["chosen"] = names[int(rep[3])]
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.cheb_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _sync_stream(self):
        self.lib.cheb_plan_set_stream(self._h, ctypes.c_void_p(_stream_handle(self.device)))

    def _field(self, t: torch.Tensor, name: str, dtype=None):
        dtype = dtype or self.dtype
        if t.device != self.device and not (t.device.type == self.device.type):
            raise ValueError(f"{name}: expected a tensor on {self.device}")
        if t.dtype != dtype or tuple(t.shape) != self.n or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {dtype} tensor of shape {self.n}, got "
                             f"{t.dtype} {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def face_count(self):
        n = self.n
        return 2 * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1])

    def workspace_bytes(self, opts: SolveOptions | None = None) -> int:
        o, _ = (opts or SolveOptions()).to_c(False)
        b = ctypes.c_size_t()
        L.check(self.lib.cheb_plan_workspace_bytes(self._h, ctypes.byref(o), ctypes.byref(b)))
        return int(b.value)

    def ensure_workspace(self, opts: SolveOptions | None = None):
        need = self.workspace_bytes(opts)
        if self._ws is None or self._ws_bytes < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need
            L.check(self.lib.cheb_plan_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                                     ctypes.c_size_t(need)))
        return self._ws

    # --- calls -------------------------------------------------------------
    def apply(self, K, u, y=None, mode: str = "full"):
        self._sync_stream()
        if y is None:
            y = torch.empty_like(u)
        L.check(self.lib.cheb_apply(self._h, self._field(K, "K"), self._field(u, "u"), self._field(y, "y"),
                                    _MODE[mode]))
        return y

    def derivative(self, u, axis: int, out=None):
        self._sync_stream()
        if out is None:
            out = torch.empty_like(u)
        L.check(self.lib.cheb_derivative(self._h, self._field(u, "u"), self._field(out, "du"), int(axis)))
        return out

    def solve(self, K, f, g, u0=None, opts: SolveOptions | None = None, out=None):
        opts = opts or SolveOptions()
        self._sync_stream()
        self.ensure_workspace(opts)
        if out is None:
            out = torch.zeros(self.n, dtype=self.dtype, device=self.device)
        if u0 is not None:
            out.copy_(u0)
        gdt = self.dtype
        if g.dtype != gdt or g.numel() != self.face_count() or not g.is_contiguous():
            raise ValueError("g: packed face data of the plan's dtype expected")
        o, hist = opts.to_c(u0 is not None)
        info = L.cheb_solve_info()
        rc = L.check(self.lib.cheb_solve(self._h, self._field(K, "K"), self._field(f, "f"),
                                         ctypes.c_void_p(g.data_ptr()), self._field(out, "u"),
                                         ctypes.byref(o), ctypes.byref(info)))
        d = info.as_dict()
        d["rc"] = rc
        if hist is not None:
            d["history"] = [hist[i] for i in range(info.history_used)]
        return out, d

    def adjoint(self, K, u, dLdu, opts: SolveOptions | None = None):
        opts = opts or SolveOptions()
        self._sync_stream()
        self.ensure_workspace(opts)
        lam = torch.empty_like(u)
        grad = torch.empty_like(u)
        o, hist = opts.to_c(False)
        info = L.cheb_solve_info()
        rc = L.check(self.lib.cheb_adjoint(self._h, self._field(K, "K"), self._field(u, "u"),
                                           self._field(dLdu, "dLdu"), self._field(lam, "lambda"),
                                           self._field(grad, "dLdlogK"), ctypes.byref(o),
                                           ctypes.byref(info)))
        d = info.as_dict()
        d["rc"] = rc
        if hist is not None:
            d["history"] = [hist[i] for i in range(info.history_used)]
        return lam, grad, d

    def picard(self, K0, f, g, u0=None, tol=1e-10, max_steps=50, opts: SolveOptions | None = None):
        opts = opts or SolveOptions()
        self._sync_stream()
        self.ensure_workspace(opts)
        u = torch.zeros(self.n, dtype=self.dtype, device=self.device)
        if u0 is not None:
            u.copy_(u0)
        Kw = torch.empty_like(u)
        o, hist = opts.to_c(u0 is not None)
        info = L.cheb_solve_info()
        steps = ctypes.c_int32()
        rc = L.check(self.lib.cheb_picard(self._h, self._field(K0, "K0"), self._field(f, "f"),
                                          ctypes.c_void_p(g.data_ptr()), self._field(u, "u"),
                                          self._field(Kw, "Kwork"), float(tol), int(max_steps),
                                          ctypes.byref(o), ctypes.byref(info), ctypes.byref(steps)))
        d = info.as_dict()
        d["rc"] = rc
        d["picard_steps"] = steps.value
        if hist is not None:
            d["history"] = [hist[i] for i in range(min(steps.value, opts.history_len))]
        return u, d

    def _newton_work(self):
        b = ctypes.c_size_t()
        L.check(self.lib.cheb_newton_work_bytes(self._h, ctypes.byref(b)))
        if getattr(self, "_nwork", None) is None or self._nwork.numel() < b.value:
            self._nwork = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        return ctypes.c_void_p(self._nwork.data_ptr())

    def newton_residual(self, K0, T, f, alpha=0.5, out=None):
        """R(T) = sum_a D_a (k(T) D_a T) - f on interior rows, k = K0 / (1 + alpha T)."""
        self._sync_stream()
        f64 = torch.float64
        r = out if out is not None else torch.empty(self.n, dtype=f64, device=self.device)
        L.check(self.lib.cheb_newton_residual(self._h, self._field(K0, "K0", f64), float(alpha),
                                              self._field(T, "T", f64), self._field(f, "f", f64),
                                              self._field(r, "r", f64), self._newton_work()))
        return r

    def newton_jacobian(self, K0, T, v, alpha=0.5, out=None):
        """Reduced Jacobian action J(T) v of newton_residual (interior rows)."""
        self._sync_stream()
        f64 = torch.float64
        y = out if out is not None else torch.empty(self.n, dtype=f64, device=self.device)
        L.check(self.lib.cheb_newton_jacobian(self._h, self._field(K0, "K0", f64), float(alpha),
                                              self._field(T, "T", f64), self._field(v, "v", f64),
                                              self._field(y, "y", f64), self._newton_work()))
        return y

    def newton(self, K0, f, g, alpha=0.5, u0=None, tol=1e-10, max_steps=30,
               opts: SolveOptions | None = None):
        """Newton-LGMRES for div(k(T) grad T) = f, k = K0 / (1 + alpha T)."""
        opts = opts or SolveOptions()
        self._sync_stream()
        self.ensure_workspace(opts)
        f64 = torch.float64
        u = torch.zeros(self.n, dtype=f64, device=self.device)
        if u0 is not None:
            u.copy_(u0)
        o, hist = opts.to_c(u0 is not None)
        info = L.cheb_solve_info()
        steps = ctypes.c_int32()
        mv = (ctypes.c_int32 * max(int(max_steps), 1))()
        rc = L.check(self.lib.cheb_newton(self._h, self._field(K0, "K0", f64), float(alpha),
                                          self._field(f, "f", f64), ctypes.c_void_p(g.data_ptr()),
                                          self._field(u, "u", f64), self._newton_work(), float(tol),
                                          int(max_steps), ctypes.byref(o), ctypes.byref(info),
                                          ctypes.byref(steps), mv))
        d = info.as_dict()
        d["rc"] = rc
        d["newton_steps"] = steps.value
        d["mv_per_step"] = [mv[i] for i in range(steps.value)]
        if hist is not None:
            d["history"] = [hist[i] for i in range(min(steps.value + 1, opts.history_len))]
        return u, d

    def precond(self, r, kc: float, out=None, transpose: bool = False):
        """Fast-diagonalisation inverse of the constant-coefficient reduced
        operator (cheb_precond_apply): out = (kc (A_x + A_y + A_z))^{-1} r on
        the interior, 0 on the boundary; r is float64 or float32."""
        self._sync_stream()
        prec = {torch.float64: L.CHEB_F64, torch.float32: L.CHEB_F32}.get(r.dtype)
        if prec is None:
            raise ValueError("r: expected float64 or float32")
        m = [d - 2 for d in self.n]
        es = 8 if prec == L.CHEB_F64 else 4
        pb = -(-m[0] * m[1] * m[2] * es // 256) * 256
        need = max(self.workspace_bytes(), 2 * pb)
        if self._ws is None or self._ws_bytes < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need
            L.check(self.lib.cheb_plan_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                                     ctypes.c_size_t(need)))
        if out is None:
            out = torch.empty_like(r)
        L.check(self.lib.cheb_precond_apply(self._h, prec, float(kc), self._field(r, "r", r.dtype),
                                            self._field(out, "out", r.dtype),
                                            L.CHEB_APPLY_TRANSPOSE if transpose else 0))
        return out

    def apparent_conductivity(self, K, u, axis: int, jump: float = 1.0):
        """Column `axis` of the apparent conductivity tensor from one load case
        (cheb_apparent_conductivity): <K du/dx_b>_CC / G, G = jump / L_axis."""
        self._sync_stream()
        self.ensure_workspace()
        out = (ctypes.c_double * 3)()
        L.check(self.lib.cheb_apparent_conductivity(self._h, self._field(K, "K"), self._field(u, "u"),
                                                    int(axis), float(jump), out))
        return [out[0], out[1], out[2]]

    def flux_average(self, K, u):
        self._sync_stream()
        self.ensure_workspace()
        out = (ctypes.c_double * 3)()
        L.check(self.lib.cheb_flux_average(self._h, self._field(K, "K"), self._field(u, "u"), out))
        return [out[0], out[1], out[2]]


class Batch:
    """Many independent systems solved in lockstep (cheb_batch_*).

    ``grids``: list of (n, lo, hi, bc) tuples, one per system (a fifth entry,
    Robin coefficients, must be all zero).  Systems with the
    same n, lo, hi share operator launches; systems that also share the face
    types share preconditioner launches."""

    def __init__(self, grids, precision="f64", device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.precision = precision
        self.grids = [(tuple(int(v) for v in gr[0]), tuple(float(v) for v in gr[1]),
                       tuple(float(v) for v in gr[2]), tuple(int(v) for v in gr[3])) for gr in grids]
        # optional fifth entry: Robin coefficients (the library accepts only zeros here)
        robins = [tuple(float(v) for v in gr[4]) if len(gr) > 4 else (0.0,) * 6 for gr in grids]
        arr = (L.cheb_grid * len(self.grids))()
        for i, (n, lo, hi, bc) in enumerate(self.grids):
            for a in range(3):
                arr[i].n[a], arr[i].lo[a], arr[i].hi[a] = n[a], lo[a], hi[a]
            for f in range(6):
                arr[i].bc[f] = bc[f]
                arr[i].robin[f] = robins[i][f]
        self._h = ctypes.c_void_p()
        L.check(self.lib.cheb_batch_create(arr, len(self.grids), _PREC[precision],
                                           ctypes.c_void_p(_stream_handle(self.device)), ctypes.byref(self._h)))
        self._ws = None
        self._ws_bytes = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.cheb_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, opts=None):
        o, _ = (opts or SolveOptions()).to_c(False)
        b = ctypes.c_size_t()
        L.check(self.lib.cheb_batch_workspace_bytes(self._h, ctypes.byref(o), ctypes.byref(b)))
        return int(b.value)

    def ensure_workspace(self, opts=None):
        need = self.workspace_bytes(opts)
        if self._ws is None or self._ws_bytes < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws_bytes = need
            L.check(self.lib.cheb_batch_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                                      ctypes.c_size_t(need)))
        return self._ws

    def tile_shapes(self, precision="f64"):
        """The autotuner's choice per matrix-core size group after a solve:
        list of dicts {n, shape, us_shape0, us_shape1} (shape -1: not tuned)."""
        buf = (ctypes.c_int32 * 256)()
        prec = L.CHEB_F64 if precision == "f64" else L.CHEB_F32
        ng = L.check(self.lib.cheb_batch_tile_shapes(self._h, prec, buf, 256))
        return [{"n": buf[4 * i], "shape": buf[4 * i + 1], "us_shape0": buf[4 * i + 2] / 1e3,
                 "us_shape1": buf[4 * i + 3] / 1e3} for i in range(ng)]

    def solve(self, Ks, fs, gs, us=None, opts=None):
        """Solve every system; returns (list of full-grid solutions, list of info dicts)."""
        opts = opts or SolveOptions()
        ns = len(self.grids)
        assert len(Ks) == len(fs) == len(gs) == ns
        warm = us is not None
        if us is None:
            us = [torch.zeros(g[0], dtype=torch.float64, device=self.device) for g in self.grids]
        for i, (n, _, _, _) in enumerate(self.grids):
            for name, t, shape in (("K", Ks[i], n), ("f", fs[i], n), ("u", us[i], n)):
                if t.dtype != torch.float64 or tuple(t.shape) != n or not t.is_contiguous():
                    raise ValueError(f"{name}[{i}]: expected a contiguous float64 tensor of shape {n}")
            if gs[i].dtype != torch.float64 or not gs[i].is_contiguous():
                raise ValueError(f"g[{i}]: expected a contiguous float64 tensor")
        self.ensure_workspace(opts)
        L.check(self.lib.cheb_batch_set_stream(self._h, ctypes.c_void_p(_stream_handle(self.device))))
        arr = lambda ts: (ctypes.c_void_p * ns)(*[t.data_ptr() for t in ts])
        o, hist = opts.to_c(warm)
        infos = (L.cheb_solve_info * ns)()
        rc = L.check(self.lib.cheb_batch_solve(self._h, arr(Ks), arr(fs), arr(gs), arr(us), ctypes.byref(o), infos))
        out = []
        for i in range(ns):
            d = infos[i].as_dict()
            d["rc"] = rc
            out.append(d)
        return us, out


def load_case(n, axis, device="cuda"):
    """Boundary data of homogenisation load case `axis`: u = 0 on the axis' lo
    face, 1 on its hi face (unit mean gradient on the unit box), zero flux on
    the other four faces.  Returns (bc, packed face data)."""
    bc = [1] * 6
    bc[2 * axis] = bc[2 * axis + 1] = 0
    sizes = [n[1] * n[2], n[1] * n[2], n[0] * n[2], n[0] * n[2], n[0] * n[1], n[0] * n[1]]
    g = torch.zeros(sum(sizes), dtype=torch.float64, device=device)
    start = sum(sizes[:2 * axis + 1])
    g[start:start + sizes[2 * axis + 1]] = 1.0
    return tuple(bc), g


def solve_2d(K, f, g, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(L.CHEB_DIRICHLET,) * 4, precision="f64", opts=None,
             device="cuda", robin=None):
    """The 2-D problem div(K grad u) = f on a rectangle (the setting in which
    Algorithms 2 and 3 are written), through the 3-D solver.  The grid gets a
    third axis of three nodes with zero-flux faces, and K, f and the face data
    are constant along it.  A z-constant field has zero z-derivative, so the 3-D
    collocation system maps z-constant fields to z-constant fields and is the
    2-D system on them.  Its solution repeats the 2-D one along z (the Krylov
    iterates stay z-constant: the same iterations, at three times the 2-D
    work per matvec).

    K, f: (n0, n1) tensors.  g: four face vectors [x_lo (n1,), x_hi (n1,),
    y_lo (n0,), y_hi (n0,)], Dirichlet values or outward normal derivatives per
    ``bc`` (plus robin[f] u on faces with a Robin coefficient).  Returns
    (u of shape (n0, n1), info)."""
    n0, n1 = K.shape
    r3 = tuple(robin) + (0.0, 0.0) if robin is not None else None
    plan = Plan((n0, n1, 3), (lo[0], lo[1], 0.0), (hi[0], hi[1], 1.0), tuple(bc) + (L.CHEB_NEUMANN,) * 2,
                precision, device, robin=r3)
    dt = plan.dtype
    col = lambda t, m: torch.as_tensor(t).to(device, dt).reshape(m, 1).expand(m, 3).reshape(-1)
    K3 = torch.as_tensor(K).to(device, dt).reshape(n0, n1, 1).expand(n0, n1, 3).contiguous()
    f3 = torch.as_tensor(f).to(device, dt).reshape(n0, n1, 1).expand(n0, n1, 3).contiguous()
    zeros = torch.zeros(2 * n0 * n1, dtype=dt, device=device)
    gp = torch.cat([col(g[0], n1), col(g[1], n1), col(g[2], n0), col(g[3], n0), zeros]).contiguous()
    u3, info = plan.solve(K3, f3, gp, opts=opts)
    return u3[:, :, 0].contiguous(), info


def solve_1d(K, f, g, lo=-1.0, hi=1.0, bc=(L.CHEB_DIRICHLET,) * 2, precision="f64", opts=None, device="cuda",
             robin=None):
    """The 1-D problem (K u')' = f on [lo, hi] (the setting of the paper's
    first example), through the 3-D solver with two further axes of three
    nodes, zero-flux faces and data constant along them (see solve_2d).
    K, f: (n,) tensors; g: [value or outward derivative at lo, at hi] (plus
    robin[f] u with a Robin coefficient).  Returns (u of shape (n,), info)."""
    n = K.shape[0]
    r3 = tuple(robin) + (0.0,) * 4 if robin is not None else None
    plan = Plan((n, 3, 3), (lo, 0.0, 0.0), (hi, 1.0, 1.0), tuple(bc) + (L.CHEB_NEUMANN,) * 4, precision, device,
                robin=r3)
    dt = plan.dtype
    K3 = torch.as_tensor(K).to(device, dt).reshape(n, 1, 1).expand(n, 3, 3).contiguous()
    f3 = torch.as_tensor(f).to(device, dt).reshape(n, 1, 1).expand(n, 3, 3).contiguous()
    gp = torch.cat([torch.full((9,), float(g[0]), dtype=dt, device=device),
                    torch.full((9,), float(g[1]), dtype=dt, device=device),
                    torch.zeros(4 * 3 * n, dtype=dt, device=device)]).contiguous()
    u3, info = plan.solve(K3, f3, gp, opts=opts)
    return u3[:, 1, 1].contiguous(), info


def homogenize(Ks, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), precision="mixed", opts=None, device="cuda",
               details=None, batch=None):
    """Apparent conductivity tensors of several microstructures (Section 3.3):
    three load cases per microstructure (unit mean gradient along x, y, z
    through Dirichlet faces, zero flux elsewhere) solved together in one batch,
    then K_app[b][a] = <K du^(a)/dx_b>_CC / G_a with Clenshaw-Curtis volume
    averages (cheb_apparent_conductivity).  Returns (list of 3x3 nested lists, per-system infos, solutions);
    a dict passed as `details` receives the batch's tuned tile shapes and the
    batch itself ("batch"), which a later call on microstructures of the same
    sizes may pass back as `batch` to skip its set-up (plans, preconditioner
    factors, tile-shape tuning)."""
    grids, KK, ff, gg = [], [], [], []
    for K in Ks:
        n = tuple(K.shape)
        for a in range(3):
            bc, g = load_case(n, a, device)
            grids.append((n, lo, hi, bc))
            KK.append(K)
            ff.append(torch.zeros(n, dtype=torch.float64, device=device))
            gg.append(g)
    if batch is None:
        batch = Batch(grids, precision, device)
    us, infos = batch.solve(KK, ff, gg, opts=opts)
    if details is not None:
        details["batch"] = batch
        details["tile_shapes_f64"] = batch.tile_shapes("f64")
        if precision == "mixed":
            details["tile_shapes_f32"] = batch.tile_shapes("f32")
    out = []
    for s, K in enumerate(Ks):
        n = tuple(K.shape)
        plan = Plan(n, lo, hi, grids[3 * s][3], "f64", device)
        Kapp = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            col = plan.apparent_conductivity(K, us[3 * s + a], a, 1.0)
            for b in range(3):
                Kapp[b][a] = col[b]
        out.append(Kapp)
    return out, infos, us


def debug_gemm(A, B):
    """D = A @ B on the matrix cores (the preconditioner's contraction kernel)."""
    lib = L.load()
    I, K = A.shape
    K2, C = B.shape
    assert K == K2 and A.dtype == B.dtype and A.is_contiguous() and B.is_contiguous()
    D = torch.empty((I, C), dtype=A.dtype, device=A.device)
    prec = L.CHEB_F32 if A.dtype == torch.float32 else L.CHEB_F64
    L.check(lib.cheb_debug_gemm(prec, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                ctypes.c_void_p(D.data_ptr()), I, K, C,
                                ctypes.c_void_p(_stream_handle(A.device))))
    return D


def prolong(coarse: Plan, fine: Plan, uc, uf=None, uf_solved=None):
    """Zero-padding prolongation of uc (coarse grid) onto the fine grid; with
    uf_solved also returns e_ref."""
    fine._sync_stream()
    fine.ensure_workspace()
    if uf is None:
        uf = torch.empty(fine.n, dtype=fine.dtype, device=fine.device)
    e = ctypes.c_double(float("nan"))
    L.check(fine.lib.cheb_prolong(coarse.handle, fine.handle, coarse._field(uc, "u_c"), fine._field(uf, "u_f"),
                                  fine._field(uf_solved, "u_f_solved") if uf_solved is not None else None,
                                  ctypes.byref(e) if uf_solved is not None else None))
    return uf, (e.value if uf_solved is not None else None)


def refine(plans, Ks, fs, gs, tol, opts: SolveOptions | None = None, u0=None):
    """Hierarchical refinement with its stopping rule (Section 2.3.3,
    Algorithm 4) through cheb_refine: plans[l] are the levels (same box and
    faces, growing sizes), Ks/fs/gs their data.  Level 0 is solved (from u0 if
    given); each later level starts from the modal prolongation of the previous
    one and is solved until the refinement indicator e_ref <= tol, after which
    finer levels are the prolongation alone.  Returns (list of per-level
    results, e_ref per level (nan where not solved or level 0), solved flags,
    per-level info dicts)."""
    opts = opts or SolveOptions()
    n = len(plans)
    assert n >= 1 and len(Ks) == len(fs) == len(gs) == n
    lib = plans[0].lib
    for pl in plans:
        pl._sync_stream()
        pl.ensure_workspace(opts)
    us = [torch.zeros(pl.n, dtype=pl.dtype, device=pl.device) for pl in plans]
    if u0 is not None:
        us[0].copy_(u0)
    tmp = torch.empty(plans[-1].n, dtype=plans[-1].dtype, device=plans[-1].device)
    for pl, g in zip(plans, gs):
        if g.dtype != pl.dtype or g.numel() != pl.face_count() or not g.is_contiguous():
            raise ValueError("g: packed face data of the plan's dtype expected")
    arr = lambda xs: (L._vp * n)(*xs)
    hp = arr([pl.handle for pl in plans])
    kp = arr([pl._field(K, "K") for pl, K in zip(plans, Ks)])
    fp = arr([pl._field(f, "f") for pl, f in zip(plans, fs)])
    gp = arr([ctypes.c_void_p(g.data_ptr()) for g in gs])
    up = arr([pl._field(u, "u") for pl, u in zip(plans, us)])
    o, _ = opts.to_c(u0 is not None)
    e = (ctypes.c_double * n)()
    solved = (ctypes.c_int32 * n)()
    infos = (L.cheb_solve_info * n)()
    rc = L.check(lib.cheb_refine(hp, n, kp, fp, gp, up, ctypes.c_void_p(tmp.data_ptr()), ctypes.byref(o),
                                 float(tol), e, solved, infos))
    out_infos = []
    for i in range(n):
        d = infos[i].as_dict()
        d["rc"] = rc
        out_infos.append(d)
    return us, [e[i] for i in range(n)], [int(solved[i]) for i in range(n)], out_infos


class SolveNotConverged(L.ChebError):
    """A solve inside autograd ended with a soft status (not converged or
    stagnated): its output is the best iterate, not the solution, so neither
    it nor a gradient computed from it is returned.  ``info`` holds the
    solver's report."""

    def __init__(self, what: str, info: dict):
        super().__init__(info["status"], f"{what} ended with status {info['status']} "
                                         f"(relres {info['relres_final']:.3e}, {info['matvecs']} matvecs)")
        self.info = info


class ChebSolveFn(torch.autograd.Function):
    """u = solve(K = exp(logK)); backward: dL/dlogK through cheb_adjoint.
    Both solves must converge (status 0); otherwise SolveNotConverged is raised."""

    @staticmethod
    def forward(ctx, logK, plan: Plan, f, g, opts):
        K = torch.exp(logK).contiguous()
        u, info = plan.solve(K, f, g, opts=opts)
        if info["status"] != 0:
            raise SolveNotConverged("forward solve", info)
        ctx.plan, ctx.opts = plan, opts
        ctx.save_for_backward(K, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        K, u = ctx.saved_tensors
        _, grad, info = ctx.plan.adjoint(K, u, grad_u.contiguous(), ctx.opts)
        if info["status"] != 0:
            raise SolveNotConverged("adjoint solve", info)
        return grad, None, None, None, None


def solve_logk(plan: Plan, logK, f, g, opts: SolveOptions | None = None):
    return ChebSolveFn.apply(logK, plan, f, g, opts or SolveOptions())
