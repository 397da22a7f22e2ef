"""lsweep for MI355X: sparsify-and-sweep preconditioned GMRES for the
discretized Lippmann-Schwinger equation (Liu & Ying, "Sparsify and sweep: an
efficient preconditioner for the Lippmann-Schwinger equation").

Python front of the HIP library liblsweep.so. Tensors live on the GPU; the
library receives their device pointers and the current HIP stream. Every
step of the solve (FFT operator, stencils, slice factorizations, sweep,
Krylov updates) runs in the library's kernels.

    solver = LSSolver(m, omega, pml_width=12, layer_thickness=4, precision="fp64")
    u, info = solver.solve(u_inc)             # scattered fields, [k][n][n] complex128
    grad = solver.adjoint(resid)              # dJ/dm for J = 1/2 sum |R u - d|^2

``LSSolve.apply(m, u_inc, omega, ...)`` wraps setup + solve as a
torch.autograd.Function whose backward is the adjoint solve.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import _lib
from ._lib import (LS_FP64, LS_MIXED, LS_RHS_INCIDENT, LS_RHS_SOURCE, LsError, LsGrid, LsOptions,
                   LsRhsInfo, LsSetupInfo)

__all__ = ["LSSolver", "LSSolve", "LSOperator3", "RhsInfo", "LsError", "host_tables", "host_green3",
           "host_tables3", "layer_candidates", "stencil_cache"]

_PRECISIONS = {"fp64": LS_FP64, "mixed": LS_MIXED}


@dataclasses.dataclass
class RhsInfo:
    iterations: int
    rel_residual: float
    converged: bool


def _stream_ptr() -> int:
    return torch.cuda.current_stream().cuda_stream


def _need(t: torch.Tensor, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


def layer_candidates(n: int, pml_width: int):
    """Layer thicknesses w >= 2 whose slices all fit the slice kernels (host only)."""
    lib = _lib.load()
    cnt = _lib.c_int()
    _lib.check(lib.ls_layer_candidates(n, pml_width, None, 0, ctypes_byref(cnt)), "ls_layer_candidates")
    out = (_lib.c_int * max(1, cnt.value))()
    _lib.check(lib.ls_layer_candidates(n, pml_width, out, cnt.value, ctypes_byref(cnt)), "ls_layer_candidates")
    return list(out[:cnt.value])


class LSSolver:
    """One setup (Algorithm 1) for a medium m; any number of solves."""

    def __init__(self, m: torch.Tensor, omega: float, pml_width: int = 12, layer_thickness: Optional[int] = 4,
                 precision: str = "fp64", restart: int = 30, max_iters: int = 1000, pml_C: float = 10.0,
                 freq_samples: int = 0, schedule: str = "interface", autotune: int = 0, fronts: int = 1,
                 block_size: int = 1):
        """layer_thickness None (with autotune = k > 0): chosen by timing solves of k
        plane waves on the device; autotune = k > 0 also tunes the kernel choice per
        batch size up to k (ls_setup, Autotuning). block_size > 1: block flexible
        GMRES over groups of that many right-hand sides (restart and max_iters then
        count block steps)."""
        self._lib = _lib.load()
        if m.dim() not in (2, 3) or len(set(m.shape)) != 1:
            raise ValueError("m must be [n, n] or [n, n, n]")
        self.dim = m.dim()
        self.n = int(m.shape[0])
        self.omega = float(omega)
        self.precision = precision
        m = _need(m, torch.float64, (self.n,) * self.dim, "m")
        opts = LsOptions()
        self._lib.ls_default_options(ctypes_byref(opts))
        opts.precision = _PRECISIONS[precision]
        opts.restart = restart
        opts.max_iters = max_iters
        opts.pml_C = pml_C
        opts.freq_samples = freq_samples
        opts.sweep_schedule = {"interface": 0, "sequential": 1}[schedule]
        opts.autotune = int(autotune)
        opts.fronts = int(fronts)
        opts.block_size = int(block_size)
        opts.hip_stream = _stream_ptr()
        self._opts = opts
        grid = LsGrid(self.dim, self.n)
        handle = _lib.c_void_p()
        _lib.check(self._lib.ls_setup(ctypes_byref(grid), self.omega, m.data_ptr(), pml_width,
                                      0 if layer_thickness is None else int(layer_thickness),
                                      ctypes_byref(opts), ctypes_byref(handle)), "ls_setup")
        self._h = handle
        info = LsSetupInfo()
        _lib.check(self._lib.ls_get_info(self._h, ctypes_byref(info)), "ls_get_info")
        self.info = info
        self.L = info.L
        self.nslices = info.nslices
        self.pml_width = pml_width
        self.layer_thickness = info.layer_thickness

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.ls_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- solves ----------------------------------------------------------
    def _cdtype(self, precision: Optional[str]):
        p = precision or self.precision
        return (torch.complex128, LS_FP64) if p == "fp64" else (torch.complex64, LS_MIXED)

    def solve(self, rhs: torch.Tensor, kind: str = "incident", tol: float = 1e-6, allow_noconv: bool = False):
        """Scattered fields u for a batch [k][n][n] (complex128) of incident
        waves (kind="incident") or right-hand sides g (kind="source")."""
        k = rhs.shape[0]
        rhs = _need(rhs, torch.complex128, (k,) + self.grid_shape, "rhs")
        u = torch.empty_like(rhs)
        infos = (LsRhsInfo * k)()
        st = self._lib.ls_solve(self._h, rhs.data_ptr(), k, LS_RHS_INCIDENT if kind == "incident" else LS_RHS_SOURCE,
                                float(tol), u.data_ptr(), infos)
        if not (allow_noconv and st == _lib.LS_E_NOCONV):
            _lib.check(st, "ls_solve")
        return u, [RhsInfo(i.iterations, i.rel_residual, bool(i.converged)) for i in infos]

    def adjoint(self, resid: torch.Tensor, tol: float = 1e-10):
        """dJ/dm for residuals r_j = R^T (R u_j - d_j) of the last solve."""
        k = resid.shape[0]
        resid = _need(resid, torch.complex128, (k,) + self.grid_shape, "resid")
        grad = torch.empty(self.grid_shape, dtype=torch.float64, device=resid.device)
        infos = (LsRhsInfo * k)()
        _lib.check(self._lib.ls_adjoint(self._h, resid.data_ptr(), k, float(tol), grad.data_ptr(), infos),
                   "ls_adjoint")
        return grad, [RhsInfo(i.iterations, i.rel_residual, bool(i.converged)) for i in infos]

    # -- single operators --------------------------------------------------
    def _unary(self, fn, name, x, out_shape, precision):
        dt, code = self._cdtype(precision)
        k = x.shape[0]
        x = _need(x, dt, x.shape, name)
        y = torch.empty(out_shape(k), dtype=dt, device=x.device)
        _lib.check(fn(self._h, x.data_ptr(), k, y.data_ptr(), code), name)
        return y

    @property
    def grid_shape(self):
        return (self.n,) * self.dim

    @property
    def ext_shape(self):
        return (self.L,) * self.dim

    def apply_A(self, x, precision=None):
        return self._unary(self._lib.ls_apply_A, "ls_apply_A", x, lambda k: (k,) + self.grid_shape, precision)

    def apply_K(self, x, precision=None):
        return self._unary(self._lib.ls_apply_K, "ls_apply_K", x, lambda k: (k,) + self.grid_shape, precision)

    def apply_Q(self, r, precision=None):
        return self._unary(self._lib.ls_apply_Q, "ls_apply_Q", r, lambda k: (k,) + self.ext_shape, precision)

    def apply_H(self, u, precision=None):
        return self._unary(self._lib.ls_apply_H, "ls_apply_H", u, lambda k: (k,) + self.ext_shape, precision)

    def apply_B(self, f, precision=None):
        """beta^* f_mu on I^h (the direct scheme's right-hand side, Sec. 4)."""
        return self._unary(self._lib.ls_apply_B, "ls_apply_B", f, lambda k: (k,) + self.ext_shape, precision)

    def solve_H(self, rhs: torch.Tensor, tol: float = 1e-10, allow_noconv: bool = False):
        """u with H u = rhs on the extended grid [k][L][L] (complex128): the
        sparse system itself, preconditioned by the sweep (ls_solve_H)."""
        k = rhs.shape[0]
        rhs = _need(rhs, torch.complex128, (k,) + self.ext_shape, "rhs")
        u = torch.empty_like(rhs)
        infos = (LsRhsInfo * k)()
        st = self._lib.ls_solve_H(self._h, rhs.data_ptr(), k, float(tol), u.data_ptr(), infos)
        if not (allow_noconv and st == _lib.LS_E_NOCONV):
            _lib.check(st, "ls_solve_H")
        return u, [RhsInfo(i.iterations, i.rel_residual, bool(i.converged)) for i in infos]

    def apply_precond(self, r, precision=None):
        return self._unary(self._lib.ls_apply_precond, "ls_apply_precond", r, lambda k: (k,) + self.grid_shape,
                           precision)

    def slice_bounds(self, k: int):
        a, b, c = _lib.c_int(), _lib.c_int(), _lib.c_int()
        _lib.check(self._lib.ls_get_slice(self._h, k, ctypes_byref(a), ctypes_byref(b), ctypes_byref(c)),
                   "ls_get_slice")
        return a.value, b.value, c.value

    def slice_solve(self, k: int, v: torch.Tensor, precision=None):
        dt, code = self._cdtype(precision)
        lo, hi, _ = self.slice_bounds(k)
        nb = v.shape[0]
        v = _need(v, dt, (nb, hi - lo + 1) + (self.L,) * (self.dim - 1), "v")
        w = torch.empty_like(v)
        _lib.check(self._lib.ls_slice_solve(self._h, k, v.data_ptr(), nb, w.data_ptr(), code), "ls_slice_solve")
        return w

    # -- autotuning ---------------------------------------------------------
    def tuning(self):
        """What the autotuner measured: {"layers": [(w, nslices, iterations, setup_ms,
        solve_ms)], "kernels": [(nrhs, slice_kernel, iface_kernel, apply_ms)]}."""
        nw, nk = _lib.c_int(), _lib.c_int()
        _lib.check(self._lib.ls_get_tuning(self._h, None, 0, ctypes_byref(nw), None, 0, ctypes_byref(nk)),
                   "ls_get_tuning")
        ws = (_lib.LsTuneLayer * max(1, nw.value))()
        ks = (_lib.LsTuneKernels * max(1, nk.value))()
        _lib.check(self._lib.ls_get_tuning(self._h, ws, nw.value, ctypes_byref(nw), ks, nk.value,
                                           ctypes_byref(nk)), "ls_get_tuning")
        return {"layers": [(w.layer_thickness, w.nslices, w.iterations, w.setup_ms, w.solve_ms)
                           for w in ws[:nw.value]],
                "kernels": [(k.nrhs, k.slice_kernel, k.iface_kernel, k.apply_ms) for k in ks[:nk.value]]}

    def set_kernels(self, nrhs: int, slice_kernel: int, iface_kernel: int):
        """Force the kernel choice for batches of nrhs (0: every batch size)."""
        _lib.check(self._lib.ls_set_kernels(self._h, nrhs, slice_kernel, iface_kernel), "ls_set_kernels")

    # -- kernel timing ------------------------------------------------------
    def profile(self, enable: bool = True):
        """Start (clear) or stop recording HIP events around the library's launches."""
        _lib.check(self._lib.ls_profile(self._h, 1 if enable else 0), "ls_profile")

    def profile_read(self):
        """{kind: (launches, total_ms, columns)} of the recorded launches; columns
        is the number of right-hand-side columns they processed in total."""
        out = (_lib.LsKernelTime * 16)()
        cnt = _lib.c_int()
        _lib.check(self._lib.ls_profile_read(self._h, out, 16, ctypes_byref(cnt)), "ls_profile_read")
        return {out[i].name.decode(): (out[i].launches, out[i].total_ms, out[i].columns) for i in range(cnt.value)}

    # -- setup tables -------------------------------------------------------
    def stencils(self):
        import numpy as np
        b, ns, d = self.pml_width, self.info.freq_samples, self.dim
        nc = 2 * b + 1
        mu = 3 ** d
        a = np.zeros(2 * mu)
        be = np.zeros(2 * mu)
        g = np.zeros(nc ** d * mu * 2)
        ax = np.zeros(b * nc ** (d - 1) * ns * mu * 2)
        _lib.check(self._lib.ls_get_stencils(self._h, a.ctypes.data, be.ctypes.data, g.ctypes.data, ax.ctypes.data),
                   "ls_get_stencils")
        c = lambda v: v.view(np.complex128)
        return (c(a), c(be), c(g).reshape((nc,) * d + (mu,)),
                c(ax).reshape((b,) + (nc,) * (d - 1) + (ns, mu)))

    def sample_map(self):
        import numpy as np
        km = np.zeros(self.ext_shape, dtype=np.int32)
        _lib.check(self._lib.ls_get_sample_map(self._h, km.ctypes.data), "ls_get_sample_map")
        return km


class LSOperator3:
    """The 3D operator A = I + omega^2 K M on [n]^3 (Sec. 1 and Sec. 2.1 with
    d = 3) applied by a zero-padded FFT convolution on the device."""

    def __init__(self, m: torch.Tensor, omega: float):
        self._lib = _lib.load()
        if m.dim() != 3 or not (m.shape[0] == m.shape[1] == m.shape[2]):
            raise ValueError("m must be [n, n, n]")
        self.n = int(m.shape[0])
        self.omega = float(omega)
        m = _need(m, torch.float64, (self.n,) * 3, "m")
        handle = _lib.c_void_p()
        _lib.check(self._lib.ls_op3_create(self.n, self.omega, m.data_ptr(), _stream_ptr(), ctypes_byref(handle)),
                   "ls_op3_create")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ls_op3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _apply(self, fn, name, x, precision):
        dt, code = (torch.complex128, LS_FP64) if precision == "fp64" else (torch.complex64, LS_MIXED)
        k = x.shape[0]
        x = _need(x, dt, (k, self.n, self.n, self.n), name)
        y = torch.empty_like(x)
        _lib.check(fn(self._h, x.data_ptr(), k, y.data_ptr(), code), name)
        return y

    def apply_A(self, x, precision="fp64"):
        return self._apply(self._lib.ls_op3_apply_A, "ls_op3_apply_A", x, precision)

    def apply_K(self, x, precision="fp64"):
        return self._apply(self._lib.ls_op3_apply_K, "ls_op3_apply_K", x, precision)


def host_green3(n: int, omega: float):
    """The 3D Green's table octant k_delta, delta in [0, n+1]^3 (host only)."""
    import numpy as np
    g = np.zeros((n + 2) ** 3 * 2)
    _lib.check(_lib.load().ls_host_green3(int(n), float(omega), g.ctypes.data), "ls_host_green3")
    return g.view(np.complex128).reshape(n + 2, n + 2, n + 2)


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)


def host_tables(m, omega: float, pml_width: int, layer_thickness: int, pml_C: float = 10.0,
                freq_samples: int = 0):
    """The library's float64 setup tables computed on the host (no GPU):
    alpha, beta, gamma [(2b+1)][(2b+1)][9], aux [b][(2b+1)][ns][9],
    kmap [L][L], green quadrant [(n+2)][(n+2)]."""
    import numpy as np
    lib = _lib.load()
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = m.shape[0]
    b = pml_width
    nc = 2 * b + 1
    L = n + 2 + 2 * b
    ns = freq_samples if freq_samples > 0 else n
    if m.max() == m.min():
        ns = 1
    a = np.zeros(18)
    be = np.zeros(18)
    g = np.zeros(nc * nc * 18)
    ax = np.zeros(b * nc * ns * 18)
    km = np.zeros((L, L), dtype=np.int32)
    gr = np.zeros((n + 2) * (n + 2) * 2)
    _lib.check(lib.ls_host_tables(n, float(omega), m.ctypes.data, b, layer_thickness, float(pml_C), freq_samples,
                                  a.ctypes.data, be.ctypes.data, g.ctypes.data, ax.ctypes.data, km.ctypes.data,
                                  gr.ctypes.data), "ls_host_tables")
    c = lambda v: v.view(np.complex128)
    return dict(alpha=c(a), beta=c(be), gamma=c(g).reshape(nc, nc, 9), aux=c(ax).reshape(b, nc, ns, 9),
                kmap=km, green=c(gr).reshape(n + 2, n + 2))


def stencil_cache(clear: bool = False):
    """(hits, misses) of the stencil cache (the m-independent setup tables,
    2D and 3D) since the last clear; clear=True empties it afterwards."""
    import ctypes
    lib = _lib.load()
    hits, misses = ctypes.c_longlong(0), ctypes.c_longlong(0)
    _lib.check(lib.ls_stencil_cache(1 if clear else 0, ctypes.byref(hits), ctypes.byref(misses)),
               "ls_stencil_cache")
    return hits.value, misses.value


def host_tables3(m, omega: float, pml_width: int, layer_thickness: int, pml_C: float = 10.0,
                 freq_samples: int = 0):
    """The library's float64 3D setup tables computed on the host (no GPU):
    alpha, beta [27], gamma [(2b+1)^3][27], aux [b][(2b+1)^2][ns][27], kmap [L]^3."""
    import numpy as np
    lib = _lib.load()
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = m.shape[0]
    b = pml_width
    nc = 2 * b + 1
    L = n + 2 + 2 * b
    ns = freq_samples if freq_samples > 0 else n
    if m.max() == m.min():
        ns = 1
    a = np.zeros(54)
    be = np.zeros(54)
    g = np.zeros(nc ** 3 * 54)
    ax = np.zeros(b * nc * nc * ns * 54)
    km = np.zeros((L, L, L), dtype=np.int32)
    _lib.check(lib.ls_host_tables3(n, float(omega), m.ctypes.data, b, layer_thickness, float(pml_C), freq_samples,
                                   a.ctypes.data, be.ctypes.data, g.ctypes.data, ax.ctypes.data, km.ctypes.data),
               "ls_host_tables3")
    c = lambda v: v.view(np.complex128)
    return dict(alpha=c(a), beta=c(be), gamma=c(g).reshape(nc, nc, nc, 27),
                aux=c(ax).reshape(b, nc, nc, ns, 27), kmap=km)


class LSSolve(torch.autograd.Function):
    """u = LSSolve.apply(m, u_inc, omega, pml_width, layer_thickness, precision, tol, adjoint_tol):
    scattered fields for incident waves u_inc [k][n][n]; backward gives dJ/dm
    through one adjoint solve with the same preconditioner."""

    @staticmethod
    def forward(ctx, m, u_inc, omega, pml_width=12, layer_thickness=4, precision="fp64", tol=1e-6,
                adjoint_tol=1e-10):
        solver = LSSolver(m.detach(), omega, pml_width, layer_thickness, precision)
        u, _ = solver.solve(u_inc.detach(), "incident", tol)
        ctx.solver = solver
        ctx.adjoint_tol = adjoint_tol
        return u

    @staticmethod
    def backward(ctx, grad_u):
        # For a real loss torch passes the conjugate-Wirtinger cotangent; for
        # J = 1/2 sum |R u - d|^2 it is R^T (R u - d), the residual the adjoint takes.
        # The handle stays open while the graph lives: backward may run more
        # than once (retain_graph, gradcheck); it is released with ctx.
        grad_m, _ = ctx.solver.adjoint(grad_u.contiguous().to(torch.complex128), ctx.adjoint_tol)
        return grad_m, None, None, None, None, None, None, None
