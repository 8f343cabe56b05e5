"""Python binding of libmgkkt, the MI355X all-at-once multigrid solver for the
Poisson-control KKT system of Takacs (arXiv 1502.03917), eq. mp2.

Argument marshalling only: every step of the solver runs in the HIP kernels of
``csrc/`` behind the C ABI of ``include/mgkkt.h``.  PyTorch supplies device
memory (FP64 CUDA tensors) and the current stream.  If ``libmgkkt.so`` is
missing the import of :func:`lib` raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgkkt.so")

MG_POISSON, MG_STOKES = 0, 1
MG_NE, MG_LSGS, MG_SLSGS, MG_CGS, MG_VANKA = 0, 1, 2, 3, 4
MG_FP64, MG_FP32_IR = 0, 1
MG_OK, MG_EINVAL, MG_EHIP, MG_ENOMEM, MG_ENOTCONV, MG_ENAN, MG_EDIVERGE, MG_EUNSUPPORTED, MG_ESTALL = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
MG_NORM_L2, MG_NORM_LINV = 0, 1
NORMS = {"l2": MG_NORM_L2, "linv": MG_NORM_LINV}

SMOOTHERS = {"ne": MG_NE, "lsgs": MG_LSGS, "slsgs": MG_SLSGS, "cgs": MG_CGS, "vanka": MG_VANKA}
PRECISIONS = {"fp64": MG_FP64, "fp32_ir": MG_FP32_IR}
PROBLEMS = {"poisson": MG_POISSON, "stokes": MG_STOKES}


class MgOpts(ctypes.Structure):
    _fields_ = [
        ("smoother", ctypes.c_int),
        ("nu1", ctypes.c_int),
        ("nu2", ctypes.c_int),
        ("gamma", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("coarse_level", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("max_cycles", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("norm", ctypes.c_int),
    ]


class MGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {lib().mg_strerror(status).decode()} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def lib():
    """The loaded libmgkkt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmgkkt.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.mg_default_opts.restype = MgOpts
    L.mg_default_opts.argtypes = [ip]
    L.mg_setup.argtypes = [ip, dp, ip, ctypes.POINTER(MgOpts), ctypes.POINTER(vp)]
    L.mg_destroy.argtypes = [vp]
    L.mg_destroy.restype = None
    L.mg_vec_len.argtypes = [vp]
    L.mg_vec_len.restype = sz
    L.mg_level_len.argtypes = [vp, ip]
    L.mg_level_len.restype = sz
    L.mg_get_opts.argtypes = [vp, ctypes.POINTER(MgOpts)]
    L.mg_set_opts.argtypes = [vp, ctypes.POINTER(MgOpts)]
    L.mg_rhs.argtypes = [vp, vp, vp, vp]
    L.mg_control.argtypes = [vp, vp, vp, vp]
    L.mg_adjoint_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mg_apply.argtypes = [vp, ip, vp, vp, vp]
    L.mg_residual.argtypes = [vp, ip, vp, vp, vp, ctypes.POINTER(dp), vp]
    L.mg_residual_nalloc.argtypes = [vp, ip, vp, vp, vp, vp, vp]
    L.mg_smooth.argtypes = [vp, ip, vp, vp, ip, vp]
    L.mg_restrict.argtypes = [vp, ip, vp, vp, vp]
    L.mg_prolong_add.argtypes = [vp, ip, vp, vp, vp]
    L.mg_coarse_solve.argtypes = [vp, vp, vp, vp]
    L.mg_cycle.argtypes = [vp, vp, vp, vp]
    L.mg_capture_cycle.argtypes = [vp, vp, vp, vp, ctypes.POINTER(vp)]
    L.mg_graph_launch.argtypes = [vp, vp]
    L.mg_graph_destroy.argtypes = [vp]
    L.mg_graph_destroy.restype = None
    L.mg_solve.argtypes = [vp, vp, vp, dp, ctypes.POINTER(ip), ctypes.POINTER(dp), vp]
    L.mg_timing_enable.argtypes = [vp, ip]
    L.mg_timing_read.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_long)]
    L.mg_batch_setup.argtypes = [ip, ctypes.POINTER(ip), ctypes.POINTER(dp), ip, ctypes.POINTER(MgOpts),
                                 ctypes.POINTER(vp)]
    L.mg_batch_setup.restype = ip
    L.mg_batch_destroy.argtypes = [vp]
    L.mg_batch_destroy.restype = None
    L.mg_batch_count.argtypes = [vp]
    L.mg_batch_count.restype = ip
    L.mg_batch_vec_len.argtypes = [vp, ip]
    L.mg_batch_vec_len.restype = sz
    L.mg_batch_sweep_tile.argtypes = [vp, ip]
    L.mg_batch_sweep_tile.restype = ip
    L.mg_batch_rhs.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.mg_batch_rhs.restype = ip
    L.mg_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), dp, ctypes.POINTER(ip),
                                 ctypes.POINTER(dp), ctypes.POINTER(ip), vp]
    L.mg_batch_solve.restype = ip
    L.mg_batch_last_error.argtypes = [vp]
    L.mg_batch_last_error.restype = ctypes.c_char_p
    L.mg_strerror.restype = ctypes.c_char_p
    L.mg_strerror.argtypes = [ip]
    L.mg_last_error.restype = ctypes.c_char_p
    L.mg_last_error.argtypes = [vp]
    for name in ("mg_setup", "mg_get_opts", "mg_set_opts", "mg_rhs", "mg_control", "mg_adjoint_grad", "mg_apply", "mg_residual", "mg_residual_nalloc", "mg_smooth",
                 "mg_restrict", "mg_prolong_add", "mg_coarse_solve", "mg_cycle", "mg_capture_cycle", "mg_graph_launch", "mg_solve", "mg_timing_enable",
                 "mg_timing_read"):
        getattr(L, name).restype = ip
    _lib = L
    return L


def default_opts(problem: str = "poisson") -> MgOpts:
    return lib().mg_default_opts(PROBLEMS[problem])


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One solver context: level k (n = 2^k cells per side), alpha, options.

    Tensors passed in are FP64 CUDA tensors on the context's device, contiguous,
    of length ``level_len(level)`` (2 (2^level+1)^2, field-major [y | lambda]).
    """

    def __init__(self, level: int, alpha: float, problem: str = "poisson", smoother: str = "lsgs", nu1: int = 2,
                 nu2: int = 2, gamma: int = 1, tau: float | None = None, coarse_level: int = 1,
                 precision: str = "fp64", max_cycles: int = 200, inner_cycles: int = 1, norm: str = "linv"):
        L = lib()
        o = L.mg_default_opts(PROBLEMS[problem])
        o.smoother = SMOOTHERS[smoother]
        o.nu1, o.nu2, o.gamma = nu1, nu2, gamma
        o.tau = -1.0 if tau is None else float(tau)
        o.coarse_level = coarse_level
        o.precision = PRECISIONS[precision]
        o.max_cycles = max_cycles
        o.inner_cycles = inner_cycles
        o.norm = NORMS[norm]
        h = ctypes.c_void_p()
        st = L.mg_setup(level, float(alpha), PROBLEMS[problem], ctypes.byref(o), ctypes.byref(h))
        if st != MG_OK:
            raise MGError(st, "mg_setup")
        self._h = h
        self.level, self.alpha, self.coarse_level = level, float(alpha), coarse_level
        self.problem = problem

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------------
    def _check(self, st: int, where: str):
        if st != MG_OK:
            raise MGError(st, where, lib().mg_last_error(self._h).decode())

    def _t(self, t, n: int, name: str):
        import torch

        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError(f"{name}: expected a contiguous float64 CUDA tensor")
        if t.numel() != n:
            raise ValueError(f"{name}: expected {n} entries, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    def vec_len(self) -> int:
        return int(lib().mg_vec_len(self._h))

    def level_len(self, level: int) -> int:
        return int(lib().mg_level_len(self._h, level))

    def nvert(self, level: int | None = None) -> int:
        return self.level_len(self.level if level is None else level) // 2

    def opts(self) -> MgOpts:
        o = MgOpts()
        self._check(lib().mg_get_opts(self._h, ctypes.byref(o)), "mg_get_opts")
        return o

    def set_opts(self, **kw):
        o = self.opts()
        for k, v in kw.items():
            if k == "smoother":
                v = SMOOTHERS[v]
            elif k == "precision":
                v = PRECISIONS[v]
            elif k == "norm":
                v = NORMS[v]
            elif k == "tau" and v is None:
                v = -1.0
            setattr(o, k, v)
        self._check(lib().mg_set_opts(self._h, ctypes.byref(o)), "mg_set_opts")

    def _empty(self, n: int):
        import torch

        return torch.empty(n, dtype=torch.float64, device="cuda")

    # -- entry points -------------------------------------------------------------
    def data_len(self) -> int:
        """Length of the data of mg_rhs: y_D at the (2^l+1)^2 vertices (Poisson)
        or [v1 | v2] at the (2^(l+1)-1)^2 interior P2 nodes (Stokes)."""
        if self.problem == "stokes":
            return 2 * ((1 << (self.level + 1)) - 1) ** 2
        return self.nvert()

    def rhs(self, yd, f=None):
        f = self._empty(self.vec_len()) if f is None else f
        self._check(lib().mg_rhs(self._h, self._t(yd, self.data_len(), "yd"), self._t(f, self.vec_len(), "f"), _stream()),
                    "mg_rhs")
        return f

    def control(self, x, u=None):
        """u = lambda / alpha (section 1)."""
        u = self._empty(self.nvert()) if u is None else u
        self._check(lib().mg_control(self._h, self._t(x, self.vec_len(), "x"), self._t(u, self.nvert(), "u"), _stream()),
                    "mg_control")
        return u

    def adjoint_grad(self, x, xadj, grad_yd=None, grad_alpha=None):
        """(M x_adj^y, -alpha^-2 (x_adj^lambda)^T M lambda) as device tensors."""
        g = self._empty(self.nvert()) if grad_yd is None else grad_yd
        a = self._empty(1) if grad_alpha is None else grad_alpha
        st = lib().mg_adjoint_grad(self._h, self._t(x, self.vec_len(), "x"), self._t(xadj, self.vec_len(), "xadj"),
                                   self._t(g, self.nvert(), "grad_yd"), self._t(a, 1, "grad_alpha"), _stream())
        self._check(st, "mg_adjoint_grad")
        return g, a

    def apply(self, x, level: int | None = None, y=None):
        l = self.level if level is None else level
        n = self.level_len(l)
        y = self._empty(n) if y is None else y
        self._check(lib().mg_apply(self._h, l, self._t(x, n, "x"), self._t(y, n, "y"), _stream()), "mg_apply")
        return y

    def residual(self, f, x, level: int | None = None, r=None, norm: bool = False):
        l = self.level if level is None else level
        n = self.level_len(l)
        r = self._empty(n) if r is None else r
        nrm = ctypes.c_double(0.0)
        st = lib().mg_residual(self._h, l, self._t(f, n, "f"), self._t(x, n, "x"), self._t(r, n, "r"),
                               ctypes.byref(nrm) if norm else None, _stream())
        self._check(st, "mg_residual")
        return (r, nrm.value) if norm else r

    def residual_nalloc(self, f, x, r, norm, level: int | None = None):
        """mg_residual_nalloc: r = f - A x and ||r||_2 written to the one-entry
        device tensor `norm`, stream-ordered; the library allocates nothing."""
        l = self.level if level is None else level
        n = self.level_len(l)
        st = lib().mg_residual_nalloc(self._h, l, self._t(f, n, "f"), self._t(x, n, "x"), self._t(r, n, "r"),
                                      self._t(norm, 1, "norm"), _stream())
        self._check(st, "mg_residual_nalloc")
        return r, norm

    def smooth(self, x, r, steps: int = 1, level: int | None = None):
        l = self.level if level is None else level
        n = self.level_len(l)
        self._check(lib().mg_smooth(self._h, l, self._t(x, n, "x"), self._t(r, n, "r"), steps, _stream()), "mg_smooth")

    def restrict(self, r, level: int | None = None, fc=None):
        l = self.level if level is None else level
        fc = self._empty(self.level_len(l - 1)) if fc is None else fc
        st = lib().mg_restrict(self._h, l, self._t(r, self.level_len(l), "r"), self._t(fc, self.level_len(l - 1), "fc"), _stream())
        self._check(st, "mg_restrict")
        return fc

    def prolong_add(self, xc, x, level: int | None = None):
        l = self.level if level is None else level
        st = lib().mg_prolong_add(self._h, l, self._t(xc, self.level_len(l - 1), "xc"), self._t(x, self.level_len(l), "x"), _stream())
        self._check(st, "mg_prolong_add")
        return x

    def coarse_solve(self, f, x=None):
        n = self.level_len(self.coarse_level)
        x = self._empty(n) if x is None else x
        self._check(lib().mg_coarse_solve(self._h, self._t(f, n, "f"), self._t(x, n, "x"), _stream()), "mg_coarse_solve")
        return x

    def cycle(self, f, x):
        n = self.vec_len()
        self._check(lib().mg_cycle(self._h, self._t(f, n, "f"), self._t(x, n, "x"), _stream()), "mg_cycle")
        return x

    def capture_cycle(self, f, x) -> "CycleGraph":
        """mg_cycle(f, x) recorded as a HIP graph; CycleGraph.launch() replays it."""
        n = self.vec_len()
        g = ctypes.c_void_p()
        st = lib().mg_capture_cycle(self._h, self._t(f, n, "f"), self._t(x, n, "x"), _stream(), ctypes.byref(g))
        self._check(st, "mg_capture_cycle")
        return CycleGraph(self, g, f, x)

    def solve(self, f, x=None, tol: float = 1e-10, raise_on_error: bool = True):
        """Returns (x, cycles, relres, status)."""
        import torch

        n = self.vec_len()
        if x is None:
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        st = lib().mg_solve(self._h, self._t(f, n, "f"), self._t(x, n, "x"), float(tol), ctypes.byref(it),
                            ctypes.byref(rel), _stream())
        if st != MG_OK and raise_on_error:
            self._check(st, "mg_solve")
        return x, it.value, rel.value, st

    def timing_enable(self, on: bool = True):
        self._check(lib().mg_timing_enable(self._h, int(on)), "mg_timing_enable")

    def timing_read(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_long(0)
        self._check(lib().mg_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)), "mg_timing_read")
        return ms.value, n.value


# --- batches of independent instances ----------------------------------------------

class CycleGraph:
    """Caller-owned graph of one iterate of a Solver (mg_capture_cycle).  It
    keeps the solver and the captured f and x alive and is destroyed before
    them."""

    def __init__(self, solver: Solver, handle, f, x):
        self._solver, self._g, self.f, self.x = solver, handle, f, x

    def launch(self):
        if not self._g or not self._solver._h:
            raise RuntimeError("CycleGraph.launch: graph or solver already closed")
        self._solver._check(lib().mg_graph_launch(self._g, _stream()), "mg_graph_launch")
        return self.x

    def close(self):
        if self._g:
            lib().mg_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent instances (level_i, alpha_i) solved together (mg_batch_*)."""

    def __init__(self, levels, alphas, smoother: str = "lsgs", precision: str = "fp64", **kw):
        o = default_opts("poisson")
        o.smoother = SMOOTHERS[smoother]
        o.precision = PRECISIONS[precision]
        for k, v in kw.items():
            setattr(o, k, NORMS[v] if k == "norm" else v)
        self.levels = [int(l) for l in levels]
        self.alphas = [float(a) for a in alphas]
        n = len(self.levels)
        self._h = ctypes.c_void_p()
        st = lib().mg_batch_setup(n, (ctypes.c_int * n)(*self.levels), (ctypes.c_double * n)(*self.alphas),
                                  MG_POISSON, ctypes.byref(o), ctypes.byref(self._h))
        if st != MG_OK:
            raise MGError(st, "mg_batch_setup")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return lib().mg_batch_count(self._h)

    def vec_len(self, i: int) -> int:
        return lib().mg_batch_vec_len(self._h, i)

    def sweep_tile(self, level: int) -> int:
        """Tile edge the setup's autotuner picked for the batched sweep on `level`."""
        return lib().mg_batch_sweep_tile(self._h, level)

    def _ptrs(self, ts, lens, name):
        import torch

        n = len(self)
        if len(ts) != n:
            raise ValueError(f"{name}: expected {n} tensors")
        for t, m in zip(ts, lens):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == m):
                raise ValueError(f"{name}: contiguous FP64 CUDA tensors of the instance sizes required")
        return (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])

    def rhs(self, yds):
        import torch

        n = len(self)
        fs = [torch.empty(self.vec_len(i), dtype=torch.float64, device="cuda") for i in range(n)]
        st = lib().mg_batch_rhs(self._h, self._ptrs(yds, [self.vec_len(i) // 2 for i in range(n)], "yd"),
                                self._ptrs(fs, [self.vec_len(i) for i in range(n)], "f"), _stream())
        if st != MG_OK:
            raise MGError(st, "mg_batch_rhs", lib().mg_batch_last_error(self._h).decode())
        return fs

    def solve(self, fs, xs=None, tol: float = 1e-10, raise_on_error: bool = True):
        """Returns (xs, cycles, relres, statuses, status)."""
        import torch

        n = len(self)
        lens = [self.vec_len(i) for i in range(n)]
        if xs is None:
            xs = [torch.zeros(m, dtype=torch.float64, device="cuda") for m in lens]
        cyc = (ctypes.c_int * n)()
        rel = (ctypes.c_double * n)()
        sts = (ctypes.c_int * n)()
        st = lib().mg_batch_solve(self._h, self._ptrs(fs, lens, "f"), self._ptrs(xs, lens, "x"), float(tol), cyc, rel,
                                  sts, _stream())
        if st != MG_OK and raise_on_error:
            raise MGError(st, "mg_batch_solve", lib().mg_batch_last_error(self._h).decode())
        return xs, list(cyc), list(rel), list(sts), st


# --- differentiable solve ---------------------------------------------------------

# A stall (MG_ESTALL: no factor 2 gained over 10 iterates) is accepted as
# convergence only when the relative residual reached is at the FP64 rounding
# floor of the solve, at most STALL_FLOOR (or tol, if larger); above it the
# differentiable solve raises instead of returning an unconverged x.
STALL_FLOOR = 1e-11


def check_solve_status(status: int, relres: float, tol: float) -> None:
    """Raise MGError unless a solve ended in success, or in a stall at or below
    max(tol, STALL_FLOOR)."""
    if status == MG_OK:
        return
    if status == MG_ESTALL and relres <= max(tol, STALL_FLOOR):
        return
    raise MGError(status, "mg_solve", f"relative residual {relres:.3e} (tol {tol:.1e})")


def _solve_or_raise(solver: "Solver", f, tol: float):
    import torch

    x = torch.zeros(solver.vec_len(), dtype=torch.float64, device="cuda")
    x, _, rel, st = solver.solve(f, x, tol=tol, raise_on_error=False)
    check_solve_status(st, rel, tol)
    return x


def _make_function():
    import torch

    class MGSolve(torch.autograd.Function):
        """x = A(alpha)^-1 (M y_D; 0), eq. mp2, with a hand-written backward:
        the adjoint system A x_adj = dLoss/dx (A symmetric) is solved by the
        same multigrid, then dLoss/dy_D = M x_adj^y and
        dLoss/dalpha = -alpha^-2 (x_adj^lambda)^T M lambda."""

        @staticmethod
        def forward(ctx, yd, alpha, solver, tol):
            f = solver.rhs(yd.detach().contiguous())
            x = _solve_or_raise(solver, f, tol)
            ctx.save_for_backward(x)
            ctx.solver, ctx.tol = solver, tol
            ctx.alpha_shape = alpha.shape
            return x

        @staticmethod
        def backward(ctx, gx):
            (x,) = ctx.saved_tensors
            xa = _solve_or_raise(ctx.solver, gx.contiguous(), ctx.tol)
            gyd, ga = ctx.solver.adjoint_grad(x, xa)
            return gyd, ga.reshape(ctx.alpha_shape), None, None

    return MGSolve


_MGSolve = None
# solver contexts of solve(), most recently used last; at most MAX_SOLVERS are
# kept (a context holds the level workspace, hundreds of MB at 1025^2)
MAX_SOLVERS = 4
_SOLVERS: "collections.OrderedDict" = None


def mg_solve_fn():
    """The torch.autograd.Function of the differentiable solve."""
    global _MGSolve
    if _MGSolve is None:
        _MGSolve = _make_function()
    return _MGSolve


def solve(yd, alpha, level: int, tol: float = 1e-12, **opts):
    """Differentiable solve of eq. mp2 for desired state yd ((2^level+1)^2
    nodal values, FP64 CUDA tensor) and alpha (float or 0-d/1-element FP64
    tensor).  Returns (y, lam, u): y and lam are differentiable views of the
    solution; u = lam / alpha is computed by the library and carries no
    gradient (differentiate lam / alpha instead).  Solver contexts are cached
    per (level, alpha, options), the MAX_SOLVERS most recently used; the
    solves raise MGError unless they converge (a stall is accepted only at
    the rounding floor, see check_solve_status)."""
    import collections

    import torch

    global _SOLVERS
    if _SOLVERS is None:
        _SOLVERS = collections.OrderedDict()
    if isinstance(alpha, torch.Tensor):
        a = alpha
        # the context is built for alpha's value: a CUDA tensor costs one
        # device-to-host read here, a float or a CPU tensor none
        aval = float(a.detach().cpu()) if a.is_cuda else float(a.detach())
        if not a.is_cuda:
            a = a.to(dtype=torch.float64, device="cuda")
    else:
        aval = float(alpha)
        a = torch.tensor(aval, dtype=torch.float64, device="cuda")
    key = (level, aval, tuple(sorted(opts.items())))
    s = _SOLVERS.get(key)
    if s is None:
        s = _SOLVERS[key] = Solver(level, aval, **opts)
        while len(_SOLVERS) > MAX_SOLVERS:
            _, old = _SOLVERS.popitem(last=False)
            old.close()
    else:
        _SOLVERS.move_to_end(key)
    x = mg_solve_fn().apply(yd, a, s, tol)
    V = s.nvert()
    with torch.no_grad():
        u = s.control(x.detach())
    return x[:V], x[V:], u
