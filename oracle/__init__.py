"""FP64 CPU oracle for the all-at-once multigrid method (Takacs, arXiv 1502.03917).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers; the product path never
imports this package.  It shares no code with the HIP library: both receive
the same seeded inputs (``workloads``) and nothing else.

The numerical core is plain C (``mgo.c``); this module is a thin ctypes layer
plus a few post-processing steps written with NumPy/SciPy primitives:

* ``rhs``: first block of the right-hand side, M_k times the nodal
  interpolant of y_D (section 1, eq. mp2; reading: interpolate, then apply M).
* ``control``: u = alpha^{-1} lambda (section 1, below eq. mp2).
* ``adjoint_gradient``: for L = 1/2 ||y - y_t||^2, the adjoint solve with the
  same (symmetric) matrix A_k gives dL/dy_D = M x_adj^y and
  dL/dalpha = -alpha^{-2} lambda_adj^T M lambda, since d A_k / d alpha has the
  single block alpha^{-2} M in position (2,2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmgo.so")
_lib = None

NE, LSGS, SLSGS, CGS = 0, 1, 2, 3
ORDER_LEX, ORDER_COL7, ORDER_COL7SEQ, ORDER_VLEX, ORDER_COL3 = 0, 1, 2, 3, 4
SMOOTHERS = {"ne": NE, "lsgs": LSGS, "slsgs": SLSGS, "cgs": CGS}
ORDERS = {"lex": ORDER_LEX, "col7": ORDER_COL7, "col7seq": ORDER_COL7SEQ, "vlex": ORDER_VLEX, "col3": ORDER_COL3}
# damping of the normal-equation smoother used in the paper's experiments
# (section 3): 0.4 for Poisson control, 0.35 for Stokes control
TAU_POISSON, TAU_STOKES = 0.4, 0.35


def build(force: bool = True) -> str:
    """Compile mgo.c into libmgo.so next to this file (plain gcc, FP64)."""
    src = [os.path.join(_HERE, "mgo.c")]
    if os.path.exists(os.path.join(_HERE, "mgo_stokes.c")):
        src.append(os.path.join(_HERE, "mgo_stokes.c"))
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp] + src + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.mgo_create.restype = vp
    lib.mgo_create.argtypes = [ip, ip, ip, dp]
    lib.mgo_destroy.argtypes = [vp]
    lib.mgo_ndof.argtypes = [vp, ip]
    lib.mgo_get_matrix.argtypes = [vp, ip, ip, ctypes.POINTER(ip), ctypes.POINTER(ip), ctypes.POINTER(ip), vp, vp, vp]
    lib.mgo_get_diag.argtypes = [vp, ip, ip, vp]
    lib.mgo_residual.argtypes = [vp, ip, vp, vp, vp]
    lib.mgo_smooth.argtypes = [vp, ip, ip, ip, dp, vp, vp]
    lib.mgo_smooth_groups.argtypes = [vp, ip, vp, vp, ip, ip, vp, vp]
    lib.mgo_coarse_solve.argtypes = [vp, vp, vp]
    lib.mgo_cycle.argtypes = [vp, ip, ip, ip, dp, ip, ip, ip, vp, vp]
    lib.mgo_solve.argtypes = [vp, ip, ip, dp, ip, ip, ip, vp, vp, dp, ip, ip, vp]
    lib.mgo_solve.restype = ip
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


class Hierarchy:
    """Levels coarse..fine of the Poisson control KKT system (eq. mp2).

    Level l has n = 2^l cells per side of the unit square, (n+1)^2 vertices
    and 2 (n+1)^2 unknowns x = (y; lambda), field-major.
    """

    def __init__(self, level: int, alpha: float, coarse: int = 1, problem: int = 0):
        self.lib = _load()
        self.level, self.coarse, self.alpha, self.problem = level, coarse, float(alpha), problem
        h = self.lib.mgo_create(problem, level, coarse, float(alpha))
        if not h:
            raise ValueError(f"oracle: invalid hierarchy (problem={problem}, level={level}, coarse={coarse}, alpha={alpha})")
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mgo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ndof(self, level: int | None = None) -> int:
        return self.lib.mgo_ndof(self._h, self.level if level is None else level)

    def nvert(self, level: int | None = None) -> int:
        l = self.level if level is None else level
        return ((1 << l) + 1) ** 2

    def matrix(self, which: str, level: int | None = None):
        """scipy CSR copy of 'A', 'M', 'Klap', 'P' (level-1 -> level), 'B', 'Mp', 'P2'."""
        import scipy.sparse as sp

        code = {"A": 0, "M": 1, "Klap": 2, "P": 3, "B": 4, "Mp": 5, "P2": 6}[which]
        l = self.level if level is None else level
        nr, nc, nz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        if self.lib.mgo_get_matrix(self._h, l, code, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nz), None, None, None) < 0:
            raise ValueError(f"oracle: no matrix {which} on level {l}")
        rp = np.zeros(nr.value + 1, dtype=np.int32)
        ci = np.zeros(nz.value, dtype=np.int32)
        va = np.zeros(nz.value, dtype=np.float64)
        self.lib.mgo_get_matrix(self._h, l, code, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nz),
                                rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p), _ptr(va))
        return sp.csr_matrix((va, ci, rp), shape=(nr.value, nc.value))

    def K(self, level: int | None = None):
        return (self.matrix("Klap", level) + self.matrix("M", level)).tocsr()

    def Ldiag(self, level: int | None = None) -> np.ndarray:
        out = np.zeros(self.ndof(level))
        self.lib.mgo_get_diag(self._h, self.level if level is None else level, 0, _ptr(out))
        return out

    def Ndiag(self, level: int | None = None) -> np.ndarray:
        out = np.zeros(self.ndof(level))
        self.lib.mgo_get_diag(self._h, self.level if level is None else level, 1, _ptr(out))
        return out

    def residual(self, f, x, level: int | None = None) -> np.ndarray:
        l = self.level if level is None else level
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        r = np.zeros(self.ndof(l))
        self.lib.mgo_residual(self._h, l, _ptr(f), _ptr(x), _ptr(r))
        return r

    def smooth(self, x: np.ndarray, r: np.ndarray, smoother="lsgs", order="col7", tau=None, level=None):
        """One smoothing step in place on (x, r), r = f - A x kept current."""
        l = self.level if level is None else level
        tau = TAU_POISSON if tau is None else tau
        self.lib.mgo_smooth(self._h, l, SMOOTHERS[smoother], ORDERS[order], float(tau), _ptr(x), _ptr(r))

    def smooth_groups(self, x: np.ndarray, r: np.ndarray, groups, reverse=False, level=None):
        """Alg. 2 over an explicit ordering: `groups` is a list of lists of unknowns;
        the unknowns of one group are updated from the same residual."""
        l = self.level if level is None else level
        ord_ = np.ascontiguousarray(np.concatenate([np.asarray(g, dtype=np.int32) for g in groups]), dtype=np.int32)
        gptr = np.zeros(len(groups) + 1, dtype=np.int32)
        gptr[1:] = np.cumsum([len(g) for g in groups])
        self.lib.mgo_smooth_groups(self._h, l, ord_.ctypes.data_as(ctypes.c_void_p), gptr.ctypes.data_as(ctypes.c_void_p),
                                   len(groups), int(reverse), _ptr(x), _ptr(r))

    def coarse_solve(self, f: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.zeros(self.ndof(self.coarse))
        self.lib.mgo_coarse_solve(self._h, _ptr(f), _ptr(x))
        return x

    def cycle(self, f, x, smoother="lsgs", order="col7", tau=None, nu1=2, nu2=2, gamma=1, level=None):
        """One multigrid iterate in place on x (x must be a float64 C array)."""
        l = self.level if level is None else level
        tau = TAU_POISSON if tau is None else tau
        f = np.ascontiguousarray(f, dtype=np.float64)
        self.lib.mgo_cycle(self._h, l, SMOOTHERS[smoother], ORDERS[order], float(tau), nu1, nu2, gamma, _ptr(f), _ptr(x))
        return x

    def solve(self, f, x0=None, tol=1e-10, max_cycles=200, smoother="lsgs", order="col7", tau=None,
              nu1=2, nu2=2, gamma=1, norm="linv"):
        """Cycles until ||f - A x|| <= tol ||f|| in the Euclidean norm ("l2") or
        the L_k^{-1} norm ("linv"). Returns (x, cycles, history)."""
        tau = TAU_POISSON if tau is None else tau
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.zeros(self.ndof()) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles + 2)
        it = self.lib.mgo_solve(self._h, SMOOTHERS[smoother], ORDERS[order], float(tau), nu1, nu2, gamma,
                                _ptr(f), _ptr(x), float(tol), max_cycles, {"l2": 0, "linv": 1}[norm], _ptr(hist))
        n = (max_cycles + 1) if it < 0 else it + 1
        return x, it, hist[:n]

    # -- post-processing written from the problem statement -----------------

    def rhs(self, yd: np.ndarray, level: int | None = None) -> np.ndarray:
        """f = (M y_D; 0) with y_D the nodal values of the desired state."""
        M = self.matrix("M", level)
        V = M.shape[0]
        f = np.zeros(2 * V)
        f[:V] = M @ np.asarray(yd, dtype=np.float64)
        return f

    def control(self, x: np.ndarray) -> np.ndarray:
        V = x.shape[0] // 2
        return x[V:] / self.alpha


def adjoint_gradient(h: Hierarchy, yd: np.ndarray, y_target: np.ndarray, tol=1e-13, **kw):
    """Loss L = 1/2 ||y - y_target||_2^2 (nodal) of the solution of eq. mp2.

    Returns (L, dL/dy_D, dL/dalpha, x, x_adj).
    """
    f = h.rhs(yd)
    x, it, _ = h.solve(f, tol=tol, **kw)
    if it < 0:
        raise RuntimeError("oracle: forward solve did not converge")
    V = f.shape[0] // 2
    g = np.zeros_like(f)
    g[:V] = x[:V] - y_target
    xa, it, _ = h.solve(g, tol=tol, **kw)
    if it < 0:
        raise RuntimeError("oracle: adjoint solve did not converge")
    M = h.matrix("M")
    loss = 0.5 * float(np.dot(x[:V] - y_target, x[:V] - y_target))
    d_yd = M @ xa[:V]
    d_alpha = -float(xa[V:] @ (M @ x[V:])) / h.alpha**2
    return loss, d_yd, d_alpha, x, xa
