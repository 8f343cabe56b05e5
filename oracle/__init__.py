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

NE, LSGS, SLSGS, CGS, VANKA = 0, 1, 2, 3, 4
ORDER_LEX, ORDER_COL7, ORDER_COL7SEQ, ORDER_VLEX, ORDER_COL3 = 0, 1, 2, 3, 4
SMOOTHERS = {"ne": NE, "lsgs": LSGS, "slsgs": SLSGS, "cgs": CGS, "vanka": VANKA}
ORDERS = {"lex": ORDER_LEX, "col7": ORDER_COL7, "col7seq": ORDER_COL7SEQ, "vlex": ORDER_VLEX, "col3": ORDER_COL3}
# damping of the normal-equation smoother used in the paper's experiments
# (section 3): 0.4 for Poisson control, 0.35 for Stokes control; the Stokes
# patch (Vanka-type) smoother is damped with 0.4
TAU_POISSON, TAU_STOKES, TAU_VANKA = 0.4, 0.35, 0.4


_OMP_PATH = os.path.join(_HERE, "libmgo_omp.so")
_omp_lib = None


def build(force: bool = True) -> str:
    """Compile mgo.c into libmgo.so next to this file (plain gcc, FP64,
    single-threaded) and into libmgo_omp.so, the same source built with
    OpenMP: its parallel loops (sparse products, transfers, and the groups of
    one colour of the COL7 order, which touch disjoint residual entries) run
    on the host's cores with bit-identical results."""
    src = [os.path.join(_HERE, "mgo.c")]
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off"] + extra + ["-o", tmp] + src + ["-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, path)
    return _LIB_PATH


def threads(threaded: bool = False) -> int:
    """Threads of the oracle's parallel loops (1 for the default build)."""
    return int(_load(threaded).mgo_threads())


def _load(threaded: bool = False):
    global _lib, _omp_lib
    if threaded:
        if _omp_lib is None:
            if not os.path.exists(_OMP_PATH):
                build(force=False)
            _omp_lib = _setup(ctypes.CDLL(_OMP_PATH))
        return _omp_lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    _lib = _setup(ctypes.CDLL(_LIB_PATH))
    return _lib


def _setup(lib):
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
    lib.mgo_project.argtypes = [vp, ip, vp]
    lib.mgo_assemble_p2.argtypes = [ip, ip, vp, vp, vp, vp]
    lib.mgo_prolongation_p2.argtypes = [ip, ip, vp]
    lib.mgo_csr_free.argtypes = [vp]
    lib.mgo_threads.restype = ip
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


class _Csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int), ("ncols", ctypes.c_int), ("nnz", ctypes.c_int),
                ("rowptr", ctypes.POINTER(ctypes.c_int)), ("col", ctypes.POINTER(ctypes.c_int)),
                ("val", ctypes.POINTER(ctypes.c_double))]


def _take(c: _Csr):
    import scipy.sparse as sp

    rp = np.ctypeslib.as_array(c.rowptr, shape=(c.nrows + 1,)).copy()
    ci = np.ctypeslib.as_array(c.col, shape=(max(c.nnz, 1),))[: c.nnz].copy()
    va = np.ctypeslib.as_array(c.val, shape=(max(c.nnz, 1),))[: c.nnz].copy()
    out = sp.csr_matrix((va, ci, rp), shape=(c.nrows, c.ncols))
    _load().mgo_csr_free(ctypes.byref(c))
    return out


def taylor_hood(n: int, full: bool = False):
    """(M, K, D1, D2) of the P2/P1 pair with n cells per side (eq. mp3 blocks):
    scalar P2 mass and Laplacian stiffness over the interior P2 nodes (or all
    nodes), and D_c = -int q d_c phi with rows over the P1 vertices."""
    mats = [_Csr() for _ in range(4)]
    _load().mgo_assemble_p2(n, int(full), *[ctypes.byref(m) for m in mats])
    return tuple(_take(m) for m in mats)


def prolongation_p2(nc: int, full: bool = False):
    c = _Csr()
    _load().mgo_prolongation_p2(nc, int(full), ctypes.byref(c))
    return _take(c)


def p2_nodes(level: int, full: bool = False):
    """Coordinates (X, Y) of the P2 nodes of level `level` in index order."""
    n = 1 << level
    idx = np.arange(0, 2 * n + 1) if full else np.arange(1, 2 * n)
    B, A = np.meshgrid(idx, idx, indexing="ij")
    return (A / (2.0 * n)).ravel(), (B / (2.0 * n)).ravel()


class Hierarchy:
    """Levels coarse..fine of the Poisson control KKT system (eq. mp2,
    problem 0 / "poisson") or of the Stokes control system (eq. mp3,
    problem 1 / "stokes", Taylor-Hood).

    Poisson: level l has n = 2^l cells per side of the unit square, (n+1)^2
    vertices and 2 (n+1)^2 unknowns x = (y; lambda), field-major.
    Stokes: [v1 | v2 | p | lambda1 | lambda2 | mu] with (2n-1)^2 interior P2
    nodes per velocity component and (n+1)^2 pressure vertices.
    """

    def __init__(self, level: int, alpha: float, coarse: int = 1, problem=0, threaded: bool = False):
        problem = {"poisson": 0, "stokes": 1}.get(problem, problem)
        self.lib = _load(threaded)
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

    def _tau(self, smoother: str) -> float:
        if smoother == "vanka":
            return TAU_VANKA
        return TAU_STOKES if self.problem == 1 else TAU_POISSON

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
        tau = self._tau(smoother) if tau is None else tau
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
        tau = self._tau(smoother) if tau is None else tau
        f = np.ascontiguousarray(f, dtype=np.float64)
        self.lib.mgo_cycle(self._h, l, SMOOTHERS[smoother], ORDERS[order], float(tau), nu1, nu2, gamma, _ptr(f), _ptr(x))
        return x

    def solve(self, f, x0=None, tol=1e-10, max_cycles=200, smoother="lsgs", order="col7", tau=None,
              nu1=2, nu2=2, gamma=1, norm="linv"):
        """Cycles until ||f - A x|| <= tol ||f|| in the Euclidean norm ("l2") or
        the L_k^{-1} norm ("linv"). Returns (x, cycles, history)."""
        tau = self._tau(smoother) if tau is None else tau
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.zeros(self.ndof()) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles + 2)
        it = self.lib.mgo_solve(self._h, SMOOTHERS[smoother], ORDERS[order], float(tau), nu1, nu2, gamma,
                                _ptr(f), _ptr(x), float(tol), max_cycles, {"l2": 0, "linv": 1}[norm], _ptr(hist))
        n = (max_cycles + 1) if it < 0 else it + 1
        return x, it, hist[:n]

    # -- post-processing written from the problem statement -----------------

    def rhs(self, yd: np.ndarray, level: int | None = None) -> np.ndarray:
        """Poisson: f = (M y_D; 0) with y_D the nodal values of the desired
        state.  Stokes: f = (M v_D; 0; 0; 0) with v_D = [v1 | v2] the desired
        velocity at the interior P2 nodes (M the P2 mass of each component)."""
        M = self.matrix("M", level)
        V = M.shape[0]
        yd = np.asarray(yd, dtype=np.float64)
        if self.problem == 1:
            f = np.zeros(self.ndof(level))
            f[:V] = M @ yd[:V]
            f[V:2 * V] = M @ yd[V:2 * V]
            return f
        f = np.zeros(2 * V)
        f[:V] = M @ yd
        return f

    def project(self, x: np.ndarray, level: int | None = None) -> np.ndarray:
        """Stokes: p and mu shifted to zero mean (in place); Poisson: no-op."""
        self.lib.mgo_project(self._h, self.level if level is None else level, _ptr(x))
        return x

    def fields(self, level: int | None = None):
        """Stokes: slices of v1, v2, p, lambda1, lambda2, mu."""
        l = self.level if level is None else level
        n = 1 << l
        nv, np_ = (2 * n - 1) ** 2, (n + 1) ** 2
        sizes = [nv, nv, np_, nv, nv, np_]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        return [slice(int(offs[i]), int(offs[i + 1])) for i in range(6)]

    def control(self, x: np.ndarray) -> np.ndarray:
        if self.problem == 1:
            fl = self.fields()
            return np.concatenate([x[fl[3]], x[fl[4]]]) / self.alpha
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
