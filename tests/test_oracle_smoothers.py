"""Pins of the oracle's smoothers (Alg. 1, Alg. 2, sLSGS, CGS) against the
compact matrix forms printed in section 2, evaluated with dense linear algebra,
and against invariants that any correct implementation must satisfy."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads

ALPHAS = [1.0, 1e-3, 1e-8]


def _setup(level, alpha, seed=5):
    h = oracle.Hierarchy(level, alpha, coarse=1)
    A = h.matrix("A").toarray()
    L = h.Ldiag()
    N = A.T @ np.diag(1.0 / L) @ A
    n = A.shape[0]
    x = workloads.uniform(n, seed)
    f = workloads.uniform(n, seed + 1)
    return h, A, L, N, x, f


def _perm_matrix(order):
    P = np.zeros((len(order), len(order)))
    P[np.arange(len(order)), order] = 1.0
    return P


def _run(h, smoother, order, x, f, tau=None):
    x1 = x.copy()
    r = h.residual(f, x1)
    h.smooth(x1, r, smoother=smoother, order=order, tau=tau)
    return x1, r


@pytest.mark.parametrize("alpha", ALPHAS)
def test_ne_matches_compact_form(alpha):
    # x <- x + tau L^{-1} A^T L^{-1} (f - A x)
    h, A, L, N, x, f = _setup(3, alpha)
    x1, r1 = _run(h, "ne", "lex", x, f, tau=0.4)
    ref = x + 0.4 * (A.T @ ((f - A @ x) / L)) / L
    np.testing.assert_allclose(x1, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(r1, f - A @ x1, atol=1e-11 * np.abs(f - A @ x1).max())


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("order", ["lex", "vlex", "col7seq"])
def test_lsgs_matches_compact_form(alpha, order):
    # x <- x + trig(N)^{-1} A^T L^{-1} (f - A x) in the ordering of the unknowns
    h, A, L, N, x, f = _setup(3, alpha)
    x1, r1 = _run(h, "lsgs", order, x, f)
    n = A.shape[0]
    V = n // 2
    nside = int(round(np.sqrt(V)))
    if order == "lex":
        perm = np.arange(n)
    elif order == "vlex":
        perm = np.ravel(np.column_stack([np.arange(V), V + np.arange(V)]))
    else:
        vs = [j * nside + i for c in range(7) for j in range(nside) for i in range(nside) if (i + 2 * j) % 7 == c]
        perm = np.ravel(np.column_stack([vs, V + np.asarray(vs)]))
    Pm = _perm_matrix(perm)
    Np = Pm @ N @ Pm.T
    b = Pm @ (A.T @ ((f - A @ x) / L))
    dz = sla.solve_triangular(np.tril(Np), b, lower=True)
    ref = x + Pm.T @ dz
    np.testing.assert_allclose(x1, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(r1, f - A @ x1, atol=1e-11 * np.abs(f - A @ x1).max())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_slsgs_matches_eq_mcNhat(alpha):
    # x <- x + Nhat^{-1} A^T L^{-1} r, Nhat = trig(N) diag(N)^{-1} trig(N)^T
    h, A, L, N, x, f = _setup(3, alpha)
    x1, _ = _run(h, "slsgs", "lex", x, f)
    # Nhat^{-1} applied through its factors: trig(N)^{-T} diag(N) trig(N)^{-1}
    T = np.tril(N)
    b = A.T @ ((f - A @ x) / L)
    w = sla.solve_triangular(T, b, lower=True)
    ref = x + sla.solve_triangular(T.T, np.diag(N) * w, lower=False)
    np.testing.assert_allclose(x1, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_cgs_is_block_gauss_seidel(alpha):
    # collective GS over vertices: block lower-triangular solve with the 2x2
    # blocks P_i^T A P_i on the diagonal, vertex-interleaved lexicographic order
    h, A, L, N, x, f = _setup(3, alpha)
    x1, _ = _run(h, "cgs", "lex", x, f)
    n = A.shape[0]
    V = n // 2
    perm = np.ravel(np.column_stack([np.arange(V), V + np.arange(V)]))
    Pm = _perm_matrix(perm)
    Ap = Pm @ A @ Pm.T
    B = np.tril(Ap)
    for v in range(V):
        B[2 * v, 2 * v + 1] = Ap[2 * v, 2 * v + 1]
    ref = x + Pm.T @ np.linalg.solve(B, Pm @ (f - A @ x))
    np.testing.assert_allclose(x1, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("alpha", [1.0, 1e-6])
def test_lsgs_coordinate_descent_identity(alpha):
    # LSGS is coordinate descent on 1/2 ||f - A x||^2_{L^-1}: updating unknown i
    # lowers ||r||^2_{L^-1} by exactly q^2 / N_ii with q = (A^T L^{-1} r)_i
    h, A, L, N, x, f = _setup(3, alpha)
    r = h.residual(f, x)
    x = x.copy()
    rng = np.random.default_rng(0)
    for i in rng.choice(A.shape[0], 12, replace=False):
        q = (A.T @ (r / L))[i]
        before = r @ (r / L)
        h.smooth_groups(x, r, [[int(i)]])
        after = r @ (r / L)
        assert before - after == pytest.approx(q * q / N[i, i], rel=1e-8, abs=1e-14 * before)


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("smoother", ["lsgs", "slsgs"])
def test_gs_like_sweeps_are_monotone(alpha, smoother):
    h, A, L, N, x, f = _setup(4, alpha)
    x = x.copy()
    r = h.residual(f, x)
    prev = r @ (r / L)
    for _ in range(5):
        h.smooth(x, r, smoother=smoother, order="col7")
        cur = r @ (r / L)
        assert cur <= prev * (1 + 1e-14)
        prev = cur


def test_seven_colours_form_perfect_code():
    # colour c(i,j) = (i + 2j) mod 7: the closed neighbourhoods of one colour
    # are pairwise disjoint and cover every vertex whose lattice neighbours all
    # lie in the domain exactly once (the boundary clips the others)
    level = 4
    h = oracle.Hierarchy(level, 1e-2, coarse=1)
    M = h.matrix("M")
    n = (1 << level) + 1
    col = np.array([(v % n + 2 * (v // n)) % 7 for v in range(n * n)])
    for c in range(7):
        cover = np.zeros(n * n, dtype=int)
        for v in np.nonzero(col == c)[0]:
            cover[M.indices[M.indptr[v]:M.indptr[v + 1]]] += 1
        assert cover.max() == 1
        inner = cover.reshape(n, n)[1:-1, 1:-1]
        assert inner.min() == 1
    # and the N stencil couples same-colour unknowns nowhere
    A = h.matrix("A")
    import scipy.sparse as sp
    Nm = (A.T @ sp.diags(1.0 / h.Ldiag()) @ A).tocoo()
    V = n * n
    iv, jv = Nm.row % V, Nm.col % V
    same = (col[iv] == col[jv]) & (iv != jv)
    assert np.all(np.abs(Nm.data[same]) == 0.0)


@pytest.mark.parametrize("alpha", [1.0, 1e-8])
def test_col7_within_colour_order_is_irrelevant(alpha):
    h, A, L, N, x, f = _setup(4, alpha)
    V = A.shape[0] // 2
    nside = int(round(np.sqrt(V)))
    groups_fwd, groups_mix = [], []
    for c in range(7):
        vs = [j * nside + i for j in range(nside) for i in range(nside) if (i + 2 * j) % 7 == c]
        groups_fwd += [[v, V + v] for v in vs]
        rng = np.random.default_rng(c)
        groups_mix += [[v, V + v] for v in rng.permutation(vs)]
    x1, x2 = x.copy(), x.copy()
    r1, r2 = h.residual(f, x1), h.residual(f, x2)
    h.smooth_groups(x1, r1, groups_fwd)
    h.smooth_groups(x2, r2, groups_mix)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(r1, r2)
    # built-in col7 ordering equals the explicit one bit for bit
    x3 = x.copy()
    r3 = h.residual(f, x3)
    h.smooth(x3, r3, smoother="lsgs", order="col7")
    np.testing.assert_array_equal(x1, x3)


@pytest.mark.parametrize("alpha", [1.0, 1e-8])
def test_simultaneous_vs_sequential_y_lambda(alpha):
    h, A, L, N, x, f = _setup(4, alpha)
    a, _ = _run(h, "lsgs", "col7", x, f)
    b, _ = _run(h, "lsgs", "col7seq", x, f)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("level", [2, 3, 4])
def test_ne_damping_keeps_spectral_radius_below_two(level):
    # tau rho(L^{-1} A^T L^{-1} A) must stay away from 2 (section 2) for tau = 0.4
    for alpha in [1.0, 1e-6, 1e-12]:
        h = oracle.Hierarchy(level, alpha, coarse=1)
        A = h.matrix("A").toarray()
        Li = 1.0 / h.Ldiag()
        G = (Li[:, None] * A.T) @ (Li[:, None] * A)
        rho = np.max(np.abs(np.linalg.eigvals(G)))
        assert 0.4 * rho < 1.9, (level, alpha, rho)
