"""Pins of the oracle's discretisation (section 1, eq. mp2) against closed forms.

P1 elements integrate products of linear functions exactly, so quadratic forms
of M and of the Laplacian stiffness matrix on the nodal values of 1, x and y
equal integrals over the unit square that are known in closed form.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads


def _h(level=3, alpha=1e-2):
    return oracle.Hierarchy(level, alpha, coarse=1)


@pytest.mark.parametrize("level", [2, 3, 5])
def test_mass_matrix_integrates_linear_products(level):
    h = _h(level)
    M = h.matrix("M")
    X, Y = workloads.grid_coords(level)
    one = np.ones_like(X)
    assert one @ M @ one == pytest.approx(1.0, abs=1e-14)          # area
    assert X @ M @ X == pytest.approx(1.0 / 3.0, abs=1e-14)        # int x^2
    assert Y @ M @ Y == pytest.approx(1.0 / 3.0, abs=1e-14)
    assert X @ M @ Y == pytest.approx(1.0 / 4.0, abs=1e-14)        # int x y
    assert one @ M @ X == pytest.approx(0.5, abs=1e-14)


@pytest.mark.parametrize("level", [2, 3, 5])
def test_laplacian_stiffness_forms(level):
    h = _h(level)
    Kl = h.matrix("Klap")
    X, Y = workloads.grid_coords(level)
    assert np.abs(Kl @ np.ones_like(X)).max() < 1e-13               # constants in kernel
    assert X @ Kl @ X == pytest.approx(1.0, abs=1e-13)              # int |grad x|^2
    assert Y @ Kl @ Y == pytest.approx(1.0, abs=1e-13)
    assert X @ Kl @ Y == pytest.approx(0.0, abs=1e-13)
    Z = X + Y
    assert Z @ Kl @ Z == pytest.approx(2.0, abs=1e-13)


def test_row_sums_equal_basis_integrals():
    # row sum of M at v = integral of phi_v = (#triangles at v) * h^2 / 6
    level = 3
    n = 1 << level
    M = _h(level).matrix("M")
    rs = np.asarray(M.sum(axis=1)).ravel().reshape(n + 1, n + 1)  # [j, i]
    h2 = 1.0 / n**2
    # triangles per vertex on the mesh split along (i,j)-(i+1,j+1)
    ntri = np.zeros((n + 1, n + 1))
    for j in range(n):
        for i in range(n):
            for tri in (((i, j), (i + 1, j), (i + 1, j + 1)), ((i, j), (i + 1, j + 1), (i, j + 1))):
                for (a, b) in tri:
                    ntri[b, a] += 1
    assert ntri[0, 0] == 2 and ntri[n, n] == 2 and ntri[0, n] == 1 and ntri[n, 0] == 1
    assert ntri[n // 2, n // 2] == 6 and ntri[0, n // 2] == 3
    np.testing.assert_allclose(rs, ntri * h2 / 6.0, rtol=1e-14, atol=0)


def test_interior_stencils():
    level = 4
    n = 1 << level
    h = _h(level)
    M = h.matrix("M").toarray()
    Kl = h.matrix("Klap").toarray()
    i, j = 7, 9
    v = j * (n + 1) + i
    nb = {(1, 0): "E", (-1, 0): "W", (0, 1): "N", (0, -1): "S", (1, 1): "NE", (-1, -1): "SW"}
    h2 = 1.0 / n**2
    assert M[v, v] == pytest.approx(h2 / 2, rel=1e-14)
    assert Kl[v, v] == pytest.approx(4.0, rel=1e-14)
    for (di, dj), name in nb.items():
        m = (j + dj) * (n + 1) + (i + di)
        assert M[v, m] == pytest.approx(h2 / 12, rel=1e-14), name
        expect = 0.0 if name in ("NE", "SW") else -1.0
        assert Kl[v, m] == pytest.approx(expect, abs=1e-14), name
    # no other couplings: 7-point stencil
    assert np.count_nonzero(M[v]) == 7


@pytest.mark.parametrize("alpha", [1.0, 1e-2, 1e-8])
def test_kkt_block_structure_and_symmetry(alpha):
    h = _h(3, alpha)
    A = h.matrix("A")
    M, K = h.matrix("M"), h.K()
    V = M.shape[0]
    assert abs(A - A.T).max() == 0.0
    Ad = A.toarray()
    np.testing.assert_array_equal(Ad[:V, :V], M.toarray())
    np.testing.assert_array_equal(Ad[:V, V:], K.toarray())
    np.testing.assert_array_equal(Ad[V:, :V], K.toarray())
    np.testing.assert_allclose(Ad[V:, V:], -M.toarray() / alpha, rtol=1e-15)


@pytest.mark.parametrize("alpha", [1.0, 1e-4, 1e-8])
def test_L_is_diag_of_Q(alpha):
    # L = blockdiag(diag(M + alpha^1/2 K), diag(alpha^-1 M + alpha^-1/2 K)), section 2
    h = _h(3, alpha)
    M, K = h.matrix("M"), h.K()
    L = h.Ldiag()
    V = M.shape[0]
    np.testing.assert_allclose(L[:V], (M + np.sqrt(alpha) * K).diagonal(), rtol=1e-14)
    np.testing.assert_allclose(L[V:], (M / alpha + K / np.sqrt(alpha)).diagonal(), rtol=1e-14)
    np.testing.assert_allclose(L[V:], L[:V] / alpha, rtol=1e-14)


@pytest.mark.parametrize("alpha", [1.0, 1e-6])
def test_N_diagonal(alpha):
    # N = A^T L^{-1} A; Alg. 2 prepares N_ii once
    h = _h(3, alpha)
    A = h.matrix("A")
    Linv = sp.diags(1.0 / h.Ldiag())
    N = (A.T @ Linv @ A).toarray()
    np.testing.assert_allclose(h.Ndiag(), np.diag(N), rtol=1e-13)
    # the (y_v, lambda_v) entries of N vanish (exact zero in exact arithmetic)
    V = A.shape[0] // 2
    scale = np.sqrt(np.outer(np.diag(N), np.diag(N)))
    assert np.max(np.abs(np.diag(N[:V, V:])) / np.diag(scale[:V, V:])) < 1e-14


@pytest.mark.parametrize("level", [2, 3, 5])
def test_prolongation_is_interpolation(level):
    h = _h(level)
    P = h.matrix("P")
    Xf, Yf = workloads.grid_coords(level)
    Xc, Yc = workloads.grid_coords(level - 1)
    np.testing.assert_array_equal(P @ np.ones_like(Xc), np.ones_like(Xf))
    np.testing.assert_allclose(P @ Xc, Xf, atol=1e-15)
    np.testing.assert_allclose(P @ Yc, Yf, atol=1e-15)
    assert set(np.unique(P.data)) <= {0.5, 1.0}


@pytest.mark.parametrize("alpha", [1.0, 1e-8])
@pytest.mark.parametrize("level", [3, 4])
def test_galerkin_identity(level, alpha):
    # nested P1 spaces: P^T A_k P = A_{k-1} for each block, restriction scale 1
    h = oracle.Hierarchy(level, alpha, coarse=1)
    P = h.matrix("P", level)
    Pb = sp.block_diag([P, P])
    Af = h.matrix("A", level)
    Ac = h.matrix("A", level - 1)
    G = (Pb.T @ Af @ Pb).toarray()
    np.testing.assert_allclose(G, Ac.toarray(), rtol=0, atol=1e-13 * np.abs(Ac).max())


def _manufactured_error(level, alpha):
    import scipy.sparse.linalg as spl

    h = oracle.Hierarchy(level, alpha, coarse=1)
    X, Y = workloads.grid_coords(level)
    c = 2 * np.pi**2 + 1
    y = np.cos(np.pi * X) * np.cos(np.pi * Y)   # Neumann data zero on the unit square
    yd = (1 + alpha * c**2) * y                 # y_D making (y, lambda = alpha c y) optimal
    f = h.rhs(yd)
    x = spl.spsolve(h.matrix("A").tocsc(), f)
    V = X.size
    M = h.matrix("M")
    ey = x[:V] - y
    eu = h.control(x) - c * y                   # u = alpha^-1 lambda
    return np.sqrt(ey @ M @ ey), np.sqrt(eu @ M @ eu)


@pytest.mark.parametrize("alpha", [1e-2, 1.0])
def test_manufactured_solution_second_order(alpha):
    errs = [_manufactured_error(l, alpha) for l in (3, 4, 5, 6)]
    ey = np.array([e[0] for e in errs])
    eu = np.array([e[1] for e in errs])
    ry = ey[:-1] / ey[1:]
    ru = eu[:-1] / eu[1:]
    assert np.all(ry > 3.5) and np.all(ry < 4.6), ry
    assert np.all(ru > 3.5) and np.all(ru < 4.6), ru
    assert ey[-1] < 1e-3 * (1 + alpha * (2 * np.pi**2 + 1) ** 2)
