"""Pins of the oracle's multigrid solver: exact solves, the iteration counts of
Table 1 (section 3), robustness in h and alpha, the control relation of
section 1 and adjoint gradients against finite differences."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spl

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_poisson.txt")


def _table1():
    rows = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if line:
            rows[(int(line[0]), line[1])] = [int(v) for v in line[2:5]]
    return rows


@pytest.mark.parametrize("coarse", [1, 2])
@pytest.mark.parametrize("alpha", [1.0, 1e-8])
def test_coarse_lu_matches_dense_solve(alpha, coarse):
    h = oracle.Hierarchy(coarse + 2, alpha, coarse=coarse)
    A = h.matrix("A", coarse).toarray()
    b = workloads.uniform(A.shape[0], 3)
    x = h.coarse_solve(b)
    ref = np.linalg.solve(A, b)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(A, 2) * np.linalg.norm(x)


@pytest.mark.parametrize("smoother", ["ne", "lsgs", "slsgs", "cgs"])
@pytest.mark.parametrize("alpha", [1.0, 1e-2, 1e-8])
@pytest.mark.parametrize("level", [4, 6])
def test_solve_matches_sparse_direct(level, alpha, smoother):
    h = oracle.Hierarchy(level, alpha, coarse=1)
    f = h.rhs(workloads.desired_state(level, 1))
    nu = 1 if smoother == "slsgs" else 2
    x, it, hist = h.solve(f, tol=1e-10, max_cycles=300, smoother=smoother, nu1=nu, nu2=nu)
    assert it > 0
    ref = spl.spsolve(h.matrix("A").tocsc(), f)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert hist[-1] <= 1e-10


def _protocol_p(level, alpha, smoother, order="lex", gamma=2, maxc=80):
    """Section 3: random x0, f = 0, cycles until ||x||_L <= 1e-6 ||x0||_L."""
    h = oracle.Hierarchy(level, alpha, coarse=1)
    L = h.Ldiag()
    x = workloads.uniform(h.ndof(), 11)
    n0 = np.sqrt(x @ (L * x))
    f = np.zeros_like(x)
    nu = 1 if smoother == "slsgs" else 2
    for it in range(1, maxc + 1):
        h.cycle(f, x, smoother=smoother, order=order, gamma=gamma, nu1=nu, nu2=nu)
        if np.sqrt(x @ (L * x)) <= 1e-6 * n0:
            return it
    return maxc + 1


@pytest.mark.parametrize("level", [5, 6, 7])
@pytest.mark.parametrize("smoother,order", [("ne", "lex"), ("lsgs", "lex"), ("slsgs", "lex"), ("cgs", "lex")])
def test_table1_iteration_counts(level, smoother, order):
    # Reading: the paper's cycle is the W-cycle (its theory covers it), coarsest
    # level k0 = 1, lexicographic unknown order.  NE and sLSGS reproduce the
    # printed counts to within 1-3 cycles; LSGS and CGS to within 3; at
    # alpha = 1e-12 the counts depend on unstated details and get a wider band.
    paper = _table1()[(level, smoother)]
    ours = [_protocol_p(level, a, smoother, order) for a in (1.0, 1e-6, 1e-12)]
    for a_idx, (p, o) in enumerate(zip(paper, ours)):
        band = 3 if a_idx < 2 else 5
        assert abs(o - p) <= band, (level, smoother, paper, ours)


@pytest.mark.slow
@pytest.mark.parametrize("smoother", ["ne", "lsgs", "slsgs", "cgs"])
def test_table1_iteration_counts_level8(smoother):
    paper = _table1()[(8, smoother)]
    ours = [_protocol_p(8, a, smoother) for a in (1.0, 1e-6, 1e-12)]
    for a_idx, (p, o) in enumerate(zip(paper, ours)):
        assert abs(o - p) <= (3 if a_idx < 2 else 5), (paper, ours)


def test_gauss_seidel_like_speedup_over_normal_equation():
    # abstract and section 3: LSGS needs about half the iterations of NE
    for level in (5, 6):
        for alpha in (1.0, 1e-6):
            ne = _protocol_p(level, alpha, "ne", gamma=1)
            ls = _protocol_p(level, alpha, "lsgs", order="col7", gamma=1)
            assert 1.7 <= ne / ls <= 3.5, (level, alpha, ne, ls)


def test_v_cycle_counts_bounded_in_h_and_alpha():
    counts = {}
    for level in (4, 5, 6, 7):
        for alpha in (1.0, 1e-4, 1e-8):
            counts[(level, alpha)] = _protocol_p(level, alpha, "lsgs", order="col7", gamma=1)
    assert max(counts.values()) <= 20, counts


@pytest.mark.parametrize("smoother,gamma,bound", [("lsgs", 1, 0.45), ("lsgs", 2, 0.4), ("ne", 1, 0.7)])
def test_iteration_matrix_spectral_radius(smoother, gamma, bound):
    # dense error-propagation matrix of one cycle (f = 0) on level 3
    for alpha in (1.0, 1e-6, 1e-12):
        h = oracle.Hierarchy(3, alpha, coarse=1)
        n = h.ndof()
        E = np.zeros((n, n))
        f = np.zeros(n)
        for c in range(n):
            e = np.zeros(n)
            e[c] = 1.0
            h.cycle(f, e, smoother=smoother, order="col7", gamma=gamma)
            E[:, c] = e
        rho = np.max(np.abs(np.linalg.eigvals(E)))
        assert rho < bound, (alpha, rho)


@pytest.mark.parametrize("alpha", [1e-2, 1e-6])
def test_control_relation_at_convergence(alpha):
    # u = alpha^{-1} lambda; second block row K y - M u = 0 at the solution
    level = 5
    h = oracle.Hierarchy(level, alpha, coarse=1)
    f = h.rhs(workloads.desired_state(level, 1))
    x, it, _ = h.solve(f, tol=1e-11)
    V = f.size // 2
    u = h.control(x)
    K, M = h.K(), h.matrix("M")
    res2 = K @ x[:V] - M @ u
    assert np.linalg.norm(res2) <= 1e-10 * np.linalg.norm(K @ x[:V])
    # first block row: M y + K lambda = M y_D
    res1 = M @ x[:V] + K @ x[V:] - f[:V]
    assert np.linalg.norm(res1) <= 1e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("alpha", [1e-2, 1e-4])
def test_adjoint_gradient_matches_central_differences(alpha):
    level = 4
    h = oracle.Hierarchy(level, alpha, coarse=1)
    yd = workloads.desired_state(level, 4)
    yt = workloads.desired_state(level, 5)
    loss, g_yd, g_alpha, _, _ = oracle.adjoint_gradient(h, yd, yt)

    def loss_at(yd_, alpha_):
        hh = oracle.Hierarchy(level, alpha_, coarse=1)
        x, it, _ = hh.solve(hh.rhs(yd_), tol=1e-14, max_cycles=400)
        V = yd_.size
        return 0.5 * float(np.sum((x[:V] - yt) ** 2))

    d = workloads.uniform(yd.size, 6)
    d /= np.abs(d).max()
    eps = 1e-6
    fd = (loss_at(yd + eps * d, alpha) - loss_at(yd - eps * d, alpha)) / (2 * eps)
    assert g_yd @ d == pytest.approx(fd, rel=1e-6)
    da = 1e-6 * alpha  # relative step
    fda = (loss_at(yd, alpha + da) - loss_at(yd, alpha - da)) / (2 * da)
    assert g_alpha == pytest.approx(fda, rel=1e-6)


def test_threaded_oracle_is_bit_identical():
    """The OpenMP build (used for the all-cores CPU baseline) steps the groups
    of one colour concurrently; they touch disjoint residual entries, so its
    cycles equal the single-threaded build's bit for bit."""
    level, alpha = 7, 1e-4
    out = []
    for threaded in (False, True):
        h = oracle.Hierarchy(level, alpha, coarse=1, threaded=threaded)
        f = h.rhs(workloads.desired_state(level, 2))
        x = np.zeros(h.ndof())
        for sm in ("lsgs", "slsgs", "ne"):
            h.cycle(f, x, smoother=sm, order="col7", nu1=1, nu2=1)
        out.append(x)
    assert np.array_equal(out[0], out[1])
