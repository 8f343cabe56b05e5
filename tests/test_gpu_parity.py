"""GPU parity: every kernel and every cycle of the HIP path against the FP64
CPU oracle on the same seeded inputs (through the C ABI)."""
import numpy as np
import pytest

import oracle
import workloads
from fieldwise import assert_fields

pytestmark = pytest.mark.gpu

ALPHAS = [1.0, 1e-2, 1e-8]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _mg():
    import paper_1502_03917_amd as mg

    return mg


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("level", [3, 6])
def test_stencil_kernels(torch_cuda, level, alpha):
    torch = torch_cuda
    mg = _mg()
    s = mg.Solver(level, alpha)
    h = oracle.Hierarchy(level, alpha, coarse=1)
    n = h.ndof()
    x = workloads.uniform(n, 21)
    f = workloads.uniform(n, 22)
    # A x and f - A x
    Ax = h.matrix("A") @ x
    assert _relmax(_host(s.apply(_dev(torch, x))), Ax) < 1e-14
    r_ref = h.residual(f, x)
    r_gpu, nrm = s.residual(_dev(torch, f), _dev(torch, x), norm=True)
    assert _relmax(_host(r_gpu), r_ref) < 1e-13
    assert nrm == pytest.approx(np.linalg.norm(r_ref), rel=1e-13)
    # right-hand side (M y_D; 0)
    yd = workloads.desired_state(level, 1)
    assert _relmax(_host(s.rhs(_dev(torch, yd))), h.rhs(yd)) < 1e-14
    # transfers between level and level-1
    fc_ref = np.concatenate([h.matrix("P").T @ r_ref[: n // 2], h.matrix("P").T @ r_ref[n // 2:]])
    assert _relmax(_host(s.restrict(_dev(torch, r_ref))), fc_ref) < 1e-14
    nc = h.ndof(level - 1)
    xc = workloads.uniform(nc, 23)
    P = h.matrix("P")
    xp_ref = x + np.concatenate([P @ xc[: nc // 2], P @ xc[nc // 2:]])
    xg = _dev(torch, x)
    s.prolong_add(_dev(torch, xc), xg)
    assert _relmax(_host(xg), xp_ref) < 1e-15


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("smoother", ["ne", "lsgs", "slsgs", "cgs"])
@pytest.mark.parametrize("level", [3, 6])
def test_smoothing_step(torch_cuda, level, alpha, smoother):
    torch = torch_cuda
    mg = _mg()
    s = mg.Solver(level, alpha, smoother=smoother)
    h = oracle.Hierarchy(level, alpha, coarse=1)
    n = h.ndof()
    x = workloads.uniform(n, 31)
    f = workloads.uniform(n, 32)
    r = h.residual(f, x)
    xg, rg = _dev(torch, x), _dev(torch, r)
    xo, ro = x.copy(), r.copy()
    for _ in range(2):
        s.smooth(xg, rg, steps=1)
        h.smooth(xo, ro, smoother=smoother, order="col7")
    assert_fields(_host(xg), xo, 1e-13, what="x")
    assert_fields(_host(rg), ro, 1e-12, what="r")


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("coarse", [1, 2, 3])
def test_coarse_solve(torch_cuda, alpha, coarse):
    torch = torch_cuda
    mg = _mg()
    s = mg.Solver(coarse + 2, alpha, coarse_level=coarse)
    h = oracle.Hierarchy(coarse + 2, alpha, coarse=coarse)
    b = workloads.uniform(h.ndof(coarse), 41)
    ref = h.coarse_solve(b)
    got = _host(s.coarse_solve(_dev(torch, b)))
    A = h.matrix("A", coarse).toarray()
    # both are backward stable FP64 LU solves of the same matrix
    assert np.linalg.norm(A @ got - b) <= 1e-13 * np.linalg.norm(A, 2) * np.linalg.norm(got)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("smoother", ["lsgs", "slsgs", "cgs", "ne"])
@pytest.mark.parametrize("level", [7, 10])
def test_fused_sweep_matches_phase_kernels(torch_cuda, monkeypatch, level, smoother):
    # one fused kernel per sweep vs one launch per colour phase: same arithmetic
    # (LSGS: 14-vertex halo; collective smoother: 7-vertex halo); NE: one pass
    # over 64 x 16 tiles with a 2-vertex ring vs the two-kernel step
    torch = torch_cuda
    mg = _mg()
    alpha = 1e-3
    monkeypatch.setenv("MGKKT_PHASE_KERNELS", "1")
    sp = mg.Solver(level, alpha, smoother=smoother)
    monkeypatch.delenv("MGKKT_PHASE_KERNELS")
    sf = mg.Solver(level, alpha, smoother=smoother)
    n = sf.vec_len()
    x = workloads.uniform(n, 51)
    f = workloads.uniform(n, 52)
    r = _host(sf.residual(_dev(torch, f), _dev(torch, x)))
    xa, ra = _dev(torch, x), _dev(torch, r)
    xb, rb = _dev(torch, x), _dev(torch, r)
    sp.smooth(xa, ra, steps=3)
    sf.smooth(xb, rb, steps=3)
    assert _relmax(_host(xb), _host(xa)) < 1e-14
    assert _relmax(_host(rb), _host(ra)) < 1e-13


@pytest.mark.parametrize("smoother,gamma", [("lsgs", 1), ("ne", 1), ("slsgs", 2), ("cgs", 1)])
@pytest.mark.parametrize("level", [4, 7])
def test_coarse_tail_matches_level_kernels(torch_cuda, monkeypatch, level, smoother, gamma):
    # the one-workgroup tail (levels <= 5 in LDS) against the per-level launches
    torch = torch_cuda
    mg = _mg()
    alpha = 1e-4
    nu = 1 if smoother == "slsgs" else 2
    monkeypatch.setenv("MGKKT_NO_TAIL", "1")
    sa = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu)
    monkeypatch.delenv("MGKKT_NO_TAIL")
    sb = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu)
    yd = _dev(torch, workloads.desired_state(level, 1))
    fa, fb = sa.rhs(yd), sb.rhs(yd)
    xa = torch.zeros(sa.vec_len(), dtype=torch.float64, device="cuda")
    xb = torch.zeros_like(xa)
    for _ in range(3):
        sa.cycle(fa, xa)
        sb.cycle(fb, xb)
    assert _relmax(_host(xb), _host(xa)) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_replays_match_eager(torch_cuda, monkeypatch, precision):
    # mg_solve replays one captured iterate per cycle; after k replays the
    # iterate equals k eager iterates bit for bit, for every k
    torch = torch_cuda
    mg = _mg()
    level, alpha = 8, 1e-3
    monkeypatch.setenv("MGKKT_NO_GRAPH", "1")
    se = mg.Solver(level, alpha, precision=precision)
    monkeypatch.delenv("MGKKT_NO_GRAPH")
    sg = mg.Solver(level, alpha, precision=precision)
    yd = _dev(torch, workloads.desired_state(level, 2))
    f = se.rhs(yd)
    for k in range(1, 6):
        se.set_opts(max_cycles=k)
        sg.set_opts(max_cycles=k)
        xe, ie, re, ste = se.solve(f, tol=1e-14, raise_on_error=False)
        xg, ig, rg, stg = sg.solve(f, tol=1e-14, raise_on_error=False)
        assert ie == ig == k and ste == stg == mg.MG_ENOTCONV
        assert torch.equal(xe, xg), k
        assert re == rg
    # sweep timing (the timed solve runs its kernels without the graph)
    sg.set_opts(max_cycles=200)
    sg.timing_enable(True)
    xg, it, rel, st = sg.solve(f, tol=1e-10)
    ms, n = sg.timing_read()
    sg.timing_enable(False)
    assert st == mg.MG_OK and n == 4 * it and ms > 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("problem,precision", [("poisson", "fp64"), ("poisson", "fp32_ir"), ("stokes", "fp64")])
def test_capture_cycle_replays_match_eager(torch_cuda, problem, precision):
    # mg_capture_cycle: capturing executes nothing; each replay equals one
    # eager mg_cycle bit for bit, with eager work of the same context
    # (residual norms, which share its workspace) between the replays;
    # mg_set_opts invalidates the graph
    torch = torch_cuda
    mg = _mg()
    level, alpha = (8, 1e-3) if problem == "poisson" else (5, 1e-2)
    se = mg.Solver(level, alpha, problem=problem, precision=precision)
    sg = mg.Solver(level, alpha, problem=problem, precision=precision)
    data = workloads.desired_state(level, 2) if problem == "poisson" else workloads.desired_velocity(level, 7)
    f = se.rhs(_dev(torch, data))
    xe = torch.zeros_like(f)
    xg = torch.zeros_like(f)
    other = _dev(torch, workloads.uniform(f.numel(), 5))
    g = sg.capture_cycle(f, xg)
    torch.cuda.synchronize()
    assert not xg.any()
    for k in range(1, 5):
        se.cycle(f, xe)
        g.launch()
        _, nrm = sg.residual(f, other, norm=True)
        assert nrm > 0
        assert torch.equal(xe, xg), k
    if problem == "poisson" and precision == "fp64":
        h = oracle.Hierarchy(level, alpha, coarse=1)
        xo = np.zeros(h.ndof())
        fo = h.rhs(workloads.desired_state(level, 2))
        for _ in range(4):
            h.cycle(fo, xo, smoother="lsgs", order="col7")
        assert_fields(_host(xg), xo, 1e-12, alpha=alpha)
    sg.set_opts(nu1=1)
    with pytest.raises(mg.MGError) as e:
        g.launch()
    assert e.value.status == mg.MG_EINVAL
    g.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("smoother,gamma", [("lsgs", 1), ("ne", 1), ("slsgs", 2), ("lsgs", 2)])
def test_coarse_map_equals_subcycle(torch_cuda, monkeypatch, smoother, gamma):
    # the tail's precomputed map of the level-3 sub-cycle gives the same
    # iterates as running that sub-cycle (MGKKT_NO_MAP=1), to rounding, for
    # V- and W-cycles, in FP64 and in FP32 refinement
    torch = torch_cuda
    mg = _mg()
    level, alpha = 7, 1e-3
    nu = 1 if smoother == "slsgs" else 2
    yd = _dev(torch, workloads.desired_state(level, 3))
    for precision, bound in (("fp64", 1e-13), ("fp32_ir", 1e-5)):
        xs = []
        for env in (None, "1"):
            if env:
                monkeypatch.setenv("MGKKT_NO_MAP", env)
            else:
                monkeypatch.delenv("MGKKT_NO_MAP", raising=False)
            s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu, precision=precision)
            f = s.rhs(yd)
            x = torch.zeros_like(f)
            for _ in range(3):
                s.cycle(f, x)
            xs.append(_host(x))
        monkeypatch.delenv("MGKKT_NO_MAP", raising=False)
        assert np.linalg.norm(xs[0] - xs[1]) <= bound * np.linalg.norm(xs[1]), precision


@pytest.mark.parametrize("smoother,gamma", [("lsgs", 1), ("ne", 1), ("slsgs", 2), ("lsgs", 2)])
@pytest.mark.parametrize("level", [6, 8])
def test_dense_map_equals_tail(torch_cuda, monkeypatch, smoother, gamma, level):
    # the dense map of the level-5 sub-cycle (one matrix-vector product per
    # coarse iterate) against the tail launch it replaces (MGKKT_NO_DENSE_MAP=1):
    # same iterates to rounding, for V- and W-cycles, in FP64 and FP32 refinement
    torch = torch_cuda
    mg = _mg()
    alpha = 1e-3
    nu = 1 if smoother == "slsgs" else 2
    yd = _dev(torch, workloads.desired_state(level, 3))
    for precision, bound in (("fp64", 1e-13), ("fp32_ir", 1e-5)):
        xs = []
        for env in (None, "1"):
            if env:
                monkeypatch.setenv("MGKKT_NO_DENSE_MAP", env)
            else:
                monkeypatch.delenv("MGKKT_NO_DENSE_MAP", raising=False)
            s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu, precision=precision)
            f = s.rhs(yd)
            x = torch.zeros_like(f)
            for _ in range(3):
                s.cycle(f, x)
            xs.append(_host(x))
        monkeypatch.delenv("MGKKT_NO_DENSE_MAP", raising=False)
        assert np.linalg.norm(xs[0] - xs[1]) <= bound * np.linalg.norm(xs[1]), precision


@pytest.mark.parametrize("smoother,nu,gamma", [("lsgs", 2, 1), ("lsgs", 3, 1), ("slsgs", 1, 1), ("slsgs", 2, 2),
                                               ("cgs", 2, 1), ("cgs", 3, 2)])
@pytest.mark.parametrize("level", [9, 10])
def test_sweep_pairs_match_single_sweeps(torch_cuda, monkeypatch, smoother, nu, gamma, level):
    # two sweeps per launch on the coarse levels up to 513^2 (halo 28, or 14
    # for the collective smoother; corrections of both sweeps in LDS; 17 x 17
    # and 33 x 33 tiles) against one launch per sweep (MGKKT_NO_SWEEP2=1)
    torch = torch_cuda
    mg = _mg()
    alpha = 1e-3
    yd = _dev(torch, workloads.desired_state(level, 4))
    for precision, bound in (("fp64", 1e-13), ("fp32_ir", 1e-5)):
        xs = []
        for env in (None, "1"):
            if env:
                monkeypatch.setenv("MGKKT_NO_SWEEP2", env)
            else:
                monkeypatch.delenv("MGKKT_NO_SWEEP2", raising=False)
            s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu, precision=precision)
            f = s.rhs(yd)
            x = torch.zeros_like(f)
            for _ in range(3):
                s.cycle(f, x)
            xs.append(_host(x))
        monkeypatch.delenv("MGKKT_NO_SWEEP2", raising=False)
        assert np.linalg.norm(xs[0] - xs[1]) <= bound * np.linalg.norm(xs[1]), precision


@pytest.mark.parametrize("smoother,nu1,nu2,gamma", [("lsgs", 2, 2, 1), ("lsgs", 1, 1, 1), ("lsgs", 3, 2, 2),
                                                    ("lsgs", 2, 1, 1), ("slsgs", 1, 1, 1), ("slsgs", 2, 2, 2),
                                                    ("cgs", 2, 2, 1), ("cgs", 1, 3, 2)])
@pytest.mark.parametrize("level", [6, 10, 11])
def test_fused_transfers_match_separate_kernels(torch_cuda, monkeypatch, smoother, nu1, nu2, gamma, level):
    # the restriction in the last pre-smoothing launch (one more ring of
    # final residuals, f_c written from LDS) and the prolongation with the new
    # residual in the first post-smoothing launch (x + P x_c and f - A (x + P
    # x_c) formed on the tile's region) against the separate restriction and
    # prolongation-residual kernels (MGKKT_NO_FUSED_TRANSFERS=1)
    torch = torch_cuda
    mg = _mg()
    if level == 11 and (nu1, nu2, gamma) not in ((2, 2, 1), (1, 3, 2)):
        pytest.skip("2049^2: the default V(2,2) and one W-cycle case")
    alpha = 1e-4
    yd = _dev(torch, workloads.desired_state(level, 6))
    for precision, bound in (("fp64", 1e-13), ("fp32_ir", 1e-5)):
        xs = []
        for env in (None, "1"):
            if env:
                monkeypatch.setenv("MGKKT_NO_FUSED_TRANSFERS", env)
            else:
                monkeypatch.delenv("MGKKT_NO_FUSED_TRANSFERS", raising=False)
            s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu1, nu2=nu2, precision=precision)
            monkeypatch.delenv("MGKKT_NO_FUSED_TRANSFERS", raising=False)
            f = s.rhs(yd)
            x = torch.zeros_like(f)
            for _ in range(3):
                s.cycle(f, x)
            xs.append(_host(x))
            s.close()
        assert np.all(np.isfinite(xs[0]))
        assert np.linalg.norm(xs[0] - xs[1]) <= bound * np.linalg.norm(xs[1]), precision


@pytest.mark.parametrize("smoother,nu", [("lsgs", 2), ("slsgs", 1), ("cgs", 2)])
def test_sweep_norm_solve(torch_cuda, monkeypatch, smoother, nu):
    # FP64 solves take each iterate's norm from the residual the last sweep
    # leaves; at convergence the recomputed f - A x is checked.  Against the
    # path that recomputes the residual after every iterate: same cycle count
    # (to one) and solution, and the reported relative residual is the true
    # one (Euclidean norm, recomputed here)
    torch = torch_cuda
    mg = _mg()
    level, alpha = 9, 1e-4
    yd = _dev(torch, workloads.desired_state(level, 2))
    out = []
    for env in (None, "1"):
        if env:
            monkeypatch.setenv("MGKKT_NO_SWEEP_NORM", env)
        s = mg.Solver(level, alpha, smoother=smoother, nu1=nu, nu2=nu, norm="l2")
        monkeypatch.delenv("MGKKT_NO_SWEEP_NORM", raising=False)
        f = s.rhs(yd)
        x, it, rel, st = s.solve(f, tol=1e-10)
        assert st == mg.MG_OK and rel <= 1e-10
        _, nrm = s.residual(f, x, norm=True)
        fn = float(torch.linalg.norm(f))
        assert rel == pytest.approx(nrm / fn, rel=1e-12)
        out.append((_host(x), it))
    assert abs(out[0][1] - out[1][1]) <= 1
    assert np.linalg.norm(out[0][0] - out[1][0]) <= 1e-8 * np.linalg.norm(out[1][0])
    # a tolerance close to rounding still ends on the recomputed residual
    s = mg.Solver(level, alpha, smoother=smoother, nu1=nu, nu2=nu, norm="l2", max_cycles=80)
    f = s.rhs(yd)
    x, it, rel, st = s.solve(f, tol=1e-14, raise_on_error=False)
    if st == mg.MG_OK:
        _, nrm = s.residual(f, x, norm=True)
        assert nrm / float(torch.linalg.norm(f)) <= 1e-14


CYCLE_CASES = [
    (5, 1e-2, "lsgs", 1),
    (5, 1e-2, "ne", 1),
    (5, 1.0, "lsgs", 2),
    (5, 1e-8, "lsgs", 1),
    (7, 1e-4, "lsgs", 1),
    (7, 1e-4, "ne", 1),
    (7, 1.0, "slsgs", 1),
    (7, 1e-8, "cgs", 1),
    (8, 1.0, "cgs", 2),
    (10, 1e-3, "cgs", 1),
    (8, 1e-6, "lsgs", 2),
    (10, 1e-2, "lsgs", 1),
    (10, 1e-5, "slsgs", 1),
]


@pytest.mark.parametrize("level,alpha,smoother,gamma", CYCLE_CASES)
def test_cycle_parity(torch_cuda, level, alpha, smoother, gamma):
    torch = torch_cuda
    mg = _mg()
    nu = 1 if smoother == "slsgs" else 2
    s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu)
    h = oracle.Hierarchy(level, alpha, coarse=1)
    yd = workloads.desired_state(level, 1)
    f = h.rhs(yd)
    fg = s.rhs(_dev(torch, yd))
    xg = torch.zeros(h.ndof(), dtype=torch.float64, device="cuda")
    xo = np.zeros(h.ndof())
    for m in range(8):
        s.cycle(fg, xg)
        h.cycle(f, xo, smoother=smoother, order="col7", gamma=gamma, nu1=nu, nu2=nu)
        # y, lambda and the control u = lambda / alpha, each to 1e-12
        assert_fields(_host(xg), xo, 1e-12, alpha=alpha, what=f"cycle {m}")


@pytest.mark.parametrize("norm", ["l2", "linv"])
@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("smoother", ["ne", "lsgs", "cgs"])
def test_solve_parity(torch_cuda, alpha, smoother, norm):
    torch = torch_cuda
    mg = _mg()
    level = 6
    s = mg.Solver(level, alpha, smoother=smoother, norm=norm)
    h = oracle.Hierarchy(level, alpha, coarse=1)
    yd = workloads.desired_state(level, 2)
    f = h.rhs(yd)
    xo, it_o, hist = h.solve(f, tol=1e-10, smoother=smoother, order="col7", norm=norm)
    xg, it_g, rel, st = s.solve(s.rhs(_dev(torch, yd)), tol=1e-10)
    assert st == mg.MG_OK and rel <= 1e-10
    assert abs(it_g - it_o) <= 1
    assert_fields(_host(xg), xo, 1e-9, alpha=alpha)
    # the control from the library's kernel against the oracle's u = lambda / alpha
    ug = _host(s.control(xg))
    uo = h.control(xo)
    assert np.abs(ug - uo).max() <= 1e-9 * np.abs(uo).max()


def test_set_opts_rejects_unsupported_smoother(torch_cuda):
    # the patch smoother is Stokes-only: a Poisson context refuses it in
    # mg_set_opts as mg_setup does, and keeps its options
    mg = _mg()
    s = mg.Solver(5, 1e-2)
    with pytest.raises(mg.MGError) as e:
        s.set_opts(smoother="vanka")
    assert e.value.status == mg.MG_EUNSUPPORTED
    assert s.opts().smoother == mg.MG_LSGS
    st = mg.Solver(3, 1e-2, problem="stokes")
    with pytest.raises(mg.MGError) as e:
        st.set_opts(smoother="cgs")
    assert e.value.status in (mg.MG_EUNSUPPORTED,)


def test_run_to_run_bitwise(torch_cuda):
    torch = torch_cuda
    mg = _mg()
    level = 7
    s = mg.Solver(level, 1e-3)
    yd = _dev(torch, workloads.desired_state(level, 3))
    f = s.rhs(yd)
    a, _, _, _ = s.solve(f, tol=1e-10)
    b, _, _, _ = s.solve(f, tol=1e-10)
    assert torch.equal(a, b)


def test_error_paths(torch_cuda):
    torch = torch_cuda
    mg = _mg()
    level = 6
    s = mg.Solver(level, 1e-2, max_cycles=2)
    f = s.rhs(_dev(torch, workloads.desired_state(level, 1)))
    x, it, rel, st = s.solve(f, tol=1e-10, raise_on_error=False)
    assert st == mg.MG_ENOTCONV and it == 2 and rel > 1e-10
    fn = f.clone()
    fn[5] = float("nan")
    x, it, rel, st = s.solve(fn, tol=1e-10, raise_on_error=False)
    assert st == mg.MG_ENAN
    with pytest.raises(mg.MGError):
        s.solve(f, tol=-1.0)
    # below the FP64 rounding floor of the Euclidean ratio the solve reports a stall
    s3 = mg.Solver(10, 1.0, norm="l2")
    f3 = s3.rhs(_dev(torch, workloads.desired_state(10, 1)))
    x, it, rel, st = s3.solve(f3, tol=1e-14, raise_on_error=False)
    assert st == mg.MG_ESTALL and it < 100 and rel < 1e-6
    # an over-damped normal-equation smoother diverges and is reported
    s2 = mg.Solver(level, 1e-2, smoother="ne", tau=1.99, max_cycles=500)
    x, it, rel, st = s2.solve(f, tol=1e-10, raise_on_error=False)
    assert st in (mg.MG_EDIVERGE, mg.MG_ENAN, mg.MG_ENOTCONV)


@pytest.mark.parametrize("smoother", ["lsgs", "cgs"])
@pytest.mark.parametrize("alpha", [1e-8, 1e-4, 1.0])
def test_fp32_refinement_reaches_tolerance(torch_cuda, alpha, smoother):
    torch = torch_cuda
    mg = _mg()
    level = 8
    h = oracle.Hierarchy(level, alpha, coarse=1)
    yd = workloads.desired_state(level, 2)
    xo, _, _ = h.solve(h.rhs(yd), tol=1e-12, smoother=smoother, order="col7")
    s = mg.Solver(level, alpha, precision="fp32_ir", smoother=smoother)
    xg, it, rel, st = s.solve(s.rhs(_dev(torch, yd)), tol=1e-10)
    assert st == mg.MG_OK and rel <= 1e-10
    # final error of FP32 cycles + FP64 refinement against the FP64 oracle,
    # per field: a solve to 1e-10 in the L^-1 norm leaves ~1e-10 per field
    err = assert_fields(_host(xg), xo, 1e-8, alpha=alpha)
    print(f"fp32 refinement vs FP64 oracle, level {level}, alpha {alpha}: {err}")


@pytest.mark.parametrize("smoother,nu1,nu2,inner", [("lsgs", 2, 2, 2), ("lsgs", 1, 1, 1), ("slsgs", 1, 1, 1),
                                                    ("cgs", 1, 3, 2), ("ne", 2, 2, 1), ("lsgs", 0, 2, 1)])
def test_fp32_refinement_step_variants(torch_cuda, smoother, nu1, nu2, inner):
    # refinement steps of a solve: the FP64 residual pass leaves r / ||f|| in
    # FP32, the step's first FP32 pre-smoothing launch takes the iterate as
    # zero (tile smoothers with nu1 >= 1; otherwise x32 is cleared), later
    # inner cycles start from the current x32; against the FP64 oracle solve,
    # per field
    torch = torch_cuda
    mg = _mg()
    level, alpha = 8, 1e-4
    h = oracle.Hierarchy(level, alpha, coarse=1)
    yd = workloads.desired_state(level, 3)
    xo, _, _ = h.solve(h.rhs(yd), tol=1e-12, smoother="lsgs", order="col7")
    s = mg.Solver(level, alpha, precision="fp32_ir", smoother=smoother, nu1=nu1, nu2=nu2, inner_cycles=inner,
                  max_cycles=400)
    xg, it, rel, st = s.solve(s.rhs(_dev(torch, yd)), tol=1e-10)
    assert st == mg.MG_OK and rel <= 1e-10
    assert_fields(_host(xg), xo, 1e-8, alpha=alpha)


@pytest.mark.parametrize("smoother", ["lsgs", "cgs"])
def test_full_size_cycle_parity(torch_cuda, smoother):
    # the benchmark's size (2049^2 vertices), one V(2,2) cycle from zero
    torch = torch_cuda
    mg = _mg()
    level, alpha = 11, 1e-4
    yd = workloads.desired_state(level, 2)
    s = mg.Solver(level, alpha, smoother=smoother)
    fg = s.rhs(_dev(torch, yd))
    xg = torch.zeros(s.vec_len(), dtype=torch.float64, device="cuda")
    s.cycle(fg, xg)
    xgh = _host(xg)
    h = oracle.Hierarchy(level, alpha, coarse=1)
    f = h.rhs(yd)
    assert _relmax(_host(fg), f) < 1e-14
    xo = np.zeros(h.ndof())
    h.cycle(f, xo, smoother=smoother, order="col7")
    assert_fields(xgh, xo, 1e-12, alpha=alpha)


def test_level12_tile_sweeps_match_phase_kernels(torch_cuda, monkeypatch):
    # 4097^2 vertices (33.6 M unknowns, the largest level mg_setup accepts;
    # 56 x 56 tiles on the finest level): one V(2,2) cycle from zero with the
    # tile sweeps and the folded transfers against the same cycle with one
    # launch per colour phase and separate transfer kernels (an independent
    # path, checked against the oracle at the smaller levels), per field; then
    # a solve to 1e-10 whose cycle count is mesh-independent (within 2 of the
    # 2049^2 solve's)
    torch = torch_cuda
    mg = _mg()
    level, alpha = 12, 1e-4
    yd = _dev(torch, workloads.desired_state(level, 2))
    xs = []
    for env in (None, "1"):
        if env:
            monkeypatch.setenv("MGKKT_PHASE_KERNELS", env)
        s = mg.Solver(level, alpha)
        monkeypatch.delenv("MGKKT_PHASE_KERNELS", raising=False)
        f = s.rhs(yd)
        x = torch.zeros_like(f)
        s.cycle(f, x)
        xs.append(_host(x))
        del x, f
        s.close()
    assert_fields(xs[0], xs[1], 1e-12, alpha=alpha)
    s = mg.Solver(level, alpha)
    f = s.rhs(yd)
    x, it12, rel, st = s.solve(f, tol=1e-10)
    assert st == mg.MG_OK and rel <= 1e-10
    del x, f
    s.close()
    s11 = mg.Solver(11, alpha)
    f11 = s11.rhs(_dev(torch, workloads.desired_state(11, 2)))
    _, it11, rel11, st11 = s11.solve(f11, tol=1e-10)
    assert st11 == mg.MG_OK and abs(it12 - it11) <= 2, (it12, it11)


@pytest.mark.parametrize("alpha", [1e-8, 1e-4, 1.0])
def test_fp32_refinement_full_size(torch_cuda, alpha):
    # the benchmark's size (2049^2 vertices): FP32 cycles inside FP64
    # refinement reach the FP64 tolerance (the outer residual is the FP64
    # residual kernel's) and the iterate agrees with the plain FP64 solve,
    # whose cycle matches the oracle at this size
    torch = torch_cuda
    mg = _mg()
    level = 11
    yd = _dev(torch, workloads.desired_state(level, 2))
    s32 = mg.Solver(level, alpha, precision="fp32_ir")
    s64 = mg.Solver(level, alpha)
    f = s64.rhs(yd)
    x32, it32, rel32, st32 = s32.solve(f, tol=1e-10)
    x64, it64, rel64, st64 = s64.solve(f, tol=1e-10)
    assert st32 == mg.MG_OK and st64 == mg.MG_OK and rel32 <= 1e-10 and rel64 <= 1e-10
    err = assert_fields(_host(x32), _host(x64), 1e-8, alpha=alpha)
    print(f"fp32 refinement vs FP64 solve at 2049^2, alpha {alpha}: {err}")


@pytest.mark.parametrize("smoother,gamma", [("lsgs", 1), ("slsgs", 2)])
def test_cycle_parity_coarse_level_2(torch_cuda, smoother, gamma):
    # coarsest level k0 = 2 (50 unknowns): the tail, its level-3 map and the
    # dense level-5 map are all built on the k0 = 2 hierarchy; four cycles
    # against the oracle on the same hierarchy
    torch = torch_cuda
    mg = _mg()
    level, alpha = 7, 1e-3
    nu = 1 if smoother == "slsgs" else 2
    s = mg.Solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu, coarse_level=2)
    h = oracle.Hierarchy(level, alpha, coarse=2)
    yd = workloads.desired_state(level, 5)
    f = h.rhs(yd)
    fg = s.rhs(_dev(torch, yd))
    xg = torch.zeros(h.ndof(), dtype=torch.float64, device="cuda")
    xo = np.zeros(h.ndof())
    for m in range(4):
        s.cycle(fg, xg)
        h.cycle(f, xo, smoother=smoother, order="col7", gamma=gamma, nu1=nu, nu2=nu)
        assert_fields(_host(xg), xo, 1e-12, alpha=alpha, what=f"cycle {m}")
