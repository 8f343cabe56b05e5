"""GPU parity for Stokes control (eq. mp3, Taylor-Hood): operator, transfers,
coarse solve, every smoother (NE, LSGS and sLSGS in the colour order, the
patch smoother in 9 colours) and whole cycles against the FP64 oracle, plus
full solves in FP64 and FP32 refinement (through the C ABI)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from fieldwise import assert_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _solver(level, alpha, **kw):
    import paper_1502_03917_amd as mg

    return mg.Solver(level, alpha, problem="stokes", **kw)


@pytest.mark.parametrize("alpha", [1.0, 1e-4])
def test_stokes_operator_transfers_and_coarse_solve(torch_cuda, alpha):
    torch = torch_cuda
    level = 3
    s = _solver(level, alpha)
    h = oracle.Hierarchy(level, alpha, coarse=1, problem="stokes")
    n = h.ndof()
    assert s.vec_len() == n and s.level_len(2) == h.ndof(2)
    x = workloads.uniform(n, 71)
    f = workloads.uniform(n, 72)
    A = h.matrix("A")
    assert _rel(_host(s.apply(_dev(torch, x))), A @ x) < 1e-13
    r, nrm = s.residual(_dev(torch, f), _dev(torch, x), norm=True)
    assert _rel(_host(r), f - A @ x) < 1e-13
    assert nrm == pytest.approx(np.linalg.norm(f - A @ x), rel=1e-12)
    vd = workloads.desired_velocity(level, 7)
    assert _rel(_host(s.rhs(_dev(torch, vd))), h.rhs(vd)) < 1e-14
    P = sp.block_diag([h.matrix("P")] * 2 + [h.matrix("P2")] + [h.matrix("P")] * 2 + [h.matrix("P2")]).tocsr()
    rc = _host(s.restrict(_dev(torch, f)))
    assert _rel(rc, P.T @ f) < 1e-14
    xc = workloads.uniform(h.ndof(2), 73)
    xg = _dev(torch, x)
    s.prolong_add(_dev(torch, xc), xg)
    assert _rel(_host(xg), x + P @ xc) < 1e-14
    A1 = h.matrix("A", 1)
    b1 = A1 @ workloads.uniform(h.ndof(1), 74)  # consistent right-hand side
    assert _rel(_host(s.coarse_solve(_dev(torch, b1))), h.coarse_solve(b1)) < 1e-10


@pytest.mark.parametrize("smoother,order", [("ne", "col7"), ("lsgs", "col7"), ("slsgs", "col7"), ("vanka", "col7")])
@pytest.mark.parametrize("alpha", [1.0, 1e-2])
def test_stokes_smoothing_step(torch_cuda, smoother, order, alpha):
    torch = torch_cuda
    level = 3
    s = _solver(level, alpha, smoother=smoother)
    h = oracle.Hierarchy(level, alpha, coarse=1, problem="stokes")
    n = h.ndof()
    x0 = workloads.uniform(n, 81)
    f = workloads.uniform(n, 82)
    r0 = f - h.matrix("A") @ x0
    xo, ro = x0.copy(), r0.copy()
    h.smooth(xo, ro, smoother=smoother, order=order)
    xg, rg = _dev(torch, x0), _dev(torch, r0)
    s.smooth(xg, rg)
    assert _rel(_host(xg), xo) < 1e-12
    assert _rel(_host(rg), ro) < 1e-11


@pytest.mark.parametrize("smoother", ["lsgs", "slsgs"])
@pytest.mark.parametrize("level", [2, 4, 5])
def test_stokes_lsgs_steps(torch_cuda, smoother, level):
    """Two smoothing steps: levels up to 4 run every phase of both steps in one
    workgroup (an odd number of phases for LSGS, even for sLSGS), level 5
    launches each colour phase."""
    torch = torch_cuda
    s = _solver(level, 1e-2, smoother=smoother)
    h = oracle.Hierarchy(level, 1e-2, coarse=1, problem="stokes")
    n = h.ndof()
    x0 = workloads.uniform(n, 91)
    f = workloads.uniform(n, 92)
    r0 = f - h.matrix("A") @ x0
    xo, ro = x0.copy(), r0.copy()
    for _ in range(2):
        h.smooth(xo, ro, smoother=smoother, order="col7")
    xg, rg = _dev(torch, x0), _dev(torch, r0)
    s.smooth(xg, rg, steps=2)
    assert _rel(_host(xg), xo) < 1e-12
    assert _rel(_host(rg), ro) < 1e-11


def test_stokes_wg_sweep_matches_phase_launches(torch_cuda, monkeypatch):
    """The one-workgroup sweep of a small level against a launch per colour
    phase (MGKKT_NO_WG_SWEEP=1) on the same input, three sLSGS steps."""
    torch = torch_cuda
    monkeypatch.setenv("MGKKT_NO_WG_SWEEP", "1")
    s_ph = _solver(4, 1e-4, smoother="slsgs")
    monkeypatch.delenv("MGKKT_NO_WG_SWEEP")
    s_wg = _solver(4, 1e-4, smoother="slsgs")
    n = s_wg.vec_len()
    x0 = workloads.uniform(n, 93)
    r0 = workloads.uniform(n, 94)
    out = []
    for s in (s_ph, s_wg):
        xg, rg = _dev(torch, x0), _dev(torch, r0)
        s.smooth(xg, rg, steps=3)
        out.append((_host(xg), _host(rg)))
    assert _rel(out[1][0], out[0][0]) < 1e-13
    assert _rel(out[1][1], out[0][1]) < 1e-13


@pytest.mark.parametrize("level,smoother,precision", [(5, "lsgs", "fp64"), (7, "slsgs", "fp64"), (8, "lsgs", "fp64"),
                                                     (7, "lsgs", "fp32_ir")])
def test_stokes_lattice_phases_match_records(torch_cuda, monkeypatch, level, smoother, precision):
    """The lattice path of the LSGS colour phases (the records of the interior
    groups formed from their index) against the record path of every group
    (MGKKT_NO_STOKES_LATTICE=1): three smoothing steps on the same input, and
    three FP32-refinement iterates, per field."""
    torch = torch_cuda
    monkeypatch.setenv("MGKKT_NO_STOKES_LATTICE", "1")
    s_rec = _solver(level, 1e-2, smoother=smoother, precision=precision, max_cycles=3)
    monkeypatch.delenv("MGKKT_NO_STOKES_LATTICE")
    s_lat = _solver(level, 1e-2, smoother=smoother, precision=precision, max_cycles=3)
    n = s_lat.vec_len()
    x0 = workloads.uniform(n, 95)
    r0 = workloads.uniform(n, 96)
    out = []
    for s in (s_rec, s_lat):
        xg, rg = _dev(torch, x0), _dev(torch, r0)
        s.smooth(xg, rg, steps=3)
        out.append((_host(xg), _host(rg)))
    assert_fields(out[1][0], out[0][0], 1e-13, problem="stokes", level=level, what="x after 3 steps")
    assert_fields(out[1][1], out[0][1], 1e-12, problem="stokes", level=level, what="r after 3 steps")
    if precision == "fp32_ir":
        f = workloads.uniform(n, 97)
        sol = []
        for s in (s_rec, s_lat):
            xg = torch.zeros(n, dtype=torch.float64, device="cuda")
            s.solve(_dev(torch, f), xg, tol=1e-12, raise_on_error=False)
            sol.append(_host(xg))
        assert_fields(sol[1], sol[0], 1e-5, problem="stokes", level=level, what="3 FP32-refinement iterates")
    s_rec.close()
    s_lat.close()


def test_stokes_fp32_refinement_inner_cycles(torch_cuda):
    """Two FP32 cycles per refinement step (inner_cycles = 2) on Stokes: the
    solve reaches 1e-10 and agrees with the FP64 solve per field."""
    torch = torch_cuda
    level, alpha = 6, 1e-2
    s64 = _solver(level, alpha)
    s32 = _solver(level, alpha, precision="fp32_ir", inner_cycles=2)
    vd = _dev(torch, workloads.desired_velocity(level, 7))
    f = s64.rhs(vd)
    x64, it64, rel64, st64 = s64.solve(f, tol=1e-10)
    x32, it32, rel32, st32 = s32.solve(f, tol=1e-10)
    assert st64 == 0 and st32 == 0 and rel32 <= 1e-10
    assert it32 < it64  # two cycles per refinement iterate
    assert_fields(_host(x32), _host(x64), 1e-8, problem="stokes", level=level, what="inner_cycles 2")
    s64.close()
    s32.close()


STOKES_CYCLES = [
    (3, 1e-2, "lsgs", 1),
    (3, 1.0, "ne", 1),
    (3, 1e-6, "slsgs", 1),
    (4, 1e-2, "vanka", 1),
    (4, 1e-4, "lsgs", 2),
    (5, 1.0, "lsgs", 1),
    (6, 1e-2, "lsgs", 1),
]


@pytest.mark.parametrize("level,alpha,smoother,gamma", STOKES_CYCLES)
def test_stokes_cycle_parity(torch_cuda, level, alpha, smoother, gamma):
    torch = torch_cuda
    nu = 1 if smoother == "slsgs" else 2
    s = _solver(level, alpha, smoother=smoother, gamma=gamma, nu1=nu, nu2=nu)
    h = oracle.Hierarchy(level, alpha, coarse=1, problem="stokes")
    vd = workloads.desired_velocity(level, 7)
    f = h.rhs(vd)
    fg = s.rhs(_dev(torch, vd))
    xg = torch.zeros(h.ndof(), dtype=torch.float64, device="cuda")
    xo = np.zeros(h.ndof())
    for m in range(5):
        s.cycle(fg, xg)
        h.cycle(f, xo, smoother=smoother, order="col7", gamma=gamma, nu1=nu, nu2=nu)
        # v1, v2, p, lambda1, lambda2, mu and the control u = lambda / alpha
        assert_fields(_host(xg), xo, 1e-12, "stokes", level, alpha, what=f"cycle {m}")


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("alpha", [1e-2, 1e-6])
def test_stokes_solve(torch_cuda, precision, alpha):
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    level = 5
    s = _solver(level, alpha, precision=precision)
    h = oracle.Hierarchy(level, alpha, coarse=1, problem="stokes")
    vd = workloads.desired_velocity(level, 7)
    xo, it_o, _ = h.solve(h.rhs(vd), tol=1e-11, smoother="lsgs", order="col7")
    xg, it, rel, st = s.solve(s.rhs(_dev(torch, vd)), tol=1e-10)
    assert st == mg.MG_OK and rel <= 1e-10
    bound = 1e-9 if precision == "fp64" else 1e-8
    err = assert_fields(_host(xg), xo, bound, "stokes", level, alpha)
    print(f"Stokes {precision} alpha {alpha} vs oracle: {err}", flush=True)
    # pressure and multiplier have zero mean
    w = np.asarray(h.matrix("Mp").sum(axis=1)).ravel()
    fl = h.fields()
    x = _host(xg)
    for t in (2, 5):
        assert abs(w @ x[fl[t]]) <= 1e-12 * np.abs(x[fl[t]]).max()


def test_stokes_graph_replays_match_eager(torch_cuda):
    torch = torch_cuda
    level, alpha = 5, 1e-2
    vd = workloads.desired_velocity(level, 7)
    out = []
    for env in (None, "1"):
        if env:
            os.environ["MGKKT_NO_GRAPH"] = env
        try:
            s = _solver(level, alpha, precision="fp32_ir")
        finally:
            os.environ.pop("MGKKT_NO_GRAPH", None)
        xg, it, rel, st = s.solve(s.rhs(_dev(torch, vd)), tol=1e-10)
        out.append((_host(xg), it))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.timeout(900)
def test_stokes_513_against_oracle(torch_cuda):
    """513^2 vertices (level 9, 4,712,454 unknowns, alpha = 1e-2).
    (1) One LSGS V-cycle from zero on the GPU equals the oracle's cycle per
    field to 1e-12, and the GPU residual of that iterate equals f - A x with
    the oracle's level-9 matrix.  (2) One patch-smoother V-cycle from zero
    against the oracle's.  (3) FP64 solves to 1e-10 and, for both alpha of the
    workload (1e-2, 1e-6), FP32 cycles inside FP64 refinement against the
    FP64 solve, per field."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    level = 9
    vd = workloads.desired_velocity(level, 7)
    print("Stokes 513^2: oracle hierarchy", flush=True)
    h = oracle.Hierarchy(level, 1e-2, coarse=1, problem="stokes")
    f = h.rhs(vd)
    s = _solver(level, 1e-2)
    assert s.vec_len() == 4 * 1023**2 + 2 * 513**2 == h.ndof()
    fg = s.rhs(_dev(torch, vd))
    assert _rel(_host(fg), f) < 1e-14
    xg = torch.zeros(h.ndof(), dtype=torch.float64, device="cuda")
    s.cycle(fg, xg)
    xo = np.zeros(h.ndof())
    h.cycle(f, xo, smoother="lsgs", order="col7")
    assert_fields(_host(xg), xo, 1e-12, "stokes", level, 1e-2, what="lsgs cycle")
    rg = s.residual(fg, xg)
    ro = f - h.matrix("A") @ _host(xg)
    assert _rel(_host(rg), ro) < 1e-12
    print("Stokes 513^2: patch smoother cycle", flush=True)
    sv = _solver(level, 1e-2, smoother="vanka")
    xv = torch.zeros(h.ndof(), dtype=torch.float64, device="cuda")
    sv.cycle(fg, xv)
    xvo = np.zeros(h.ndof())
    h.cycle(f, xvo, smoother="vanka", order="col7")
    assert_fields(_host(xv), xvo, 1e-12, "stokes", level, 1e-2, what="patch cycle")
    del h
    for alpha in (1e-2, 1e-6):
        print(f"Stokes 513^2: solves at alpha {alpha}", flush=True)
        s64 = _solver(level, alpha)
        s32 = _solver(level, alpha, precision="fp32_ir")
        fa = s64.rhs(_dev(torch, vd))
        x64, it64, rel64, st64 = s64.solve(fa, tol=1e-10)
        x32, it32, rel32, st32 = s32.solve(fa, tol=1e-10)
        assert st64 == mg.MG_OK and st32 == mg.MG_OK and rel64 <= 1e-10 and rel32 <= 1e-10
        assert it64 <= 40 and it32 <= 40
        err = assert_fields(_host(x32), _host(x64), 1e-8, "stokes", level, alpha)
        print(f"Stokes 513^2 alpha {alpha}: FP32 refinement vs FP64 solve {err}", flush=True)
