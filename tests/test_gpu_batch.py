"""GPU: batches of independent Poisson-control instances (mg_batch_*), each
on its own level with its own alpha and data, solved by batched V-cycles
(section 2) against the FP64 oracle and against one-instance solves."""
import os

import numpy as np
import pytest

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


# ragged mix of levels (6..8) and alphas; y_D seeds 3000 + i
LEVELS = [7, 6, 8, 6, 7]
ALPHAS = [1e-2, 1.0, 1e-4, 1e-8, 1e-6]


def _batch_inputs(torch, levels):
    return [_dev(torch, workloads.desired_state(l, 3000 + i)) for i, l in enumerate(levels)]


@pytest.mark.parametrize("smoother", ["lsgs", "ne", "slsgs", "cgs"])
def test_batch_cycles_match_oracle(torch_cuda, smoother):
    """Three batched V-cycles from x = 0 (max_cycles = 3): every instance equals
    three oracle cycles (7-colour order) to 1e-12."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    nu = 1 if smoother == "slsgs" else 2
    b = mg.Batch(LEVELS, ALPHAS, smoother=smoother, nu1=nu, nu2=nu, max_cycles=3)
    fs = b.rhs(_batch_inputs(torch, LEVELS))
    xs, cyc, rel, sts, st = b.solve(fs, tol=1e-30, raise_on_error=False)
    assert st == mg.MG_ENOTCONV and cyc == [3] * len(LEVELS) and sts == [mg.MG_ENOTCONV] * len(LEVELS)
    for i, (l, a) in enumerate(zip(LEVELS, ALPHAS)):
        h = oracle.Hierarchy(l, a, coarse=1)
        f = h.rhs(workloads.desired_state(l, 3000 + i))
        assert np.abs(_host(fs[i]) - f).max() <= 1e-14 * np.abs(f).max()
        xo = np.zeros(h.ndof())
        for _ in range(3):
            h.cycle(f, xo, smoother=smoother, order="col7", nu1=nu, nu2=nu)
        assert_fields(_host(xs[i]), xo, 1e-12, alpha=a, what=(i, l, a))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_matches_single_solves(torch_cuda, precision):
    """Full solves to 1e-10: the batch reproduces one-instance solves (same
    cycle counts, solutions equal to rounding) and each solution is within
    1e-9 (FP64) / 1e-8 (FP32 refinement) of the oracle's."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    b = mg.Batch(LEVELS, ALPHAS, precision=precision)
    yds = _batch_inputs(torch, LEVELS)
    fs = b.rhs(yds)
    xs, cyc, rel, sts, st = b.solve(fs, tol=1e-10)
    assert st == mg.MG_OK and all(r <= 1e-10 for r in rel)
    for i, (l, a) in enumerate(zip(LEVELS, ALPHAS)):
        s = mg.Solver(l, a, precision=precision)
        x1, it1, rel1, st1 = s.solve(s.rhs(yds[i]), tol=1e-10)
        assert st1 == mg.MG_OK and it1 == cyc[i], (i, it1, cyc[i])
        assert np.abs(_host(xs[i]) - _host(x1)).max() <= 1e-13 * np.abs(_host(x1)).max()
        h = oracle.Hierarchy(l, a, coarse=1)
        xo, _, _ = h.solve(h.rhs(workloads.desired_state(l, 3000 + i)), tol=1e-12)
        bound = 1e-9 if precision == "fp64" else 1e-8
        assert_fields(_host(xs[i]), xo, bound, alpha=a, what=i)


def test_batch_graph_replays_match_eager(torch_cuda, monkeypatch):
    """Graph replays and eager launches give bitwise the same iterates.  Both
    batches take the default tile shapes: the autotuner times its candidates,
    so two batches may pick different shapes (and round differently)."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    monkeypatch.setenv("MGKKT_NO_AUTOTUNE", "1")
    out = []
    for env in (None, "1"):
        if env:
            os.environ["MGKKT_NO_GRAPH"] = env
        try:
            b = mg.Batch(LEVELS, ALPHAS, precision="fp32_ir")
        finally:
            os.environ.pop("MGKKT_NO_GRAPH", None)
        fs = b.rhs(_batch_inputs(torch, LEVELS))
        xs, cyc, _, _, st = b.solve(fs, tol=1e-10)
        assert st == mg.MG_OK
        out.append(([_host(x) for x in xs], cyc))
    for a, c in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, c)
    assert out[0][1] == out[1][1]


def test_batch_instances_stop_independently(torch_cuda):
    """An instance that starts converged does no cycles and is left untouched;
    a second solve from the converged iterates does no cycles at all."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    b = mg.Batch(LEVELS, ALPHAS)
    fs = b.rhs(_batch_inputs(torch, LEVELS))
    fs[1].zero_()  # instance 1: f = 0, x = 0 is exact
    xs, cyc, rel, sts, st = b.solve(fs, tol=1e-10)
    assert st == mg.MG_OK and cyc[1] == 0 and not _host(xs[1]).any()
    assert all(c > 0 for i, c in enumerate(cyc) if i != 1)
    snap = [_host(x).copy() for x in xs]
    xs2, cyc2, _, _, st2 = b.solve(fs, xs, tol=1e-10)
    assert st2 == mg.MG_OK and cyc2 == [0] * len(LEVELS)
    for a, x in zip(snap, xs2):
        assert np.array_equal(a, _host(x))


def test_batch_64_instances_fp32_refinement(torch_cuda):
    """64 instances of 257^2, 513^2 and 1025^2 vertices, alpha log-uniform in
    [1e-8, 1], FP32 cycles inside FP64 refinement, to relative residual 1e-10;
    three sampled instances against one-instance FP64 solves."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    inst = workloads.batch_instances(64, seed=3)
    levels = [l for l, _, _ in inst]
    alphas = [a for _, a, _ in inst]
    b = mg.Batch(levels, alphas, precision="fp32_ir")
    yds = [_dev(torch, workloads.desired_state(l, sd)) for l, _, sd in inst]
    fs = b.rhs(yds)
    xs, cyc, rel, sts, st = b.solve(fs, tol=1e-10)
    print(f"64 instances: cycles {min(cyc)}..{max(cyc)}, max relres {max(rel):.2e}", flush=True)
    assert st == mg.MG_OK and all(r <= 1e-10 for r in rel)
    for i in (0, int(np.argmax(levels)), int(np.argmin(alphas))):
        l, a, _ = inst[i]
        s = mg.Solver(l, a)
        x1, _, _, st1 = s.solve(s.rhs(yds[i]), tol=1e-12, raise_on_error=False)
        assert st1 in (mg.MG_OK, mg.MG_ESTALL)
        err = assert_fields(_host(xs[i]), _host(x1), 1e-8, alpha=a, what=i)
        print(f"instance {i} (level {l}, alpha {a:.2e}) vs FP64 solve: {err}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_autotuned_tiles_match_default(torch_cuda, monkeypatch, precision):
    """The setup's autotuner picks a tile shape per level for the batched
    sweep; its solves equal those with the default shape (MGKKT_NO_AUTOTUNE=1)
    to rounding, with the same cycle counts, and every picked edge is one of
    the candidates."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    levels, alphas = [9, 7, 10, 8], [1e-4, 1.0, 1e-8, 1e-2]
    yds = _batch_inputs(torch, levels)
    out = []
    for env in (None, "1"):
        if env:
            monkeypatch.setenv("MGKKT_NO_AUTOTUNE", env)
        else:
            monkeypatch.delenv("MGKKT_NO_AUTOTUNE", raising=False)
        b = mg.Batch(levels, alphas, precision=precision)
        tiles = {l: b.sweep_tile(l) for l in range(6, 11)}
        fs = b.rhs(yds)
        xs, cyc, rel, sts, st = b.solve(fs, tol=1e-10)
        out.append(([_host(x) for x in xs], cyc, tiles))
        b.close()
    monkeypatch.delenv("MGKKT_NO_AUTOTUNE", raising=False)
    (xa, ca, ta), (xb, cb, tb) = out
    cand = {48, 65, 56} if precision == "fp64" else {48, 46, 65}
    assert all(t in cand for t in ta.values()) and all(t == 48 for t in tb.values()), (ta, tb)
    assert ca == cb
    for a, bb, al in zip(xa, xb, alphas):
        assert_fields(a, bb, 1e-9, alpha=al)


def test_batch_autotuned_cycles_match_oracle(torch_cuda):
    """With the autotuner's tile shapes (whatever it picks per level), three
    batched FP64 V-cycles of every instance equal three oracle cycles to 1e-12
    per field."""
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    levels, alphas = [9, 7, 10, 8], [1e-4, 1.0, 1e-8, 1e-2]
    b = mg.Batch(levels, alphas, max_cycles=3)
    tiles = {l: b.sweep_tile(l) for l in range(6, 11)}
    fs = b.rhs(_batch_inputs(torch, levels))
    xs, cyc, rel, sts, st = b.solve(fs, tol=1e-30, raise_on_error=False)
    assert cyc == [3] * len(levels), cyc
    print(f"autotuned tiles {tiles}", flush=True)
    for i, (l, a) in enumerate(zip(levels, alphas)):
        h = oracle.Hierarchy(l, a, coarse=1)
        f = h.rhs(workloads.desired_state(l, 3000 + i))
        xo = np.zeros(h.ndof())
        for _ in range(3):
            h.cycle(f, xo, smoother="lsgs", order="col7")
        assert_fields(_host(xs[i]), xo, 1e-12, alpha=a, what=(i, l, a, tiles))
