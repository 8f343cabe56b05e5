"""GPU: mg_residual_nalloc (the entry point that allocates nothing; its norm
partial sums live in a static device array of the library) against
mg_residual on the same inputs, through the C ABI: two calls in a row on one
context, the second on a smaller level, then a Stokes context, and the size
limit of the static array."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _check(torch, s, level, seed):
    """One mg_residual_nalloc call against mg_residual on seeded f and x of
    `level`: r bit-identical (same kernel, same inputs), norm within one
    rounding of the host square root mg_residual takes."""
    n = s.level_len(level)
    f = torch.from_numpy(workloads.uniform(n, seed)).cuda()
    x = torch.from_numpy(workloads.uniform(n, seed + 1)).cuda()
    r_ref, nrm_ref = s.residual(f, x, level=level, norm=True)
    r = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    nrm = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"no-alloc residual: level {level}, {n} unknowns, seed {seed}", flush=True)
    s.residual_nalloc(f, x, r, nrm, level=level)
    torch.cuda.synchronize()
    assert torch.equal(r, r_ref), float(torch.max(torch.abs(r - r_ref)))
    got = float(nrm.item())
    assert np.isfinite(got) and abs(got - nrm_ref) <= 2e-16 * nrm_ref, (got, nrm_ref)
    # the norm is that of the returned residual
    assert abs(got - float(torch.linalg.vector_norm(r_ref))) <= 1e-13 * nrm_ref


def test_no_alloc_residual_matches_mg_residual(torch_cuda):
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    s = mg.Solver(11, 1e-4)
    _check(torch, s, 11, 41)  # 2049^2 vertices: 16,929 partial sums
    _check(torch, s, 7, 43)   # then a smaller level on the same context
    s.close()
    st = mg.Solver(5, 1e-2, problem="stokes")
    _check(torch, st, 5, 45)
    _check(torch, st, 3, 47)
    st.close()


def test_no_alloc_residual_rejects_oversized_level(torch_cuda):
    import paper_1502_03917_amd as mg

    torch = torch_cuda
    s = mg.Solver(12, 1.0)  # 4097^2 vertices: 66,625 partial sums > 32,768
    n = s.vec_len()
    f = torch.zeros(n, dtype=torch.float64, device="cuda")
    r = torch.zeros(n, dtype=torch.float64, device="cuda")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = mg.lib().mg_residual_nalloc(s._h, 12, f.data_ptr(), f.data_ptr(), r.data_ptr(), nrm.data_ptr(), None)
    assert st == mg.MG_EUNSUPPORTED
    assert b"static scratch" in mg.lib().mg_last_error(s._h)
    # the level below still works on the same context
    _check(torch, s, 11, 49)
    s.close()
