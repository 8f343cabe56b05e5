"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol its header declares, and rejects invalid arguments before any HIP call."""
import ctypes
import math
import os
import re

import pytest

import paper_1502_03917_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgkkt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mg.lib()
    names = _declared()
    assert "mg_setup" in names and "mg_solve" in names and "mg_cycle" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_opts():
    o = mg.default_opts("poisson")
    assert (o.smoother, o.nu1, o.nu2, o.gamma, o.coarse_level, o.precision) == (mg.MG_LSGS, 2, 2, 1, 1, mg.MG_FP64)
    # tau <= 0: the context picks section 3's damping for its problem and smoother
    assert o.tau < 0 and o.max_cycles == 200 and o.inner_cycles == 1
    assert o.norm == mg.MG_NORM_LINV
    assert mg.default_opts("stokes").tau < 0


def _setup(level=5, alpha=1e-2, problem=0, **kw):
    L = mg.lib()
    o = L.mg_default_opts(problem)
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    st = L.mg_setup(level, alpha, problem, ctypes.byref(o), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("level", [-1, 0, 1, 13, 40])
def test_setup_rejects_levels(level):
    assert _setup(level=level)[0] == mg.MG_EINVAL


@pytest.mark.parametrize("alpha", [0.0, -1.0, math.nan, math.inf, -math.inf])
def test_setup_rejects_alpha(alpha):
    st, h = _setup(alpha=alpha)
    assert st == mg.MG_EINVAL and not h.value


@pytest.mark.parametrize("field,value", [("smoother", 5), ("smoother", -1), ("gamma", 0), ("gamma", 3),
                                         ("tau", 2.5), ("tau", math.nan), ("coarse_level", 0),
                                         ("coarse_level", 4), ("precision", 2), ("nu1", -1), ("max_cycles", -5),
                                         ("inner_cycles", 0), ("norm", 2), ("norm", -1)])
def test_setup_rejects_options(field, value):
    assert _setup(**{field: value})[0] == mg.MG_EINVAL


@pytest.mark.parametrize("problem,field,value", [(0, "smoother", 4), (1, "smoother", 3), (1, "coarse_level", 3)])
def test_setup_unsupported_combinations(problem, field, value):
    # patch smoother is Stokes-only, collective point smoother Poisson-only; the
    # bordered Stokes coarse solve holds at most 248 unknowns (coarse level <= 2)
    assert _setup(level=5, problem=problem, **{field: value})[0] == mg.MG_EUNSUPPORTED


@pytest.mark.parametrize("level", [11, 12])
def test_setup_stokes_level_cap(level):
    # the Stokes host assembly keeps 32-bit row pointers: levels above 10 are
    # refused before any allocation
    st, h = _setup(level=level, problem=mg.MG_STOKES)
    assert st == mg.MG_EUNSUPPORTED and not h.value


def test_host_allocation_failure_is_a_status(tmp_path):
    """A std::bad_alloc inside an entry point comes back as MG_ENOMEM with the
    output handle cleared (program tests/host/abi_alloc_check.cpp replaces
    operator new; no GPU is touched)."""
    import shutil
    import subprocess

    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    mg.lib()  # built library
    libdir = os.path.join(ROOT, "paper_1502_03917_amd")
    exe = tmp_path / "abi_alloc_check"
    subprocess.run([gxx, "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "abi_alloc_check.cpp"), "-L" + libdir, "-lmgkkt",
                    "-Wl,-rpath," + libdir, "-Wl,--allow-shlib-undefined", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")


def test_solve_status_check():
    # success passes; a stall passes only at the rounding floor; anything else raises
    mg.check_solve_status(mg.MG_OK, 1e-3, 1e-12)
    mg.check_solve_status(mg.MG_ESTALL, 4e-12, 1e-12)
    mg.check_solve_status(mg.MG_ESTALL, 5e-9, 1e-8)
    for st, rel in [(mg.MG_ESTALL, 2e-11), (mg.MG_ESTALL, 0.5), (mg.MG_ENOTCONV, 1e-13), (mg.MG_ENAN, math.nan),
                    (mg.MG_EDIVERGE, 1e4)]:
        with pytest.raises(mg.MGError):
            mg.check_solve_status(st, rel, 1e-12)


def test_setup_rejects_level_not_above_coarse():
    assert _setup(level=3, coarse_level=3)[0] == mg.MG_EINVAL


def test_setup_rejects_bad_problem_and_null_out():
    L = mg.lib()
    assert _setup(problem=7)[0] == mg.MG_EINVAL
    assert L.mg_setup(5, 1.0, 0, None, None) == mg.MG_EINVAL


def test_null_context_calls():
    L = mg.lib()
    assert L.mg_vec_len(None) == 0
    assert L.mg_level_len(None, 3) == 0
    assert L.mg_last_error(None) == b"no context"
    assert L.mg_cycle(None, None, None, None) == mg.MG_EINVAL
    g = ctypes.c_void_p(1)
    assert L.mg_capture_cycle(None, None, None, None, ctypes.byref(g)) == mg.MG_EINVAL
    assert g.value is None  # *out cleared on error
    assert L.mg_capture_cycle(None, None, None, None, None) == mg.MG_EINVAL
    assert L.mg_graph_launch(None, None) == mg.MG_EINVAL
    L.mg_graph_destroy(None)
    assert L.mg_solve(None, None, None, 1e-10, None, None, None) == mg.MG_EINVAL
    assert L.mg_rhs(None, None, None, None) == mg.MG_EINVAL
    assert L.mg_smooth(None, 3, None, None, 1, None) == mg.MG_EINVAL
    assert L.mg_timing_enable(None, 1) == mg.MG_EINVAL
    assert L.mg_control(None, None, None, None) == mg.MG_EINVAL
    assert L.mg_adjoint_grad(None, None, None, None, None, None) == mg.MG_EINVAL
    assert L.mg_batch_count(None) == 0
    assert L.mg_batch_vec_len(None, 0) == 0
    assert L.mg_batch_last_error(None) == b"no batch"
    assert L.mg_batch_rhs(None, None, None, None) == mg.MG_EINVAL
    assert L.mg_batch_solve(None, None, None, 1e-10, None, None, None, None) == mg.MG_EINVAL
    L.mg_batch_destroy(None)
    L.mg_destroy(None)


def _batch_setup(levels, alphas, **kw):
    L = mg.lib()
    o = L.mg_default_opts(0)
    for k, v in kw.items():
        setattr(o, k, v)
    n = len(levels)
    h = ctypes.c_void_p()
    st = L.mg_batch_setup(n, (ctypes.c_int * n)(*levels), (ctypes.c_double * n)(*alphas), 0, ctypes.byref(o),
                          ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("levels,alphas", [([], []), ([5], [1.0]), ([13], [1.0]), ([7, 8], [1.0, 0.0]),
                                           ([7], [math.nan]), ([7], [-1.0])])
def test_batch_setup_rejects_arguments(levels, alphas):
    st, h = _batch_setup(levels, alphas) if levels else (mg.lib().mg_batch_setup(0, None, None, 0, None,
                                                                                  ctypes.byref(ctypes.c_void_p())), None)
    assert st == mg.MG_EINVAL


@pytest.mark.parametrize("field,value", [("gamma", 2), ("inner_cycles", 2), ("coarse_level", 3)])
def test_batch_setup_unsupported_options(field, value):
    # rejected before any device allocation
    assert _batch_setup([7, 8], [1.0, 1e-4], **{field: value})[0] == mg.MG_EUNSUPPORTED


def test_strerror_covers_all_codes():
    L = mg.lib()
    texts = {st: L.mg_strerror(st).decode() for st in range(mg.MG_ESTALL, 1)}
    assert texts[mg.MG_OK] == "success"
    assert len(set(texts.values())) == len(texts)
    assert L.mg_strerror(5) == b"unknown status"
    assert L.mg_strerror(-99) == b"unknown status"
