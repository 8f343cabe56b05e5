"""Host-side pins of the Stokes operator compression (no GPU): the stencil
classes of the rows, the merged LSGS groups (union of the two rows, both
coefficients, L^-1 per entry, N^-1 per group) and the patch classes of the
patch smoother (unknowns, LU factors and pivots recomputed from the CSR
entries, coefficient block over the union of the rows' columns) reproduce
the assembled operator exactly, and the groups / patches of one colour share
no residual entry.  The check program is built from the library's own host
code with hipcc."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1502_03917_amd", "csrc")


@pytest.mark.timeout(600)
def test_stokes_host_classes(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "stokes_classes_check"
    srcs = [os.path.join(HERE, "host", "stokes_classes_check.hip")] + [
        os.path.join(CSRC, f) for f in ("kernels.hip", "sweep.hip", "tail.hip", "host.hip")
    ]
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")] + srcs + ["-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_stokes_host_classes_sanitized(tmp_path):
    """The same check program with AddressSanitizer and UndefinedBehaviour-
    Sanitizer on the host code (the device code is built without them):
    the Stokes assembly, class compression, merged groups, entry codes and
    patch classes run without an out-of-bounds access, overflow or other
    undefined behaviour for n = 2 ... 64."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "stokes_classes_check_san"
    srcs = [os.path.join(HERE, "host", "stokes_classes_check.hip")] + [
        os.path.join(CSRC, f) for f in ("kernels.hip", "sweep.hip", "tail.hip", "host.hip")
    ]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")] + san + srcs + ["-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=900, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr

