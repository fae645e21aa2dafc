"""CPU test of the adjoint's backward sweeps: tests/vjp_host_check.cpp compiles
the device headers for the host (as the op count does) and compares the
hand-written pair-flux and face eigen-structure VJPs with dual-number
derivatives of the same device functions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_backward_sweeps_match_dual_numbers(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "vjp_host_check"
    cmd = [hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2107_12027_amd", "csrc"),
           "-o", str(exe), os.path.join(ROOT, "tests", "vjp_host_check.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout
