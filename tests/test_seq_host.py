"""CPU test of the segment positions of the residual kernels: tests/seq_host_check.cpp
compiles es_seq.h for the host and compares its carried line / coordinate
bookkeeping with a plain division of every position."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_segment_positions_match_division(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    assert cxx is not None, "a host C++ compiler is required"
    exe = tmp_path / "seq_host_check"
    cmd = [cxx, "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "paper_2107_12027_amd", "csrc"),
           "-o", str(exe), os.path.join(ROOT, "tests", "seq_host_check.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout
