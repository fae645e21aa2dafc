"""The algorithmic FP64 operations per node that the benchmark's roofline divides
by the residual's time are the ones the op-counting build of the device
arithmetic reports (csrc/opcount.cpp, a host program: CPU only).  The counting
build takes a division or reciprocal as one operation however the device forms it."""
import re

import pytest

import bench
from paper_2107_12027_amd import build


def test_roofline_op_counts_match_the_counter():
    out = build.opcount()
    got = {(int(d), p): float(v) for d, p, v in
           re.findall(r"dim (\d) (RHD|RMHD):.*per node \(all \d directions\) ([\d.]+) FP64 ops", out)}
    want = {(2, "RHD"): bench.RESIDUAL_FLOPS_PER_NODE_2D_RHD, (3, "RHD"): bench.RESIDUAL_FLOPS_PER_NODE_3D_RHD,
            (2, "RMHD"): bench.RESIDUAL_FLOPS_PER_NODE_2D_RMHD, (3, "RMHD"): bench.RESIDUAL_FLOPS_PER_NODE_3D_RMHD}
    assert set(got) == set(want), out
    for k, v in want.items():
        assert got[k] == pytest.approx(v, abs=0.05), (k, got[k], v)
