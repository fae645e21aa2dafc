"""The roofline constants of the benchmark against their sources (CPU only).  The
algorithmic FP64 operations per node that the roofline divides
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


def test_roofline_traffic_matches_the_counter_summaries():
    # bench.py's HBM bytes per es_residual call are the totals of the committed
    # rocprofv3 counter summaries, one per workload
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    files = {"rhd3d_blast_128": "es_residual_hbm_counters_rhd3d_blast_128.txt",
             "rhd2d_quadrant_riemann_400_seed2": "es_residual_hbm_counters_rhd2d_quadrant_400.txt",
             "rmhd2d_rotor_512": "es_residual_hbm_counters_rmhd2d_rotor_512.txt"}
    assert set(files) == set(bench.RESIDUAL_TRAFFIC_BYTES)
    for name, f in files.items():
        text = open(os.path.join(root, "profiles", f)).read()
        total = re.search(r"= ([\d.]+) MB of HBM traffic", text)
        assert total is not None, f
        assert float(total.group(1)) * 1e6 == pytest.approx(bench.RESIDUAL_TRAFFIC_BYTES[name], rel=1e-6), name
