"""Build libes.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2107_12027_amd.build            # compile
    python -m paper_2107_12027_amd.build --verbose

The library is written next to this file so that it travels with the source
tree; tests, smoke() and bench.py load it from there and never compile.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libes.so")
ARCH = "gfx950"

SOURCES = ["es_api.hip", "es_kernels.hip", "es_kernels_rmhd.hip", "es_adjoint.hip", "es_adjoint_rmhd.hip"]
HEADERS = ["es_common.h", "es_internal.h", "es_launch.h", "es_seq.h", "es_rhd.h", "es_rmhd.h", "es_dual.h", "es_pair_vjp.h", "es_eigen_vjp.h"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libes.so)")


FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
         # packed FP32 instructions are kept out of all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
         "-I" + INCLUDE, "-I" + CSRC]


def compile_command(src: str, obj: str):
    return [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs, out: str = LIB):
    return [hipcc(), "--offload-arch=" + ARCH, "-fPIC", "-shared", "-o", out] + list(objs)


def build(verbose: bool = False) -> str:
    """Compile every source (one hipcc process each, in parallel) and link libes.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(src)[0] + ".o") for src in SOURCES]

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), max(1, (os.cpu_count() or 1) // 2))) as ex:
        results = list(ex.map(run, [compile_command(s, o) for s, o in zip(SOURCES, objs)]))
    for src, res in zip(SOURCES, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed compiling %s" % src)
        if verbose and res.stderr.strip():
            sys.stderr.write(res.stderr)
    tmp = LIB + ".tmp"
    res = run(link_command(objs, tmp))
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libes.so")
    os.replace(tmp, LIB)
    return LIB


def opcount() -> str:
    """Build and run the host op-counting program (csrc/opcount.cpp) that gives the
    algorithmic FP64 work per node of the residual; returns its report."""
    exe = os.path.join(ROOT, "_build", "opcount")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    cmd = [hipcc(), "-O1", "-std=c++17", "--offload-arch=" + ARCH, "-I" + INCLUDE, "-I" + CSRC, "-o", exe,
           os.path.join(CSRC, "opcount.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building opcount failed")
    return subprocess.run([exe], capture_output=True, text=True, check=True).stdout


if __name__ == "__main__":
    if "--opcount" in sys.argv:
        print(opcount(), end="")
    else:
        print(build(verbose="--verbose" in sys.argv))
