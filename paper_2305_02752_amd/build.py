"""Build libhemo.so (HIP kernels + C ABI) for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhemo.so")
SOURCES = ["api.hip", "lbm.hip", "ibm.hip", "membrane.hip", "binning.hip", "batch_kernel.hip",
           "batch_api.hip", "mesh_host.hip", "interior.hip", "packing.hip",
           "adjoint.hip", "cell.hip"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep packed fp32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, `jobs` at a time; 0: one per CPU,
    at most 16) and link libhemo.so."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src.replace(".hip", ".o"))
        cmds.append([hipcc, "-c", os.path.join(CSRC, src), "-o", obj] + [f for f in FLAGS if f != "-shared"])
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    n = jobs or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=n) as ex:
        list(ex.map(compile_one, cmds))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-o", tmp] + objs + ["-shared", "-fPIC", "--offload-arch=gfx950"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
