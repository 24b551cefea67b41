"""Build the msv HIP library for gfx950 in-tree (libmsv.so next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmsv.so")
SOURCES = ["plan.hip", "tabulate.hip", "assemble.hip", "lu.hip", "solve.hip", "trsv.hip", "fields.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wno-unused-command-line-argument"]


# per-file flags: the tabulation kernel is compiled without machine-level
# loop-invariant hoisting, which would keep dozens of 64-bit constants live
# across its sampling loop and halve its occupancy
EXTRA = {"tabulate.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False, jobs: int = 5) -> str:
    """Compile every source for gfx950 and link libmsv.so (always rebuilds)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

    def compile_one(src):
        obj = os.path.join(SRC, src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(SRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
