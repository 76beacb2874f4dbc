"""Build the HIP library libpentago.so for gfx950 (in-tree, with hipcc)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpentago.so")
SOURCES = ["tables.cpp", "sweep.hip", "endgame.hip", "api.hip", "eval.hip", "debug.hip", "tune.hip", "batch.hip",
           "serve.hip", "symmetry.hip",
           "deep.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-pthread"]


def build(verbose=False):
    """Compile every source into libpentago.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc"] + FLAGS + ["-x", "hip"] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
