"""Build the HIP library libpentago.so for gfx950 (in-tree, with hipcc).

Every source is compiled to its own object in parallel (the sources share no
device code across files), then the objects are linked into one library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpentago.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["tables.cpp", "sweep.hip", "endgame.hip", "api.hip", "eval.hip", "debug.hip", "tune.hip", "batch.hip",
           "serve.hip", "symmetry.hip", "deep.hip", "noalloc.hip", "terminal.hip", "check.hip"]
HIPCC = "/opt/rocm/bin/hipcc"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-pthread"]


def _jobs():
    n = os.cpu_count() or 1
    return max(1, min(16, n, len(SOURCES)))


def build(verbose=False):
    """Compile every source into libpentago.so (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    pid = os.getpid()

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".%d.o" % pid)
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return src, obj, r.returncode, r.stdout

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = False
    for src, obj, rc, text in results:
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if lines and (verbose or rc):
            print("\n".join(lines), flush=True)
        if rc:
            print("compiling %s failed (%d)" % (src, rc), file=sys.stderr, flush=True)
            failed = True
    objs = [obj for _, obj, _, _ in results]
    try:
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc -c")
        tmp = LIB + ".tmp%d" % pid
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-pthread"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
