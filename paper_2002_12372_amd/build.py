"""Build libqqmc.so (HIP for gfx950 plus host C++) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqqmc.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["qqmc_kernels.hip", "qqmc_kernels_pair.hip", "qqmc_kernels_cur.hip",
           "qqmc_kernels_sob.hip", "qqmc_kernels_sob_model.hip", "qqmc_kernels_sob_batch.hip",
           "qqmc_kernels_model.hip", "qqmc_kernels_geo.hip", "qqmc_noalloc.hip",
           "qqmc_api.cpp",
           "qqmc_tables.cpp", "qqmc_plan.cpp",
           "qqmc_model.cpp", "qqmc_server.cpp"]

# gfx950 only; packed-FP32 instructions are kept out of the generated code.
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["hipcc", *HIP_FLAGS, "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-value", "-x", "c++",
                   "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError("hipcc failed for %s" % [s for s, r in zip(SOURCES, rc) if r])
    tmp = LIB + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
          "-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
