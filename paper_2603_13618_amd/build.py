"""Builds liblks.so (the HIP kernels and the C ABI) for gfx950 with hipcc:
each source to an object in parallel, then one link.

    python -m paper_2603_13618_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblks.so")
SOURCES = ["lks_api.hip", "common.hip", "d2q9.hip", "d2q9_adjoint.hip", "d2q25.hip", "regrid.hip",
           "cluster.cpp", "macro.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMPILE = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]
LINK = ["--offload-arch=gfx950", "-fPIC", "-shared", "-fno-gpu-rdc", "-Wl,-z,defs"]


def _jobs():
    n = os.cpu_count() or 1
    cap = os.environ.get("MAX_JOBS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, min(n, len(SOURCES)))


def build(verbose=False):
    """Compile every source into paper_2603_13618_amd/liblks.so."""
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + COMPILE + ["-c"] + lang + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(_jobs()) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + LINK + ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
