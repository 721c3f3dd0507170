"""Builds libglam.so (all HIP kernels and the C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libglam.so")
SOURCES = ["api.cpp", "project.hip", "binsort.hip", "render.hip", "loss.hip", "decode.hip", "optim.hip", "deform.hip", "epipolar.hip", "voxel.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are left to the compiler off: ordinary scalar code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


CEIL_LIB = os.path.join(HERE, "libglam_ceilings.so")


def build_ceilings(verbose: bool = False) -> str:
    """The ceiling microbenchmarks (include/glam_ceilings.h) as their own library."""
    tmp = CEIL_LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "ceilings.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, CEIL_LIB)
    return CEIL_LIB


def build(verbose: bool = False, jobs: int = 6) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = ["hipcc", "-c"] + FLAGS + inc + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        while len([p for p in procs if p.poll() is None]) >= jobs:
            procs[0].wait()
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_ceilings(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
