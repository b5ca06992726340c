"""Build the C-ABI library libls.so in-tree for gfx950.

Host set-up (C++17, OpenMP) is compiled with g++; the device code and the
ABI layer with hipcc.  Run:  python -m paper_1509_05063_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libls.so")

HOST_SRC = ["ls_math.cpp", "ls_setup.cpp"]
DEV_SRC = ["ls_kernels.hip", "ls_api.hip", "ls_server.hip", "ls_conv3d.hip", "ls_fft3d.hip"]
ARCH = "gfx950"


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(["g++", "-std=c++17", "-O2", "-fPIC", "-fopenmp", "-I", INC, "-c",
                     os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEV_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(["hipcc", "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-I", INC, "-I", CSRC, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    procs = [subprocess.Popen(j) for j in jobs]
    for j in jobs:
        print(" ".join(j), flush=True)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError(f"compilation failed: {rc}")
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-fopenmp", "-o", LIB + ".tmp"] + objs)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
