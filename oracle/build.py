"""Builds the CPU oracle shared library (plain C, FP64, OpenMP).

Built with -ffp-contract=off so that no multiply-add is fused except where the
source writes fma() explicitly, and without -ffast-math.  The target is
x86-64-v3 so the library runs on any AVX2 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["oracle.c", "surfel.c", "posegraph.c"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           *[os.path.join(HERE, f) for f in SOURCES], "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
