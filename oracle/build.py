"""Compile the FP64 CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain gcc, -O2 -ffp-contract=off (no fused multiply-add, no fast math), OpenMP
over component grids.  Run as ``python -m oracle.build`` or through the repo's
``__graft_entry__.build()``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-D_GNU_SOURCE", "-Wall", "-Wno-unused-function", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
