"""Build the FP64 oracle shared library (test infrastructure).

Plain gcc, -O2, no fast-math and no FP contraction so the neighbour predicate
evaluates exactly the IEEE operations written in the source; OpenMP for the
parallel-for over target particles.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sphx_oracle.c")
LIB = os.path.join(HERE, "liboracle_sphx.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
