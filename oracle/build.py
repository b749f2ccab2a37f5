"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle_fsmi.so.

Plain gcc, -O2, no fast-math, no FMA contraction, OpenMP over beams.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_fsmi.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "fsmi_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
