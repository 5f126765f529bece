"""Build the FP64 oracle (test infrastructure) as oracle/liboracle.so with gcc.

Portable x86-64-v2 code (it is built here and also loaded on other hosts);
FMA contraction off so that the oracle's double-precision arithmetic is the
plain IEEE sequence written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
# optimisation and portability flags (also reported with the oracle's timings)
FLAGS = ["-std=c11", "-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fopenmp"]


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
