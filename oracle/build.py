"""Build the CPU oracle library (test infrastructure).

gcc, -O2, no floating-point contraction, no fast-math, glibc libm, single
threaded: every double operation in the oracle rounds once, in source order.
A second build of the same source with -fopenmp (liboracle_omp.so) spreads
the region evaluation over the host's cores, for timing only; its results
are the same, since each region's arithmetic is unchanged and every sum
stays sequential.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pagani_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(verbose: bool = False) -> str:
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        tmp = lib + ".tmp"
        cmd = ["gcc", *CFLAGS, *extra, "-o", tmp, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
