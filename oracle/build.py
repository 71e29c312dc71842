"""Builds the CPU oracle (test infrastructure) into oracle/libsidm_oracle.so.

Plain C, double precision, no fused multiply-add (-ffp-contract=off) so that
each expression is evaluated as written.  OpenMP parallelises the loops over
particles only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsidm_oracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "sidm_oracle.c")
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
