"""Builds the oracle's shared library (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librts_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "rts_oracle.c")
    # -ffp-contract=off keeps the float decisions unfused; no -march so that
    # no FMA instructions are available to the compiler either.
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-D_GNU_SOURCE", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB, src, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
