"""Compile the FP64 oracle into a shared library beside its sources (test infrastructure)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcgdir_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "cgdir_oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-Wall", "-shared", "-fPIC",
           src, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
