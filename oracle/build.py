"""Build the FP64 CPU oracle (test infrastructure) into oracle/libmcg_oracle.so.

Plain gcc, OpenMP, and -ffp-contract=off so that every product and sum is
rounded exactly as written in mcg_oracle.c.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mcg_oracle.c")
LIB = os.path.join(HERE, "libmcg_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
