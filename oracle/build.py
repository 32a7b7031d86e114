"""Build the oracle's C library (gcc, FP64, OpenMP).  Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bfref.c")
LIB = os.path.join(HERE, "libbfref.so")


def build(verbose=False):
    # -ffp-contract=off keeps every product and sum a separately rounded FP64 op
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True), file=sys.stderr)
