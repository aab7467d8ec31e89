"""Build the oracle's shared library with gcc (plain IEEE FP64, no FMA
contraction).  Test infrastructure: see ldpm_oracle.c."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ldpm_oracle.c")
LIB = os.path.join(HERE, "libldpm_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
