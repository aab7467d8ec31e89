"""Build the oracle's shared library with gcc (plain IEEE FP64, no FMA
contraction).  Test infrastructure: see ldpm_oracle.c."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ldpm_oracle.c")
LIB = os.path.join(HERE, "libldpm_oracle.so")


COMMON = ["-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
          "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False):
    """The library the tests load (portable code: it travels with the tree)."""
    cmd = ["gcc", "-O2"] + COMMON + ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_native(path, verbose=False):
    """The same source optimised for the host it is built on
    (-O3 -march=native, still without FMA contraction or fast math, so the
    results are the same IEEE operations): for timing the oracle on the
    machine that runs it.  Built at run time into `path`, never shipped."""
    cmd = ["gcc", "-O3", "-march=native"] + COMMON + ["-o", path + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(path + ".tmp", path)
    return path, " ".join(["gcc", "-O3", "-march=native"] + COMMON)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
