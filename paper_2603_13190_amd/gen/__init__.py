"""Native helpers of the input generator (host C, built with gcc).

placement.c: the acceptance loop of the random sequential addition of
particles.  It is part of the seeded input generator, not of the solver:
it is built into its own library, which neither the HIP library nor the
oracle links.
"""
import ctypes as C
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "placement.c")
LIB = os.path.join(HERE, "libplacement.so")
# no contraction into FMAs: the same roundings as the generator's Python loop
FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]

_lib = None


def build(verbose=False):
    cmd = ["gcc"] + FLAGS + ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    """The placement library (built on first use if missing), or None when
    no C compiler is available."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            try:
                build()
            except (OSError, subprocess.CalledProcessError):
                return None
        L = C.CDLL(LIB)
        L.place_create.restype = C.c_void_p
        L.place_create.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64]
        L.place_free.restype = None
        L.place_free.argtypes = [C.c_void_p]
        L.place_try.restype = C.c_int64
        L.place_try.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_double, C.c_double]
        _lib = L
    return _lib
