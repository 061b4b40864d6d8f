"""Build the FP64 CPU oracle shared library (test infrastructure only).

Compiled for the baseline x86-64 target with no fast-math and no FMA, so the
oracle's rounding is the same on every host it runs on.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src: str = SRC, lib: str = LIB) -> str:
    cmd = ["gcc", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-O3", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function", "-o", lib + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
