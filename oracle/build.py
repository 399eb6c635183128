"""Compile the plain-C oracle into oracle/liboracle_resize.so (test infrastructure)."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "ref_resize.c")
LIBRARY = os.path.join(HERE, "liboracle_resize.so")


def build_oracle(verbose: bool = False) -> str:
    """Always recompiles; returns the library path. g++/gcc -O2, no fast-math."""
    tmp = LIBRARY + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           SOURCE, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build_oracle(verbose=True))
