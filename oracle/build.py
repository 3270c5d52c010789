"""Build the oracle's C core (test infrastructure only).

Compiles ``dedisp_ref.c`` with gcc into ``_liboracle.so`` next to this file.
Plain ``-O2``, no ``-march=native`` (the library may run on another host),
no fast-math and no FMA contraction, so every FP64 add happens as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dedisp_ref.c")
LIB = os.path.join(HERE, "_liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-std=c99", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
