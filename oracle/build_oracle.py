"""Build the CPU oracle's shared library (test infrastructure only).

``python -m oracle.build_oracle`` (or :func:`build`) compiles
``heatbath_oracle.c`` and ``green_cg.c`` with gcc and OpenMP into
``oracle/liboracle.so``.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "heatbath_oracle.c")
SRCS = [SRC, os.path.join(HERE, "green_cg.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
