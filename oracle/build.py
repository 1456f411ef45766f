"""Build the CPU oracle library (test infrastructure).

g++ -O2 -fno-fast-math -ffp-contract=off keeps every floating-point operation
as written (no fused multiply-add contraction, no reassociation).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "janc_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
         "-shared", "-Wall"]


def build(verbose: bool = False) -> str:
    cmd = ["g++"] + FLAGS + ["-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
