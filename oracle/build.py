"""Build the CPU oracle library (test infrastructure).

g++ -O2 -fno-fast-math -ffp-contract=off keeps every floating-point operation
as written (no fused multiply-add contraction, no reassociation).

The "fma" variant (liboracle_fma.so) is the same source built with fused
multiply-add contraction (-mfma -ffp-contract=fast): the same arithmetic with a
different rounding of every a*b+c. It is used only to measure the oracle's own
round-off floor (how far a change of rounding alone moves a result), never as
the oracle of a parity test.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "janc_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
         "-shared", "-Wall"]
VARIANTS = {None: ([], LIB),
            "fma": (["-mfma", "-ffp-contract=fast"], os.path.join(HERE, "liboracle_fma.so"))}


def lib_path(variant=None):
    return VARIANTS[variant][1]


def build(verbose: bool = False, variant=None) -> str:
    extra, out = VARIANTS[variant]
    flags = [f for f in FLAGS if not (extra and f.startswith("-ffp-contract"))] + extra
    cmd = ["g++"] + flags + ["-o", out + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, variant="fma" if "--fma" in sys.argv else None)
