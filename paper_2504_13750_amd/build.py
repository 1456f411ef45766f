"""Build libjanc.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Flags: -O3; FP64 everywhere; packed-FP32 instruction selection disabled
(the library has no FP32 arithmetic on its hot path, and the packed forms are
kept out deliberately); a*b+c is fused into an FMA only within one source
expression (-ffp-contract=on), so that the rounding of a formula does not depend
on how the compiler schedules a particular kernel instantiation: tile shapes and
launch forms give bitwise-identical results.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjanc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["janc_kernels.hip", "janc_adjoint.hip", "janc_regrid.hip", "janc_api.hip"]
# the detailed model's kernels: janc_species.hip once per species count (2 .. 12)
SPECIES = list(range(2, 13))
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-value", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for ns in SPECIES:
        obj = os.path.join(CSRC, f"janc_species_{ns}.o")
        cmds.append([HIPCC] + FLAGS + [f"-DJANC_NS={ns}", "-c", os.path.join(CSRC, "janc_species.hip"),
                                       "-o", obj])
        objs.append(obj)
    # the largest translation units first, at most one compiler per host core
    cmds.sort(key=lambda c: "janc_species" not in c[-3])
    with cf.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 4)) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        list(ex.map(lambda c: subprocess.run(c, check=True), cmds))
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
