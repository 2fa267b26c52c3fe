"""Build step for the HIP library: compiles every kernel file for gfx950 with
hipcc and links libfmm_mi355.so next to this file."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm_mi355.so")

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# Files whose arithmetic feeds discrete decisions (tree, moments, walk) keep
# every floating-point operation separately rounded, as in their definition.
NO_CONTRACT = {"build.hip", "moments.hip", "walk.hip", "mutual.hip", "stats.hip",
               "integrate.hip", "asym.hip", "build_com.hip"}
SOURCES = ["api.cpp", "build.hip", "moments.hip", "walk.hip", "mutual.hip", "forces.hip",
           "stats.hip", "vjp.hip", "integrate.hip", "asym.hip", "build_com.hip"]


def _compile(src: str) -> str:
    out = os.path.join(OBJ, src + ".o")
    flags = list(COMMON)
    flags.append("-ffp-contract=off" if src in NO_CONTRACT else "-ffp-contract=fast")
    if src.endswith(".cpp"):
        flags = ["-x", "hip"] + flags
    cmd = ["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True)
    return out


def build(jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
