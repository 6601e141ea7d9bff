"""Build the HIP library libsmc.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsmc.so")
SOURCES = ["kernels.hip", "batch.hip", "abi.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(jobs: int = 2) -> str:
    tmp = LIB + ".tmp"
    cmd = (["/opt/rocm/bin/hipcc"] + HIPCC_FLAGS
           + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
           + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp])
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("hipcc failed building libsmc.so")
    if err.strip():
        sys.stderr.write(err + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
