"""Build the HIP library libsmc.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsmc.so")
SOURCES = ["kernels.hip", "ops_linreg.hip", "ops_egarch.hip", "ops_mixture64.hip",
           "ops_mixture32.hip", "ops_shapes32.hip", "ops_shapes64.hip", "ops_shapes_mix32.hip",
           "ops_shapes_mix64.hip", "batch.hip", "abi.hip", "noalloc.hip"]

HIPCC = "/opt/rocm/bin/hipcc"
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# hipcc's host pass does not know the device feature named above; harmless.
_NOISE = "is not a recognized feature for this target"


def _report(r, what):
    err = "\n".join(l for l in r.stderr.splitlines() if _NOISE not in l)
    if err.strip():
        sys.stderr.write(err + "\n")
    if r.returncode != 0:
        raise RuntimeError("hipcc failed: " + what)


def build(jobs: int = 0) -> str:
    """Compile every translation unit (in parallel, `jobs` at a time; 0 = one
    per source up to the CPU count) and link libsmc.so."""
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd))
    running = []
    for src, cmd in procs:
        while len(running) >= jobs:
            s0, p0 = running.pop(0)
            out, err = p0.communicate()
            _report(subprocess.CompletedProcess(p0.args, p0.returncode, out, err), s0)
        running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                              stderr=subprocess.PIPE, text=True)))
    for s0, p0 in running:
        out, err = p0.communicate()
        _report(subprocess.CompletedProcess(p0.args, p0.returncode, out, err), s0)
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp],
                       capture_output=True, text=True)
    _report(r, "link")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
