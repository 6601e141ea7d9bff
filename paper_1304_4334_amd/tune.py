"""Autotuner of the batched M-step launch: times adaptive batches of the
given runs for several persistent wave counts and records the fastest in
tuned.json beside this file (read by smc_run_batch when waves=0 is passed
through `tuned_waves()`)."""
from __future__ import annotations

import json
import os
import time

import torch

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")


def tuned_waves(default: int = 2048) -> int:
    try:
        with open(TUNED) as f:
            return int(json.load(f).get("batch_waves", default))
    except (OSError, ValueError):
        return default


def tune_batch_waves(models, pops, seeds, candidates=(1024, 2048, 4096, 8192), out=TUNED):
    """Returns {waves: seconds} and stores the best choice in `out` (None:
    do not write)."""
    times = {}
    for w in candidates:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _lib.smc_run_batch(models, pops, seeds, waves=w, Lmax=2048, RmaxRec=64)
        torch.cuda.synchronize()
        times[w] = time.perf_counter() - t0
    best = min(times, key=times.get)
    if out:
        with open(out, "w") as f:
            json.dump({"batch_waves": best, "seconds": times}, f, indent=1)
    return times


if __name__ == "__main__":
    import sys

    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synthdata as SD

    specs = SD.batched_specs()
    ms = [_lib.Model.from_workload(w, precision=_lib.SMC_FP32) for w in specs]
    ps = [_lib.Population(m, w.J, w.N, max_chunk=256) for m, w in zip(ms, specs)]
    out = sys.argv[1] if len(sys.argv) > 1 else TUNED
    print(tune_batch_waves(ms, ps, list(range(1, 33)), out=out))
