"""Autotuner of the launch shapes: times the random-walk step of each tuned
model (EGARCH(1,1) Gaussian, EGARCH(2) Student-t and egarch_23's
normal-mixture shocks, FP64 and FP32) at its workload's full size for every
launch shape (particles per block 64, 128 or 256; observations per load batch
4, 8 or 16), and whole adaptive batches of the batched workload for every
shape and several persistent wave counts, and records the fastest in
tuned.json beside this file.  Every shape gives the same results to the bit,
so the choice changes only the speed.

Run on the GPU:  python -m paper_1304_4334_amd.tune  [out.json]
                 python -m paper_1304_4334_amd.tune --only egarch23/fp32,egarch23/fp64
(the second form re-tunes the named steps and keeps every other entry)
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")
SHAPES = [(b, u) for b in (64, 128, 256) for u in (4, 8, 16)]
MODELS = [("egarch11", "fp64"), ("egarch11", "fp32"), ("egarch2t", "fp32"), ("egarch2t", "fp64"),
          ("egarch23", "fp32"), ("egarch23", "fp64")]


def _load():
    try:
        with open(TUNED) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned_waves(default: int = 2048) -> int:
    return int(_load().get("batch", {}).get("waves", default))


def tuned_shape(name, precision):
    """(block, unroll) recorded for a workload's random-walk step, or (0, 0)."""
    e = _load().get("mutate", {}).get(f"{name}/{precision}")
    return (int(e["block"]), int(e["unroll"])) if e else (0, 0)


def tuned_batch_shape():
    e = _load().get("batch")
    return (int(e["block"]), int(e["unroll"])) if e else (0, 0)


def apply(model, name, precision):
    """Sets the recorded shape on a model of a tuned workload (no-op else)."""
    b, u = tuned_shape(name, precision)
    if b or u:
        model.set_launch(b, u)


def time_mutate(model, pop, t, hl, reps=6):
    """Mean seconds of one random-walk step at date t."""
    na = torch.zeros(1, dtype=torch.int64, device=model.device)
    _lib.smc_mutate(model, pop, t, hl, seed=1, cycle=1, it=1, n_accept=na)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for it in range(reps):
        _lib.smc_mutate(model, pop, t, hl, seed=2, cycle=1, it=2 + it, n_accept=na)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def tune_mutate(name, precision):
    """{shape: seconds of a step at t = T plus one at t = T/4} for one workload."""
    import numpy as np

    import synthdata as SD

    w = SD.workload(name)
    prec = _lib.SMC_FP64 if precision == "fp64" else _lib.SMC_FP32
    m = _lib.Model.from_workload(w, precision=prec)
    th = SD.random_thetas(w, w.P, 3, spread=0.01)
    pop = _lib.Population(m, w.J, w.N, max_chunk=16)
    hl = torch.from_numpy(np.linalg.cholesky(np.cov(th[::16].T)) * 0.5).cuda()
    out = {}
    for b, u in SHAPES:
        m.set_launch(b, u)
        pop.theta.copy_(torch.from_numpy(th.T.copy()))
        pop.loglik.copy_(_lib.smc_loglik(m, pop.theta, w.T))
        out[(b, u)] = time_mutate(m, pop, w.T, hl) + time_mutate(m, pop, w.T // 4, hl)
    m.set_launch(0, 0)
    return out


def tune_batch(wave_counts=(1024, 2048, 4096)):
    """{(block, unroll, waves): seconds of one adaptive batch} of the batched
    workload."""
    import synthdata as SD

    specs = SD.batched_specs()
    models = [_lib.Model.from_workload(w, precision=_lib.SMC_FP32) for w in specs]
    pops = [_lib.Population(m, w.J, w.N, max_chunk=256) for m, w in zip(models, specs)]
    seeds = list(range(1, 33))
    _lib.smc_run_batch(models, pops, seeds, Lmax=2048, RmaxRec=64)
    out = {}
    for b, u in SHAPES:
        for mm in models:
            mm.set_launch(b, u)
        for wv in wave_counts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _lib.smc_run_batch(models, pops, seeds, waves=wv, Lmax=2048, RmaxRec=64)
            torch.cuda.synchronize()
            out[(b, u, wv)] = time.perf_counter() - t0
    return out


def main(out_path=TUNED, only=None):
    """Tunes every model and the batch, or with `only` (a list of
    (name, precision)) just those steps, keeping the file's other entries."""
    res = {"mutate": {}, "batch": {}} if only is None else _load()
    res.setdefault("mutate", {})
    for name, prec in (MODELS if only is None else only):
        t = tune_mutate(name, prec)
        (b, u) = min(t, key=t.get)
        res["mutate"][f"{name}/{prec}"] = {"block": b, "unroll": u,
                                           "seconds": {f"{k[0]}x{k[1]}": v for k, v in t.items()}}
        print(f"[tune] {name}/{prec}: best {b} x {u} ({t[(b, u)] * 1e6:.1f} us; "
              f"default {t[(64, 8)] * 1e6:.1f} us)", flush=True)
    if only is not None:
        with open(out_path, "w") as f:
            json.dump(res, f, indent=1)
        return res
    t = tune_batch()
    (b, u, wv) = min(t, key=t.get)
    res["batch"] = {"block": b, "unroll": u, "waves": wv,
                    "seconds": {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in t.items()}}
    print(f"[tune] batch: best {b} x {u}, {wv} waves ({t[(b, u, wv)]:.3f} s; "
          f"default {t[(64, 8, 2048)]:.3f} s)", flush=True)
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    import sys

    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    args = sys.argv[1:]
    only = None
    if "--only" in args:
        i = args.index("--only")
        only = [tuple(x.split("/")) for x in args[i + 1].split(",")]
        del args[i:i + 2]
    main(args[0] if args else TUNED, only)
