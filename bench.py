#!/usr/bin/env python3
"""Throughput of the sequential posterior simulator on one MI355X.

A step is one whole adaptive run of the simulator (prior draw, C/S/M cycles
to T with the Section 3.3 rules, marginal likelihood) on a synthetic
workload resident in HBM.  The headline workload is the EGARCH model with two
volatility factors and Student-t(8) shocks, T = 10,000, 64 groups of 1,024
particles, FP32 likelihood recursion with FP64 weights, log-sum-exp and
moments.  `value` is particle x observation log-likelihood evaluations per
second over the K timed steps (C-phase and M-phase evaluations, divided by
wall time including every host decision).

The roofline object describes the dominant kernel (the Metropolis mutation
kernel): algorithmic VALU lane-operations per particle-observation (the
counts of the hot-path scope table, and the builder's own counts beside
them) times the evaluations of each launch, divided by the launch durations
measured with HIP events on the launch stream inside the timed region.

The cpu_baseline object times the oracle (plain FP64 C, OpenMP over
particles) on a bounded sample of the same work: its Metropolis step over
4,096 particles at t = T on every host core, with likelihood-throughput legs
at the EGARCH(1,1) and EGARCH(2)-t shapes on one core and on all of them.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("particle·obs log-lik evals/s; wall time to log-ML at NSE≤0.05 "
          "(MALA vs RW)")

# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock for unpacked FP32/FP64 VALU
# operations at 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
N_SIMD = 256 * 4
TIME_EVERY = 4  # timed runs put HIP events on every 4th Metropolis iteration

# Algorithmic VALU lane-operations per particle-observation of the recursion
# (FMA = 1; FP32 exp2/log2 = 4, quarter rate; FP64 exp/log1p = 17, the
# range reduction, degree-11 polynomial and scaling of a full-precision
# software exponential).
def mixture_ops(K, I, exp_cost, fp32):
    """Lane-operations per particle-observation of egarch_KI with an
    I-component normal mixture.  The recursion: FP64 (the form whose chain is
    one exp2 and one fma) 4 per factor plus 3 per extra factor for the
    cross-factor sums; FP32 (the eps form) 3 per factor plus one addition per
    extra factor; then z, eps = z E and the exponent sum's accumulation (3).
    Per component eps - mu_i and the quadratic (3), the shift by the maximum
    and the sum (about 2 each), the running maximum term and product (2); one
    exp2 for E and one per component."""
    rec = (3 * K + (K - 1) if fp32 else 4 * K + (3 * (K - 1) if K > 1 else 0)) + 3
    mix = 3 * I + 2 * (I - 1) + I + 2
    return rec + mix + (1 + I) * exp_cost


# The builder's counts of the kernels' algorithmic work (see above).
# FP32 (the eps form): z, eps, 3 per factor, K - 1 additions, the exponent
# sum's accumulation; the Gaussian term 1, or the Student-t factor 1, the
# product of four factors (3/4), the log2's accumulation (1/4) and a quarter
# of a log2 (one log2 per four observations).
OPS_PER_EVAL = {
    ("linreg", "fp64"): 4,
    ("egarch23", "fp64"): mixture_ops(2, 3, 17, False),
    ("egarch23", "fp32"): mixture_ops(2, 3, 4, True),
    ("egarch11", "fp64"): 7 + 17,
    ("egarch11", "fp32"): 1 + 1 + 3 + 1 + 1 + 4,
    ("egarch2t", "fp64"): 10 + 17 + 3 + 17,
    ("egarch2t", "fp32"): 1 + 1 + 6 + 1 + 1 + 1 + 0.75 + 0.25 + 4 + 1,
}

# Algorithmic VALU lane-slots per particle-observation from the hot-path
# scope table (a transcendental = 4 slots); None where it gives no figure.
OPS_SCOPE = {
    ("linreg", "fp64"): 4,
    ("egarch11", "fp64"): 29,
    ("egarch11", "fp32"): 14,
    ("egarch2t", "fp32"): 25,
}


SCOPE_NOTE = ("achieved counts the scope table's lane-slots per evaluation; the FP32 kernels "
              "need fewer (one log2 per four observations and the eps form of the factor update: "
              "ops_per_eval_builder), so frac may exceed 1; frac_builder_ops is the fraction "
              "of the VALU issue peak the kernel's own operations reach")


def ops_for(name, precision):
    """(count used for the roofline, its source, the builder's count)."""
    b = OPS_PER_EVAL[(name, precision)]
    s = OPS_SCOPE.get((name, precision))
    return (s, "scope table", b) if s is not None else (b, "builder", b)


DESCR = {
    "linreg": "conjugate Gaussian regression, k=3, T=200, J=4 x N=256",
    "egarch11": "EGARCH(1,1) Gaussian shocks, T=5000 synthetic returns, J=16 x N=1024",
    "egarch2t": "EGARCH 2 factors, Student-t(8) shocks, T=10000 synthetic returns, J=64 x N=1024",
    "egarch23": ("egarch_23: EGARCH 2 factors, 3-component normal-mixture shocks, T=5100 "
                 "synthetic returns, J=64 x N=1024"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mutate_traffic_pmc.md")
TRAFFIC_KEYS = {("egarch11", "fp64"): "k_mutate_rw egarch11 fp64 P=16384 t=5000 bytes",
                ("egarch2t", "fp32"): "k_mutate_rw egarch2t fp32 P=65536 t=10000 bytes",
                ("egarch23", "fp32"): "k_mutate_rw egarch23 fp32 P=65536 t=5100 bytes"}
# Sources whose text defines the mutation kernels the traffic was measured on.
TRAFFIC_SOURCES = ["paper_1304_4334_amd/csrc/model_kernels.h", "paper_1304_4334_amd/csrc/model.h",
                   "paper_1304_4334_amd/csrc/rng.h", "paper_1304_4334_amd/csrc/common.h",
                   "paper_1304_4334_amd/csrc/ops_egarch.hip",
                   "paper_1304_4334_amd/csrc/ops_mixture32.hip",
                   "paper_1304_4334_amd/csrc/ops_shapes32.hip",
                   "paper_1304_4334_amd/csrc/ops_shapes64.hip",
                   "paper_1304_4334_amd/csrc/ops_shapes_mix32.hip",
                   "paper_1304_4334_amd/csrc/chol.h", "paper_1304_4334_amd/csrc/launch.h"]


def measured_traffic(name, precision):
    """HBM bytes per mutation launch (at t = T) from the committed counter
    passes, or None when the kernel sources changed since they were taken."""
    key = TRAFFIC_KEYS.get((name, precision))
    if key is None or not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    try:
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (IndexError, ValueError):
        return None
    if rec.get("sources") != TRAFFIC_SOURCES or sources_sha256() != rec["sources_sha256"]:
        return None
    return rec.get(key)


def sources_sha256():
    """Hash of the mutation kernels' sources (the traffic record's key)."""
    import hashlib

    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def time_to_nse(name, precision, kernel, target=0.05, ladder=(5, 8, 13, 21, 34, 55),
                seeds=(1, 2, 3)):
    """Wall time to a log-ML with NSE <= target, as in the paper's Table 3:
    for each seed, whole adaptive runs climb the Fibonacci ladder of Rbar
    until one reaches the target; that run's seconds, NSE and precision per
    time 1/(NSE^2 s) are kept.  One untimed run first (kernel load, first
    launches).  Returns the per-seed results and their mean and sd."""
    import numpy as np
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD

    w = SD.workload(name)
    prec = S.SMC_FP64 if precision == "fp64" else S.SMC_FP32
    kern = S.SMC_KERNEL_MALA if kernel == "mala" else S.SMC_KERNEL_RW
    m = S.Model.from_workload(w, precision=prec)
    pop = S.Population(m, w.J, w.N, max_chunk=1024, with_grad=kern == S.SMC_KERNEL_MALA)
    S.smc_run(m, pop, seed=900, Rbar=ladder[0], kernel=kern,
              record=S.Record(m, w.J, Lmax=2048, RmaxRec=3 * ladder[0] + 1))
    torch.cuda.synchronize()
    per_seed = []
    for seed in seeds:
        tried = []
        hit = None
        for Rbar in ladder:
            rec = S.Record(m, w.J, Lmax=2048, RmaxRec=3 * Rbar + 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.smc_run(m, pop, seed=seed, Rbar=Rbar, kernel=kern, record=rec)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s = rec.summary()
            tried.append(dict(Rbar=Rbar, secs=el, nse=s["nse"], log_ml=s["log_ml"],
                              mh_steps=s["mh_steps"]))
            log(f"[bench] time-to-NSE {name}/{precision}/{kernel} seed {seed} Rbar={Rbar}: "
                f"{el:.3f} s, NSE {s['nse']:.4f}")
            if s["nse"] <= target:
                hit = dict(seed=seed, Rbar=Rbar, secs=el, nse=s["nse"], log_ml=s["log_ml"],
                           precision_per_time=1.0 / (s["nse"] ** 2 * el),
                           ladder_secs=sum(x["secs"] for x in tried))
                break
        per_seed.append(hit if hit else dict(seed=seed, Rbar=None, ladder=tried))
    ok = [x for x in per_seed if x.get("Rbar")]

    def ms(key):
        v = np.array([x[key] for x in ok], dtype=np.float64)
        return (float(v.mean()), float(v.std(ddof=1)) if len(v) > 1 else 0.0) if len(v) else (None, None)

    out = dict(kernel=kernel, precision=precision, batched=False, seeds=list(seeds),
               reached=len(ok), per_seed=per_seed)
    for key in ("secs", "nse", "precision_per_time", "Rbar"):
        out[key + "_mean"], out[key + "_sd"] = ms(key)
    return out


def time_to_nse_batched(name, precision, kernel, target=0.05, ladder=(5, 8, 13, 21, 34, 55),
                        seed_sets=((1, 2, 3), (4, 5, 6), (7, 8, 9))):
    """The same criterion for B independent runs advanced together in one
    batch (one persistent M-step launch per batch step): their J groups are
    pooled into one estimate of the marginal likelihood with B*J groups
    (eq ML_se over all of them, computed by smc_log_ml from the groups'
    summed log weights), and the ladder is climbed until its NSE <= target.
    The seconds are the whole batch call's."""
    import numpy as np
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD

    w = SD.workload(name)
    prec = S.SMC_FP64 if precision == "fp64" else S.SMC_FP32
    kern = S.SMC_KERNEL_MALA if kernel == "mala" else S.SMC_KERNEL_RW
    B = len(seed_sets[0])
    m = S.Model.from_workload(w, precision=prec)
    models = [m] * B
    pops = [S.Population(m, w.J, w.N, max_chunk=1024, with_grad=kern == S.SMC_KERNEL_MALA)
            for _ in range(B)]

    def batch(seeds, Rbar):
        recs = S.smc_run_batch(models, pops, list(seeds), Rbar=Rbar, kernel=kern, Lmax=2048,
                               RmaxRec=3 * Rbar + 1)
        tot = torch.cat([r.group_logwbar[:r.L].sum(0) for r in recs]).reshape(1, -1)
        out = S.smc_log_ml(tot).cpu().numpy()
        return recs, float(out[0]), float(out[1])

    batch([900 + i for i in range(B)], ladder[0])
    torch.cuda.synchronize()
    per_set = []
    for seeds in seed_sets:
        hit = None
        spent = 0.0
        for Rbar in ladder:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs, lml, nse = batch(seeds, Rbar)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            spent += el
            log(f"[bench] time-to-NSE batched {name}/{precision}/{kernel} seeds {seeds} "
                f"Rbar={Rbar}: {el:.3f} s, pooled NSE {nse:.4f}")
            if nse <= target:
                hit = dict(seeds=list(seeds), Rbar=Rbar, secs=el, nse=nse, log_ml=lml,
                           precision_per_time=1.0 / (nse ** 2 * el), ladder_secs=spent,
                           run_nse=[r.summary()["nse"] for r in recs])
                break
        per_set.append(hit if hit else dict(seeds=list(seeds), Rbar=None))
    ok = [x for x in per_set if x.get("Rbar")]

    def ms(key):
        v = np.array([x[key] for x in ok], dtype=np.float64)
        return (float(v.mean()), float(v.std(ddof=1)) if len(v) > 1 else 0.0) if len(v) else (None, None)

    out = dict(kernel=kernel, precision=precision, batched=True, runs_per_batch=B,
               reached=len(ok), per_seed=per_set)
    for key in ("secs", "nse", "precision_per_time", "Rbar"):
        out[key + "_mean"], out[key + "_sd"] = ms(key)
    return out


def run_gpu(name, precision, steps, warmup):
    import numpy as np
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD

    from paper_1304_4334_amd import tune

    w = SD.workload(name)
    prec = S.SMC_FP64 if precision == "fp64" else S.SMC_FP32
    m = S.Model.from_workload(w, precision=prec)
    tune.apply(m, name, precision)
    pop = S.Population(m, w.J, w.N, max_chunk=1024)
    # HIP events on every 4th Metropolis iteration (all cycles are sampled
    # alike); the untimed launches' entries are -1
    rec = S.Record(m, w.J, Lmax=2048, RmaxRec=64, time_mutate=True, time_every=TIME_EVERY)
    force = 20 if name == "linreg" else 0

    def one(seed):
        S.smc_run(m, pop, seed=seed, check_every=1, force_every=force, record=rec)

    for i in range(warmup):
        one(10_000 + i)
        log(f"[bench] {name}/{precision} warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    evals = 0
    mut_ms = 0.0
    mut_evals = 0
    n_launch = 0
    log_mls, nses, cycles, msteps = [], [], [], []
    t0 = time.perf_counter()
    for k in range(steps):
        one(1 + k)
        s = rec.summary()
        evals += s["evals"]
        L = s["L"]
        for l in range(L):
            Rl = int(s["R"][l])
            ms_l = rec.mutate_ms[l, :Rl].astype(np.float64)
            timed = ms_l >= 0
            mut_ms += float(ms_l[timed].sum())
            mut_evals += int(timed.sum()) * w.P * int(s["t_end"][l])
            n_launch += int(timed.sum())
        log_mls.append(s["log_ml"])
        nses.append(s["nse"])
        cycles.append(L)
        msteps.append(s["mh_steps"])
        log(f"[bench] {name}/{precision} step {k + 1}/{steps}: {L} cycles, "
            f"{s['mh_steps']} M steps, log ML {s['log_ml']:.3f} +- {s['nse']:.3f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    ops, src, ops_b = ops_for(name, precision)
    rate = mut_evals / (mut_ms * 1e-3)
    achieved = ops * rate / 1e12
    occupied = min(1.0, math.ceil(w.P / 64) / N_SIMD)
    return dict(
        w=w, value=evals / secs, ms_per_step=1e3 * secs / steps, evals_per_step=evals / steps,
        log_ml=float(np.mean(log_mls)), nse=float(np.mean(nses)), cycles=float(np.mean(cycles)),
        mh_steps=float(np.mean(msteps)), mutate_avg_ms=mut_ms / max(n_launch, 1),
        mutate_launches=n_launch, mutate_evals_per_s=rate,
        mutate_avg_t=mut_evals / max(n_launch, 1) / w.P,
        roofline=dict(bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS,
                      unit="T VALU lane-ops/s", frac=achieved / VALU_PEAK_TOPS,
                      traffic=measured_traffic(name, precision),
                      traffic_unit="bytes per launch at t=T",
                      kernel="k_mutate_rw", ops_per_eval=ops, ops_source=src,
                      ops_per_eval_builder=ops_b,
                      frac_builder_ops=ops_b * rate / 1e12 / VALU_PEAK_TOPS,
                      simd_occupancy=occupied,
                      frac_of_occupied=achieved / (VALU_PEAK_TOPS * occupied),
                      launch_shape=dict(zip(("block", "unroll"),
                                            getattr(m, "launch", (0, 0)))),
                      note=SCOPE_NOTE if src == "scope table" else None),
        secs=secs)


def run_batched(steps):
    """The batched workload: 32 independent adaptive runs (EGARCH(1,1)-N and
    EGARCH(2)-t alternating, T in [1000, 20000], J*N in 4096..65536), FP32
    recursion, one persistent M-step launch per batch step.  The roofline
    adds, over the timed persistent launches, each run's evaluations times
    its model's algorithmic count, over the launches' summed durations."""
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD
    from paper_1304_4334_amd import tune

    specs = SD.batched_specs()
    models = [S.Model.from_workload(w, precision=S.SMC_FP32) for w in specs]
    bshape = tune.tuned_batch_shape()
    for mm in models:
        mm.set_launch(*bshape)
    pops = [S.Population(m, w.J, w.N, max_chunk=256) for m, w in zip(models, specs)]
    waves = tune.tuned_waves()
    S.smc_run_batch(models, pops, list(range(100, 132)), waves=waves, Lmax=2048, RmaxRec=64)
    torch.cuda.synchronize()
    evals = 0
    ms_sum, lane_ops, lane_ops_b, m_evals, launches = 0.0, 0.0, 0.0, 0, 0
    o1, _, b1 = ops_for("egarch11", "fp32")
    o2, _, b2 = ops_for("egarch2t", "fp32")
    t0 = time.perf_counter()
    for k in range(steps):
        recs, tim = S.smc_run_batch(models, pops, [1 + 32 * k + i for i in range(32)],
                                    waves=waves, Lmax=2048, RmaxRec=64, timing=8192)
        evals += sum(r.c.evals for r in recs)
        ms_sum += sum(tim["ms"])
        launches += len(tim["ms"])
        for e1, e2 in tim["evals"]:
            lane_ops += o1 * e1 + o2 * e2
            lane_ops_b += b1 * e1 + b2 * e2
            m_evals += e1 + e2
        log(f"[bench] batched step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    achieved = lane_ops / (ms_sum * 1e-3) / 1e12
    return dict(value=evals / secs, ms_per_step=1e3 * secs / steps, runs=len(specs),
                total_particles=sum(w.P for w in specs), waves=waves,
                launch_shape={"block": bshape[0], "unroll": bshape[1]},
                evals_per_step=evals / steps,
                mutate_launches_per_step=launches / steps,
                mutate_ms_per_step=ms_sum / steps,
                mutate_evals_per_s=m_evals / (ms_sum * 1e-3),
                roofline=dict(bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS,
                              unit="T VALU lane-ops/s", frac=achieved / VALU_PEAK_TOPS,
                              traffic=None, kernel="k_batch_mutate",
                              ops_per_eval={"egarch11_fp32": o1, "egarch2t_fp32": o2},
                              ops_source="scope table",
                              ops_per_eval_builder={"egarch11_fp32": b1, "egarch2t_fp32": b2},
                              frac_builder_ops=lane_ops_b / (ms_sum * 1e-3) / 1e12
                              / VALU_PEAK_TOPS,
                              note=SCOPE_NOTE))


def run_device_driven(name, precision, steps, warmup):
    """Whole adaptive runs driven on the device (smc_run with graph=True: one
    captured step graph launched until the run ends) beside the same runs
    driven from the host, with the same seeds: mean ms per run each, and
    whether the two agree to the bit (log ML, cycles)."""
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD
    from paper_1304_4334_amd import tune

    w = SD.workload(name)
    prec = S.SMC_FP64 if precision == "fp64" else S.SMC_FP32
    m = S.Model.from_workload(w, precision=prec)
    tune.apply(m, name, precision)
    pop = S.Population(m, w.J, w.N, max_chunk=1024)
    out = {}
    mls = {}
    for mode, graph in (("host_driven", False), ("device_driven", True)):
        rec = S.Record(m, w.J, Lmax=2048, RmaxRec=64)
        for i in range(warmup):
            S.smc_run(m, pop, seed=10_000 + i, record=rec, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = []
        for k in range(steps):
            S.smc_run(m, pop, seed=1 + k, record=rec, graph=graph)
            s = rec.summary()
            got.append((s["log_ml"], s["L"], s["mh_steps"]))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        mls[mode] = got
        out[mode] = dict(ms_per_run=1e3 * secs / steps)
        log(f"[bench] {name}/{precision} {mode}: {1e3 * secs / steps:.2f} ms per run")
    out["same_results"] = mls["host_driven"] == mls["device_driven"]
    out["device_over_host_time"] = (out["device_driven"]["ms_per_run"]
                                    / out["host_driven"]["ms_per_run"])
    return out


def run_variants(name, precision, steps):
    """Whole adaptive runs of one workload under each option of the method
    beside the default (residual resampling, deterministic R, RW steps):
    the other resamplers, the RNE stop rule, the independent sampler, the
    moment reports and log score of every cycle, the fixed-design replay and
    the two-step hybrid.  Each entry: mean ms per run over `steps` runs after
    one warm-up, particle-observation evaluations per second, log ML and NSE."""
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD

    w = SD.workload(name)
    prec = S.SMC_FP64 if precision == "fp64" else S.SMC_FP32
    m = S.Model.from_workload(w, precision=prec)
    pop = S.Population(m, w.J, w.N, max_chunk=1024)
    burn = w.T // 2
    variants = {
        "resample_multinomial": dict(scheme=S.SMC_RESAMPLE_MULTINOMIAL),
        "resample_stratified": dict(scheme=S.SMC_RESAMPLE_STRATIFIED),
        "resample_systematic": dict(scheme=S.SMC_RESAMPLE_SYSTEMATIC),
        "rne_stop_E1_0.35": dict(stop_rule=1, E1=0.35, test_fn=S.SMC_TEST_MODEL),
        "independent_sampler": dict(kernel=S.SMC_KERNEL_INDEPENDENT),
        "reports_and_log_score": dict(test_fn=S.SMC_TEST_MODEL, burn_in=burn, report=True),
    }
    out = {}
    for key, kw in variants.items():
        kw = dict(kw)
        rep = kw.pop("report", False)
        tf = kw.get("test_fn", S.SMC_TEST_PARAMS)
        rec = S.Record(m, w.J, Lmax=2048, RmaxRec=128, test_fn=tf if rep else None)
        S.smc_run(m, pop, seed=20_000, record=rec, **kw)
        torch.cuda.synchronize()
        evals, lm, nse = 0, 0.0, 0.0
        t0 = time.perf_counter()
        for k in range(steps):
            S.smc_run(m, pop, seed=1 + k, record=rec, **kw)
            s = rec.summary()
            evals += s["evals"]
            lm += s["log_ml"] / steps
            nse += s["nse"] / steps
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[key] = dict(ms_per_run=1e3 * secs / steps, value=evals / secs, log_ml=lm, nse=nse)
        if rep:
            out[key]["log_score"] = s["log_score"][:2]
        log(f"[bench] {name}/{precision} {key}: {1e3 * secs / steps:.1f} ms per run")
    # The fixed-design replay of an adaptive run's design, with a new key.
    rec = S.Record(m, w.J, Lmax=2048, RmaxRec=128)
    S.smc_run(m, pop, seed=30_000, record=rec)
    S.smc_run(m, pop, seed=30_001, record=rec, replay=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for k in range(steps):
        S.smc_run(m, pop, seed=30_002 + k, record=rec, replay=True)
        evals += rec.summary()["evals"]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    s = rec.summary()
    out["replay"] = dict(ms_per_run=1e3 * secs / steps, value=evals / secs, log_ml=s["log_ml"],
                         nse=s["nse"])
    log(f"[bench] {name}/{precision} replay: {1e3 * secs / steps:.1f} ms per run")
    # Algorithm 3: adaptive run, then its design replayed with a second key.
    t0 = time.perf_counter()
    r1, r2, hs = S.smc_run_hybrid(m, pop, seed=40_000, seed2=40_001, test_fn=S.SMC_TEST_MODEL,
                                  burn_in=burn)
    torch.cuda.synchronize()
    rep = S.hybrid_report(r1, r2, hs)
    out["hybrid"] = dict(ms_total=1e3 * (time.perf_counter() - t0),
                         step_ms=[1e3 * float(x) for x in hs], z_log_ml=rep["z_log_ml"],
                         z_log_score=rep["z_log_score"])
    log(f"[bench] {name}/{precision} hybrid: {out['hybrid']['ms_total']:.1f} ms")
    return out


def _host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = sorted(os.sched_getaffinity(0))
    except AttributeError:
        aff = list(range(os.cpu_count() or 1))
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity_cpus=len(aff),
                affinity=f"{aff[0]}-{aff[-1]}" if aff else "")


def _oracle_pop(O, SD, w, om, P, seed):
    pop = O.Pop(om, 2, P // 2)
    pop.theta[:] = SD.random_thetas(w, P, seed, spread=0.01)
    for p in range(P):
        pop.logprior[p] = O.logprior(om, pop.theta[p])
    return pop


def cpu_baseline(name, seconds, legs=True):
    """The oracle (FP64 C, OpenMP over particles, the host's cores) on a
    bounded sample of the workload: its random-walk Metropolis step over
    4,096 particles at t = T, repeated for about `seconds`; with `legs`, the
    likelihood throughput at the EGARCH(1,1) and EGARCH(2)-t shapes on one
    thread and on every allowed thread."""
    import numpy as np

    import oracle as O
    import synthdata as SD

    info = _host_info()
    n_all = max(1, info["affinity_cpus"])
    O.set_num_threads(n_all)
    w = SD.workload(name)
    om = O.Model.from_workload(w)
    Ps = 4096
    pop = _oracle_pop(O, SD, w, om, Ps, 3)
    pop.loglik[:] = O.loglik_batch(om, pop.theta, w.T)[0]
    hl = np.linalg.cholesky(np.cov(pop.theta.T)) * 0.5
    iters = 0
    t0 = time.perf_counter()
    while True:
        O.mutate(om, pop, w.T, hl, seed=5, cycle=1, it=iters + 1)
        iters += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rate = iters * Ps * w.T / el
    out = dict(value=rate, unit="particle·obs/s", cores=O.num_threads(), kind="oracle",
               sample=(f"oracle RW Metropolis step (FP64) on the {name} workload over {Ps} "
                       f"particles at t=T={w.T}, {iters} iterations in {el:.1f} s on "
                       f"{O.num_threads()} threads"), host=info)
    log(f"[bench] cpu baseline {name}: {rate:.3e} particle-obs/s on {O.num_threads()} threads")
    if legs:
        out["loglik_legs"] = {}
        for lname in ("egarch11", "egarch2t"):
            lw = SD.workload(lname)
            lom = O.Model.from_workload(lw)
            th = SD.random_thetas(lw, 4096, 7, spread=0.01)
            for nthr, P in ((1, 256), (n_all, 4096)):
                O.set_num_threads(nthr)
                t0 = time.perf_counter()
                O.loglik_batch(lom, th[:P], lw.T)
                el = time.perf_counter() - t0
                key = f"{lname}_{'1thread' if nthr == 1 else 'all'}"
                out["loglik_legs"][key] = dict(value=P * lw.T / el, particles=P, T=lw.T,
                                               threads=nthr, secs=el)
                log(f"[bench] oracle loglik {key}: {P * lw.T / el:.3e} particle-obs/s")
        O.set_num_threads(n_all)
    return out


def kernel_probe():
    """A short fixed sequence for hardware-counter passes: a 256 MiB device
    copy (calibration of the byte counters), then one whole adaptive run of
    each roofline workload (EGARCH(1,1) FP64 16,384 particles; EGARCH(2)-t
    FP32 and egarch_23 FP32, 65,536 particles), in the bench's launch shapes.  The last cycle of each run
    ends at t = T; its M steps are the last `R_last` mutation dispatches of
    the run, whose counters give the traffic per launch at t = T."""
    import torch

    import paper_1304_4334_amd as S
    import synthdata as SD
    from paper_1304_4334_amd import tune

    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("[probe] copies done")
    runs = []
    for name, prec in (("egarch11", S.SMC_FP64), ("egarch2t", S.SMC_FP32),
                       ("egarch23", S.SMC_FP32)):
        w = SD.workload(name)
        m = S.Model.from_workload(w, precision=prec)
        tune.apply(m, name, "fp64" if prec == S.SMC_FP64 else "fp32")  # the bench's shape
        pop = S.Population(m, w.J, w.N, max_chunk=1024)
        rec = S.Record(m, w.J, Lmax=2048, RmaxRec=64)
        S.smc_run(m, pop, seed=1, record=rec)
        torch.cuda.synchronize()
        s = rec.summary()
        runs.append(dict(workload=name, precision="fp64" if prec == S.SMC_FP64 else "fp32",
                         P=w.P, T=w.T, mutate_launches=int(s["mh_steps"]),
                         R_last=int(s["R"][-1]), t_last=int(s["t_end"][-1])))
        log(f"[probe] {name} done")
    print(json.dumps({"probe": "done", "copy_bytes": 2 * a.numel() * 4, "runs": runs,
                      "sources_sha256": sources_sha256()}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="egarch2t", choices=sorted(DESCR))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="recursion precision (default: fp32 for egarch2t, else fp64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--kernel-probe", action="store_true",
                    help="run only the short fixed sequence used for counter passes")
    ap.add_argument("--batch-probe", action="store_true",
                    help="run only one adaptive batch of the batched workload (for profiles)")
    ap.add_argument("--no-companions", action="store_true",
                    help="skip the companion workloads, the batch and the time-to-NSE comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path (a run would shard by whole groups, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        sys.exit("--steps must be >= 1")
    if args.kernel_probe:
        kernel_probe()
        return
    if args.batch_probe:
        print(json.dumps(run_batched(1)), flush=True)
        return
    precision = args.precision or ("fp32" if args.workload == "egarch2t" else "fp64")

    main_run = run_gpu(args.workload, precision, args.steps, args.warmup)
    comp = {}
    tnse = batched = variants = driven = None
    if not args.no_companions and args.workload == "egarch2t":
        driven = {f"{n}_{p}": run_device_driven(n, p, args.steps, args.warmup)
                  for n, p in (("egarch2t", "fp32"), ("egarch11", "fp64"))}
        for prec in ("fp64", "fp32"):
            comp[f"egarch11_{prec}"] = run_gpu("egarch11", prec, args.steps, args.warmup)
        for prec in ("fp32", "fp64"):
            comp[f"egarch23_{prec}"] = run_gpu("egarch23", prec, 2, 1)
        batched = run_batched(2)
        tnse = [time_to_nse("egarch2t", "fp64", "rw"), time_to_nse("egarch2t", "fp32", "rw"),
                time_to_nse("egarch2t", "fp32", "mala"),
                time_to_nse_batched("egarch2t", "fp32", "mala"),
                time_to_nse_batched("egarch2t", "fp32", "rw")]
        variants = run_variants("egarch11", "fp64", 2)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload, args.cpu_seconds)

    w = main_run["w"]
    out = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "particle·obs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESCR[args.workload]}, RW-Metropolis, "
                               f"adaptive C/S/M (D1=0.5, D2=0.2, Rbar=7, kappa=3), residual "
                               f"resampling, {precision.upper()} likelihood recursion, FP64 "
                               "weights, log-sum-exp, covariance and Cholesky",
                   "J": w.J, "N": w.N, "T": w.T, "precision": precision,
                   "parallelism": "single GPU"},
        "roofline": main_run["roofline"],
        "cpu_baseline": cpu,
        "run": {"log_ml": main_run["log_ml"], "nse": main_run["nse"],
                "cycles": main_run["cycles"], "mh_steps": main_run["mh_steps"],
                "evals_per_step": main_run["evals_per_step"],
                "mutate_avg_ms": main_run["mutate_avg_ms"],
                "mutate_avg_t": main_run["mutate_avg_t"],
                "mutate_launches": main_run["mutate_launches"],
                "mutate_evals_per_s": main_run["mutate_evals_per_s"]},
    }
    for key, r in comp.items():
        name, prec = key.split("_")
        out[key] = {"workload": f"{name}: {DESCR[name]}, RW, {prec.upper()} recursion, FP64 weights",
                    "value": r["value"], "ms_per_step": r["ms_per_step"], "log_ml": r["log_ml"],
                    "nse": r["nse"], "cycles": r["cycles"], "mh_steps": r["mh_steps"],
                    "mutate_avg_ms": r["mutate_avg_ms"], "mutate_avg_t": r["mutate_avg_t"],
                    "mutate_evals_per_s": r["mutate_evals_per_s"], "roofline": r["roofline"]}
    if batched is not None:
        out["batched"] = dict(batched, workload="32 independent adaptive runs: EGARCH(1,1)-N / "
                              "EGARCH(2)-t alternating, T in [1000, 20000], J=16, J*N in "
                              "4096..65536, FP32 recursion, RW")
    if tnse is not None:
        out["time_to_nse_0.05"] = {
            "workload": "egarch2t: " + DESCR["egarch2t"] + ", adaptive, Fibonacci Rbar ladder, "
                        "3 seeds (batched: 3 sets of 3 runs in one batch, groups pooled), after "
                        "one untimed run",
            "runs": tnse}
    if driven is not None:
        out["device_driven_runs"] = dict(
            driven, workload="whole adaptive runs driven on the device from one captured step "
                             "graph, beside the host-driven runs with the same seeds")
    if variants is not None:
        out["variants"] = dict(variants, workload=f"egarch11: {DESCR['egarch11']}, FP64 "
                               "recursion; defaults otherwise")
    if cpu is not None:
        out["gpu_over_cpu"] = main_run["value"] / cpu["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
