"""The FP32 likelihood recursion against the FP64 oracle, result by result.

The recursion's per-observation terms are FP32 (added to FP64 totals every
sixteen observations); weights, log-sum-exp, moments, the marginal likelihood
and its NSE stay FP64.  Each test measures the error of one result and
prints it ("[fp32] ..." lines):
  - the log-likelihood at t = T of sampled particles at the workloads' full
    sizes (EGARCH(1,1) T = 5,000; EGARCH(2)-t T = 10,000; egarch_23
    T = 5,100), absolute and relative to |log p(y | theta)|;
  - the group log mean weights of a C phase over a fixed range (the terms
    the log-ML is built from, Section 4.2), absolute;
  - the log-ML of whole adaptive runs, FP32 on the GPU against the FP64
    oracle with the same seed, in units of the two runs' combined NSE (the
    runs part ways at the first decision an FP32 log-ratio flips, after
    which they are independent simulations of the same posterior).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from tests.gpu_helpers import gpu_model, ora_model, pop_to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["egarch11", "egarch2t", "egarch23"])
def test_fp32_loglik_error_at_full_length(name):
    w = SD.workload(name)
    gm, om = gpu_model(w, S.SMC_FP32), ora_model(w)
    P = 64
    th = SD.random_thetas(w, P, 41, spread=0.01)
    got = S.smc_loglik(gm, torch.from_numpy(th.T.copy()).cuda(), w.T).cpu().numpy()
    want = O.loglik_batch(om, th, w.T)[0]
    ok = np.isfinite(want)
    assert ok.sum() > P // 2
    ab = np.abs(got[ok] - want[ok])
    rel = ab / np.abs(want[ok])
    print(f"[fp32] loglik {name} T={w.T}: max abs {ab.max():.3e}, max rel {rel.max():.3e}, "
          f"median abs {np.median(ab):.3e} (|loglik| ~ {np.median(np.abs(want[ok])):.0f})")
    assert rel.max() < 1e-6
    assert ab.max() < 1e-6 * w.T


@pytest.mark.parametrize("name", ["egarch11", "egarch2t", "egarch23"])
def test_fp32_group_weights_error(name):
    w = SD.workload(name, T=400)
    gm, om = gpu_model(w, S.SMC_FP32), ora_model(w)
    J, N = 8, 128
    opop = O.Pop(om, J, N)
    opop.theta[:] = SD.random_thetas(w, J * N, 43, spread=0.02)
    g = pop_to_gpu(gm, opop)
    # the first 150 observations, then the next 250, each as one C phase
    errs = []
    t0 = 0
    for t1 in (150, 400):
        _, _, glw_g = S.smc_correct(gm, g, t0, t1, check_every=1, rss_min=0.0, want_rss=False)
        _, _, glw_o = O.correct(om, opop, t0, t1, check_every=1, rss_min=0.0)
        errs.append(np.abs(glw_g.cpu().numpy() - glw_o).max())
        t0 = t1
    print(f"[fp32] group log weights {name}: max abs error {max(errs):.3e} per cycle")
    assert max(errs) < 1e-3


@pytest.mark.parametrize("name,T,J,N,seed", [("egarch11", 600, 16, 128, 2),
                                             ("egarch2t", 500, 16, 128, 3)])
def test_fp32_adaptive_log_ml_within_nse_of_oracle(name, T, J, N, seed):
    w = SD.workload(name, T=T)
    gm, om = gpu_model(w, S.SMC_FP32), ora_model(w)
    rc, orec, _ = O.run(om, J, N, seed, Lmax=400, RmaxRec=64)
    assert rc == 0
    so = orec.summary()
    g = S.Population(gm, J, N, max_chunk=64)
    sg = S.smc_run(gm, g, seed=seed, Lmax=400, RmaxRec=64).summary()
    z = abs(sg["log_ml"] - so["log_ml"]) / math.hypot(sg["nse"], so["nse"])
    print(f"[fp32] log-ML {name} T={T} P={J * N}: GPU FP32 {sg['log_ml']:.4f} +- {sg['nse']:.4f}, "
          f"oracle FP64 {so['log_ml']:.4f} +- {so['nse']:.4f}, |diff|/NSE = {z:.2f}; "
          f"first cycles' ends equal: {int(np.argmin(np.append(sg['t_end'][:min(sg['L'], so['L'])] == so['t_end'][:min(sg['L'], so['L'])], False)))}")
    assert z < 3.0
