"""Batched runs (many independent simulators advanced together with one
persistent M-step launch): each run equals the same run on its own, and a
replayed batch captured in a graph reproduces the eager replay on every
graph replay."""
import numpy as np
import pytest
import torch

import paper_1304_4334_amd as S
import synthdata as SD
from tests.gpu_helpers import theta_np

pytestmark = pytest.mark.gpu


def _runs(prec, specs, with_grad=False):
    out = []
    for name, T, J, N, seed_off in specs:
        w = SD.workload(name, T=T, J=J, N=N, seed_offset=seed_off)
        m = S.Model(w.kind, w.y[:T], K=w.K, shock=w.shock, precision=prec)
        out.append((w, m, S.Population(m, J, N, max_chunk=64, with_grad=with_grad)))
    return out


SPECS = [("egarch11", 400, 4, 64, 0), ("egarch2t", 250, 4, 96, 1), ("egarch11", 700, 2, 200, 2),
         ("egarch2t", 333, 8, 32, 3)]


@pytest.mark.parametrize("prec", [S.SMC_FP64, S.SMC_FP32])
@pytest.mark.parametrize("waves", [0, 3])
def test_batch_equals_single_runs(prec, waves):
    runs = _runs(prec, SPECS)
    models = [m for _, m, _ in runs]
    pops = [p for _, _, p in runs]
    seeds = [11, 12, 13, 14]
    recs = S.smc_run_batch(models, pops, seeds, waves=waves, Lmax=400, RmaxRec=64)
    torch.cuda.synchronize()
    for i, (w, m, _) in enumerate(runs):
        p1 = S.Population(m, w.J, w.N, max_chunk=64)
        r1 = S.smc_run(m, p1, seed=seeds[i], Lmax=400, RmaxRec=64)
        a, b = recs[i].summary(), r1.summary()
        assert a["L"] == b["L"] and a["L"] > 1
        assert np.array_equal(a["t_end"], b["t_end"]) and np.array_equal(a["R"], b["R"])
        assert np.array_equal(a["n_accept"], b["n_accept"])
        assert np.array_equal(a["group_logwbar"], b["group_logwbar"])
        assert a["log_ml"] == b["log_ml"] and a["nse"] == b["nse"]
        assert a["evals"] == b["evals"] and a["mh_steps"] == b["mh_steps"]
        assert np.array_equal(theta_np(pops[i]), theta_np(p1))


def test_batch_replay_in_a_graph():
    runs = _runs(S.SMC_FP64, SPECS[:3])
    models = [m for _, m, _ in runs]
    pops = [p for _, _, p in runs]
    seeds = [5, 6, 7]
    design = S.smc_run_batch(models, pops, seeds, Lmax=400, RmaxRec=64)
    torch.cuda.synchronize()
    # eager replay with new seeds (step 2 of Algorithm 3)
    new = [21, 22, 23]
    eager = S.smc_run_batch(models, pops, new, records=design, replay=True)
    torch.cuda.synchronize()
    want_ml = [r.log_ml.clone() for r in eager]
    want_th = [p.theta.clone() for p in pops]
    nb = S._lib.lib().smc_batch_ws_bytes(3)
    bws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream's side, as torch requires
        S.smc_run_batch(models, pops, new, records=design, replay=True, bws=bws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.smc_run_batch(models, pops, new, records=design, replay=True, bws=bws)
    for rep in range(3):
        for p in pops:  # unrelated eager work between replays
            p.theta.add_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(3):
            assert torch.equal(design[i].log_ml, want_ml[i]), rep
            assert torch.equal(pops[i].theta, want_th[i]), rep


def test_batch_timing_accounts_for_every_m_step():
    """The timed persistent launches carry every M-step evaluation of the
    batch once: their evaluation counts add up to sum_l R_l P t_l over the
    runs, split by model family."""
    runs = _runs(S.SMC_FP32, SPECS)
    models = [m for _, m, _ in runs]
    pops = [p for _, _, p in runs]
    recs, tim = S.smc_run_batch(models, pops, [31, 32, 33, 34], Lmax=400, RmaxRec=64,
                                timing=4096)
    assert len(tim["ms"]) > 10 and all(ms > 0 for ms in tim["ms"])
    want = [0, 0]
    for (w, m, p), r in zip(runs, recs):
        s = r.summary()
        want[0 if w.K == 1 else 1] += sum(int(s["R"][l]) * w.J * w.N * int(s["t_end"][l])
                                          for l in range(s["L"]))
    got = np.array(tim["evals"]).sum(axis=0).tolist()
    assert got == want


@pytest.mark.parametrize("prec", [S.SMC_FP64, S.SMC_FP32])
def test_langevin_batch_equals_single_runs(prec):
    """Langevin (MALA) runs in one batch: each run's decisions, weights,
    estimates, particles and gradients equal those of the same run on its
    own, to the bit."""
    runs = _runs(prec, SPECS, with_grad=True)
    models = [m for _, m, _ in runs]
    pops = [p for _, _, p in runs]
    seeds = [41, 42, 43, 44]
    recs = S.smc_run_batch(models, pops, seeds, Lmax=400, RmaxRec=64, kernel=S.SMC_KERNEL_MALA)
    torch.cuda.synchronize()
    for i, (w, m, _) in enumerate(runs):
        p1 = S.Population(m, w.J, w.N, max_chunk=64, with_grad=True)
        r1 = S.smc_run(m, p1, seed=seeds[i], Lmax=400, RmaxRec=64, kernel=S.SMC_KERNEL_MALA)
        a, b = recs[i].summary(), r1.summary()
        assert a["L"] == b["L"] and a["L"] > 1
        assert np.array_equal(a["t_end"], b["t_end"]) and np.array_equal(a["R"], b["R"])
        assert np.array_equal(a["n_accept"], b["n_accept"])
        assert np.array_equal(a["group_logwbar"], b["group_logwbar"])
        assert a["log_ml"] == b["log_ml"] and a["nse"] == b["nse"]
        assert np.array_equal(theta_np(pops[i]), theta_np(p1))
        assert torch.equal(pops[i].grad, p1.grad)
