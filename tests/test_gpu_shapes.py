"""Launch shapes of the random-walk step (particles per block 64, 128 or 256;
observations per load batch 4, 8 or 16): every shape gives the default
shape's results to the bit - single steps, whole adaptive runs (the proposal
scale folded into the step, one wave factoring it for a multi-wave block)
and batches - for the six model / precision pairs that have tuned shapes."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from tests.gpu_helpers import theta_np

pytestmark = pytest.mark.gpu

SHAPES = [(b, u) for b in (64, 128, 256) for u in (4, 8, 16)]
PAIRS = [("egarch11", S.SMC_FP64), ("egarch11", S.SMC_FP32), ("egarch2t", S.SMC_FP32),
         ("egarch2t", S.SMC_FP64), ("egarch23", S.SMC_FP32), ("egarch23", S.SMC_FP64)]


@pytest.mark.parametrize("name,prec", PAIRS)
def test_every_shape_steps_to_the_same_bits(name, prec):
    w = SD.workload(name, T=517)
    m = S.Model(w.kind, w.y[:w.T], K=w.K, shock=w.shock, precision=prec, I=w.I)
    J, N = 3, 333  # ragged blocks for every shape
    th = SD.random_thetas(w, J * N, 5, spread=0.02)
    om = O.Model.from_workload(w)
    lp = torch.tensor([O.logprior(om, th[p]) for p in range(J * N)], dtype=torch.float64)
    hl = torch.from_numpy(np.linalg.cholesky(np.cov(th.T)) * 0.1).cuda()
    # t = 517 and 509: 64 and 63 whole groups of 8 observations (the FP32
    # sums are added to FP64 every two groups, so 63 leaves one group open)
    for t in (w.T, w.T - 8):
        out = {}
        for b, u in SHAPES:
            m.set_launch(b, u)
            g = S.Population(m, J, N)
            g.theta.copy_(torch.from_numpy(th.T.copy()))
            g.loglik.copy_(S.smc_loglik(m, g.theta, t))
            g.logprior.copy_(lp)
            acc = torch.zeros(J * N, dtype=torch.uint8, device="cuda")
            n = S.smc_mutate(m, g, t, hl, seed=3, cycle=2, it=1, accepted=acc)
            out[(b, u)] = (theta_np(g), g.loglik.cpu().numpy(), g.state.cpu().numpy(),
                           acc.cpu().numpy(), int(n.item()))
        m.set_launch(0, 0)
        ref = out[(64, 8)]
        assert 0 < ref[4] < J * N
        for k, v in out.items():
            for a, b_ in zip(v[:4], ref[:4]):
                assert np.array_equal(a, b_), (t, k)
            assert v[4] == ref[4], (t, k)


@pytest.mark.parametrize("name,prec", PAIRS)
def test_adaptive_run_in_any_shape_is_the_same_run(name, prec):
    w = SD.workload(name, T=300)
    m = S.Model(w.kind, w.y[:w.T], K=w.K, shock=w.shock, precision=prec, I=w.I)
    J, N = 4, 160
    res = {}
    for b, u in ((64, 8), (256, 16), (128, 4)):
        m.set_launch(b, u)
        g = S.Population(m, J, N, max_chunk=32)
        s = S.smc_run(m, g, seed=9, Lmax=300, RmaxRec=64).summary()
        res[(b, u)] = (s, theta_np(g))
    m.set_launch(0, 0)
    a, tha = res[(64, 8)]
    for k, (s, th) in res.items():
        assert np.array_equal(s["t_end"], a["t_end"]) and np.array_equal(s["R"], a["R"]), k
        assert np.array_equal(s["n_accept"], a["n_accept"]), k
        assert s["log_ml"] == a["log_ml"] and s["nse"] == a["nse"], k
        assert np.array_equal(th, tha), k


@pytest.mark.parametrize("shape", [(128, 16), (256, 4)])
def test_batch_in_any_shape_is_the_same_batch(shape):
    specs = [("egarch11", 400, 4, 64, 0), ("egarch2t", 250, 4, 96, 1), ("egarch11", 700, 2, 200, 2)]
    res = {}
    for sh in ((64, 8), shape):
        models, pops = [], []
        for name, T, J, N, off in specs:
            w = SD.workload(name, T=T, J=J, N=N, seed_offset=off)
            m = S.Model(w.kind, w.y[:T], K=w.K, shock=w.shock, precision=S.SMC_FP32)
            m.set_launch(*sh)
            models.append(m)
            pops.append(S.Population(m, J, N, max_chunk=64))
        recs = S.smc_run_batch(models, pops, [5, 6, 7], waves=7, Lmax=400, RmaxRec=64)
        res[sh] = ([r.summary() for r in recs], [theta_np(p) for p in pops])
    for (a, tha), (b, thb) in zip(zip(*res[(64, 8)]), zip(*res[shape])):
        assert np.array_equal(a["n_accept"], b["n_accept"])
        assert a["log_ml"] == b["log_ml"]
        assert np.array_equal(tha, thb)


def test_shape_arguments_are_checked():
    w = SD.workload("egarch34", T=50)
    m = S.Model.from_workload(w)
    with pytest.raises(S.SmcError):
        m.set_launch(256, 8)  # tuned shapes for egarch_23 alone among the mixtures
    m.set_launch(64, 8)  # the default is always allowed
    w = SD.workload("egarch11", T=50)
    m = S.Model.from_workload(w)
    with pytest.raises(S.SmcError):
        m.set_launch(96, 8)
    with pytest.raises(S.SmcError):
        m.set_launch(64, 5)
