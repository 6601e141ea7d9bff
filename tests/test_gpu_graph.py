"""Device-driven adaptive runs (smc_run with graph=True): one captured step
graph -- a C-phase chunk, the S phase, Rbar M slots, the step's end -- is
launched until the run ends, every decision taken on the device.  The run
equals the host-driven one to the bit, also when the cached graph is launched
again after unrelated eager work.  The device-driven C phase alone
(smc_correct_async) equals smc_correct to the bit and can be captured."""
import numpy as np
import pytest
import torch

import paper_1304_4334_amd as S
import synthdata as SD
from tests.gpu_helpers import theta_np

pytestmark = pytest.mark.gpu

CASES = [
    # name, T, J, N, check_every, force_every, burn_in, max_chunk
    ("egarch11", 600, 4, 128, 1, 0, 0, 64),
    ("egarch2t", 500, 8, 64, 1, 0, 0, 256),
    ("egarch11", 700, 4, 128, 20, 0, 0, 64),  # chunks with no checked date
    ("egarch2t", 450, 4, 96, 7, 100, 130, 32),  # dates of interest and a burn-in date
]


def _same(a, b):
    assert a["L"] == b["L"] and a["L"] > 1
    for k in ("t_end", "R", "rss", "n_accept", "group_logwbar"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("log_ml", "nse", "evals", "mh_steps"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("prec", [S.SMC_FP64, S.SMC_FP32])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_device_driven_run_equals_host_driven(prec, case):
    name, T, J, N, ce, fe, bi, mc = case
    w = SD.workload(name, T=T, J=J, N=N)
    m = S.Model(w.kind, w.y[:T], K=w.K, shock=w.shock, precision=prec)
    kw = dict(check_every=ce, force_every=fe, burn_in=bi, Lmax=400, RmaxRec=64)
    p1 = S.Population(m, J, N, max_chunk=mc)
    r1 = S.smc_run(m, p1, seed=17, **kw)
    torch.cuda.synchronize()
    want = r1.summary()
    want_h = r1.hchol[:want["L"]].clone()
    p2 = S.Population(m, J, N, max_chunk=mc)
    r2 = S.smc_run(m, p2, seed=17, graph=True, **kw)
    torch.cuda.synchronize()
    _same(r2.summary(), want)
    assert torch.equal(r2.hchol[:want["L"]], want_h)
    assert np.array_equal(theta_np(p2), theta_np(p1))
    assert torch.equal(p2.loglik, p1.loglik) and torch.equal(p2.logw, p1.logw)
    # the cached step graph again, after unrelated eager work on the same
    # arrays: first with another key (the graph reads it from the device),
    # then with the first one
    r2.n_accept.fill_(-1)
    r4 = S.smc_run(m, p2, seed=18, graph=True, record=r2, **kw)
    p4 = S.Population(m, J, N, max_chunk=mc)
    r5 = S.smc_run(m, p4, seed=18, **kw)
    torch.cuda.synchronize()
    _same(r4.summary(), r5.summary())
    assert np.array_equal(theta_np(p2), theta_np(p4))
    for rep in range(2):
        p2.theta.add_(1.0)
        p2.logw.zero_()
        torch.cuda.synchronize()
        r3 = S.smc_run(m, p2, seed=17, graph=True, record=r2, **kw)
        torch.cuda.synchronize()
        _same(r3.summary(), want)
        assert torch.equal(r3.hchol[:want["L"]], want_h)
        assert np.array_equal(theta_np(p2), theta_np(p1)), rep


def test_device_driven_run_rejects_what_it_does_not_drive():
    w = SD.workload("egarch11", T=200, J=2, N=64)
    m = S.Model(w.kind, w.y[:200], K=w.K, shock=w.shock)
    p = S.Population(m, 2, 64, max_chunk=64)
    for kw in (dict(stop_rule=1), dict(kernel=S.SMC_KERNEL_INDEPENDENT), dict(RmaxRec=16)):
        with pytest.raises(S.SmcError):
            S.smc_run(m, p, seed=3, graph=True, Lmax=64, **kw)


C_CASES = [
    # name, T, J, N, check_every, max_chunk, rss_min
    ("egarch11", 400, 4, 128, 1, 16, 0.5),
    ("egarch2t", 300, 4, 96, 7, 32, 0.5),
    ("egarch11", 250, 2, 64, 20, 16, 0.5),  # chunks with no checked date
    ("linreg", 200, 4, 64, 1, 16, 0.0),     # the whole range, then its RSS
]


def _bits(x):
    """The tensor's bit patterns (prior draws far in the tails leave NaN in
    some particles' recursion state, and NaN equals nothing)."""
    return x.view(torch.int64 if x.element_size() == 8 else torch.int32)


def _pair(m, J, N, mc):
    p1 = S.Population(m, J, N, max_chunk=mc)
    p2 = S.Population(m, J, N, max_chunk=mc)
    for p in (p1, p2):
        S.smc_init_from_prior(m, p, seed=9)
    return p1, p2


@pytest.mark.parametrize("prec", [S.SMC_FP64, S.SMC_FP32])
@pytest.mark.parametrize("case", C_CASES, ids=lambda c: "-".join(map(str, c)))
def test_device_driven_c_phase_equals_smc_correct(prec, case):
    """smc_correct_async (every stopping decision on the device, outputs in
    device memory) gives smc_correct's end date, RSS, group weights and
    particles to the bit, over three cycles with S phases between them."""
    name, T, J, N, ce, mc, rss_min = case
    if name == "linreg" and prec == S.SMC_FP32:
        pytest.skip("the regression has no FP32 recursion")
    w = SD.workload(name, T=T)
    m = S.Model(w.kind, w.y[:T], X=None if w.X is None else w.X[:T], K=w.K, shock=w.shock,
                precision=prec)
    p1, p2 = _pair(m, J, N, mc)
    t = 0
    for cyc in range(3):
        t_h, rss_h, g_h = S.smc_correct(m, p1, t, T, check_every=ce, rss_min=rss_min)
        t_d, rss_d, g_d = S.smc_correct_async(m, p2, t, T, check_every=ce, rss_min=rss_min)
        torch.cuda.synchronize()
        assert int(t_d.item()) == t_h and t_h > t, cyc
        assert float(rss_d.item()) == rss_h, cyc
        assert torch.equal(_bits(g_d), _bits(g_h)), cyc
        for a, b in ((p1.logw, p2.logw), (p1.loglik, p2.loglik)):
            assert torch.equal(_bits(a), _bits(b)), cyc
        if m.S:
            assert torch.equal(_bits(p1.state), _bits(p2.state)), cyc
        if t_h >= T:
            break
        for p in (p1, p2):
            S.smc_resample(m, p, seed=4, cycle=cyc + 1)
        t = t_h


def test_device_driven_c_phase_in_a_graph():
    """The device-driven C phase captured in a graph: every replay (after the
    population's arrays are restored, with unrelated eager work between
    replays) gives the host-driven call's results."""
    w = SD.workload("egarch2t", T=400)
    m = S.Model(w.kind, w.y[:400], K=w.K, shock=w.shock, precision=S.SMC_FP32)
    p1, p2 = _pair(m, 4, 128, 32)
    t_h, rss_h, g_h = S.smc_correct(m, p1, 0, 400, check_every=1, rss_min=0.5)
    torch.cuda.synchronize()
    saved = [x.clone() for x in (p2.state, p2.logw, p2.loglik)]
    t_to = torch.zeros(1, dtype=torch.int64, device="cuda")
    rss = torch.zeros(1, dtype=torch.float64, device="cuda")
    glw = torch.zeros(4, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream's side, as torch requires
        S.smc_correct_async(m, p2, 0, 400, rss_min=0.5, group_logwbar=glw, t_to=t_to, rss=rss)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.smc_correct_async(m, p2, 0, 400, rss_min=0.5, group_logwbar=glw, t_to=t_to, rss=rss)
    for rep in range(3):
        for x, v in zip((p2.state, p2.logw, p2.loglik), saved):
            x.copy_(v)
        t_to.zero_()
        rss.zero_()
        p2.theta.add_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(t_to.item()) == t_h and float(rss.item()) == rss_h, rep
        assert torch.equal(_bits(glw), _bits(g_h)), rep
        for a, b in ((p1.logw, p2.logw), (p1.loglik, p2.loglik), (p1.state, p2.state)):
            assert torch.equal(_bits(a), _bits(b)), rep
