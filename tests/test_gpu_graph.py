"""Device-driven adaptive runs (smc_run with graph=True): one captured step
graph -- a C-phase chunk, the S phase, Rbar M slots, the step's end -- is
launched until the run ends, every decision taken on the device.  The run
equals the host-driven one to the bit, also when the cached graph is launched
again after unrelated eager work."""
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
