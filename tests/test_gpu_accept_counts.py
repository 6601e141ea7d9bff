"""Accepted-move counts of the Metropolis steps (Algorithm 1 step 2c; the
step-size rule of Section 3.3 reads them).  Each wave of a step stores its
count in the population's workspace and a later kernel adds them to the
caller's counter; without a workspace the step adds them atomically.  Either
way the counter gains exactly the number of set `accepted` flags, on every
call (a second call adds to the first), for the random-walk, independent and
Langevin kernels, with a population whose last wave is only partly filled."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from paper_1304_4334_amd import _lib
from tests.gpu_helpers import ora_model

pytestmark = pytest.mark.gpu

T = 200
J, N = 4, 300  # 1,200 particles: the last of 19 waves holds 48


def _population(name, prec, with_grad):
    w = SD.workload(name, T=T)
    m = S.Model(w.kind, w.y[:T], X=None if w.X is None else w.X[:T], K=w.K, shock=w.shock,
                precision=prec)
    pop = S.Population(m, J, N, max_chunk=32, with_grad=with_grad)
    th = SD.random_thetas(w, J * N, 7, spread=0.05)
    om = ora_model(w, T=T)
    pop.theta.copy_(torch.from_numpy(th.T.copy()))
    pop.logprior.copy_(torch.tensor([O.logprior(om, th[p]) for p in range(J * N)],
                                    dtype=torch.float64))
    pop.loglik.copy_(S.smc_loglik(m, pop.theta, T))
    if with_grad:
        S.smc_posterior_grad(m, pop, T)
    return m, pop, th


def _scale(th, kernel):
    cov = np.cov(th.T)
    chol = np.linalg.cholesky(cov)
    if kernel == S.SMC_KERNEL_INDEPENDENT:  # the factor, then the mean
        return torch.from_numpy(np.concatenate([chol.ravel(), th.mean(0)])).cuda()
    return torch.from_numpy((0.3 * chol).ravel().copy()).cuda()


KERNELS = [S.SMC_KERNEL_RW, S.SMC_KERNEL_INDEPENDENT, S.SMC_KERNEL_MALA]


@pytest.mark.parametrize("workspace", [True, False], ids=["workspace", "atomic"])
@pytest.mark.parametrize("kernel", KERNELS, ids=["rw", "indep", "mala"])
@pytest.mark.parametrize("name,prec", [("egarch2t", S.SMC_FP32), ("egarch11", S.SMC_FP64)])
def test_count_equals_accepted_flags(name, prec, kernel, workspace):
    if kernel == S.SMC_KERNEL_MALA and not workspace:
        pytest.skip("the Langevin step keeps its checkpoints in the workspace")
    m, pop, th = _population(name, prec, kernel == S.SMC_KERNEL_MALA)
    hl = _scale(th, kernel)
    c = pop.c
    if not workspace:
        c = _lib.Particles.from_buffer_copy(pop.c)
        c.ws = None
        c.ws_bytes = 0
    na = torch.zeros(1, dtype=torch.int64, device="cuda")
    total = 0
    for it in (1, 2):
        acc = torch.zeros(J * N, dtype=torch.uint8, device="cuda")
        st = _lib.lib().smc_mutate(m.h, C.byref(c), T, kernel, C.c_void_p(hl.data_ptr()),
                                   _lib.Rng(11, 0), 1, it, C.c_void_p(na.data_ptr()),
                                   C.c_void_p(acc.data_ptr()),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == S.SMC_OK, _lib.lib().smc_last_error().decode()
        torch.cuda.synchronize()
        n = int(acc.sum().item())
        total += n
        print(f"[counts] call {it}: {n} of {J * N} accepted")
        assert int(na.item()) == total, (it, int(na.item()), total)
    assert 0 < total < 2 * J * N
