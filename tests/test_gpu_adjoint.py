"""GPU parity of the adjoint kernel, the posterior gradient and the Langevin
(MALA) M step against the oracle's forward-mode gradients and its MALA step,
plus finite differences of the GPU's own FP64 likelihood.

Tolerances: FP64 gradients 1e-8 relative to the gradient's norm; FP32
gradients 3e-3 relative to the norm (a sum over t observations in FP32).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from oracle import closed_form as CF
from paper_1304_4334_amd import autograd as SA
from tests.gpu_helpers import accept_audit, gpu_model, ora_model, pop_to_gpu, theta_np

pytestmark = pytest.mark.gpu

CASES = [("linreg", S.SMC_FP64), ("egarch11", S.SMC_FP64), ("egarch11", S.SMC_FP32),
         ("egarch2t", S.SMC_FP64), ("egarch2t", S.SMC_FP32), ("egarch23", S.SMC_FP64),
         ("egarch23", S.SMC_FP32), ("egarch12", S.SMC_FP64), ("egarch44", S.SMC_FP64)]


def _gtol(prec):
    return 1e-8 if prec == S.SMC_FP64 else 3e-3


def _grad_close(got, want, prec):
    nrm = np.linalg.norm(want, axis=-1, keepdims=True)
    ok = np.abs(got - want) <= _gtol(prec) * (np.abs(want) + nrm)
    if not np.all(ok):
        i = np.argwhere(~ok)[0]
        print("worst", i, got[tuple(i)], want[tuple(i)])
    return bool(np.all(ok))


@pytest.mark.parametrize("name,prec", CASES)
@pytest.mark.parametrize("t", [1, 31, 32, 33, 64, 65, 333])
def test_loglik_backward_matches_oracle_gradient(name, prec, t):
    w = SD.workload(name, T=333)
    gm, om = gpu_model(w, prec), ora_model(w)
    P = 70
    th = SD.random_thetas(w, P, 17, spread=0.05)
    dl = np.random.default_rng(t).uniform(0.5, 2.0, P)
    got = S.smc_loglik_backward(gm, torch.from_numpy(th.T.copy()).cuda(), t,
                                torch.from_numpy(dl).cuda()).cpu().numpy().T
    want = np.array([dl[p] * O.loglik_grad(om, th[p], t)[1] for p in range(P)])
    assert _grad_close(got, want, prec)


@pytest.mark.parametrize("name", ["egarch11", "egarch2t", "linreg", "egarch23"])
def test_gpu_gradient_matches_finite_differences(name):
    """Central differences (h = 1e-5) of the GPU's own FP64 log-likelihood."""
    w = SD.workload(name, T=500)
    gm = gpu_model(w)
    P = 8
    th = SD.random_thetas(w, P, 3, spread=0.05)
    d = th.shape[1]
    g = S.smc_loglik_backward(gm, torch.from_numpy(th.T.copy()).cuda(), w.T,
                              torch.ones(P, dtype=torch.float64, device="cuda")).cpu().numpy().T
    h = 1e-5
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        up = S.smc_loglik(gm, torch.from_numpy((th + e).T.copy()).cuda(), w.T).cpu().numpy()
        dn = S.smc_loglik(gm, torch.from_numpy((th - e).T.copy()).cuda(), w.T).cpu().numpy()
        fd = (up - dn) / (2 * h)
        assert np.allclose(g[:, i], fd, rtol=2e-6, atol=1e-6 * (1 + np.abs(fd).max())), i


def test_autograd_function():
    w = SD.workload("egarch11", T=200)
    gm, om = gpu_model(w), ora_model(w)
    th = torch.from_numpy(SD.random_thetas(w, 16, 5, spread=0.05).T.copy()).cuda()
    th.requires_grad_(True)
    ll = SA.loglik(th, gm, 200)
    (ll * torch.arange(1, 17, dtype=torch.float64, device="cuda")).sum().backward()
    got = th.grad.cpu().numpy().T
    thn = th.detach().cpu().numpy().T
    want = np.array([(p + 1) * O.loglik_grad(om, thn[p], 200)[1] for p in range(16)])
    assert _grad_close(got, want, S.SMC_FP64)
    assert np.allclose(ll.detach().cpu().numpy(), O.loglik_batch(om, thn, 200)[0], rtol=1e-10)


@pytest.mark.parametrize("name,prec", [("linreg", 0), ("egarch11", 0), ("egarch2t", 1),
                                       ("egarch23", 0), ("egarch23", 1)])
def test_posterior_grad_matches_oracle(name, prec):
    w = SD.workload(name, T=300)
    gm, om = gpu_model(w, prec), ora_model(w)
    opop = O.Pop(om, 2, 40)
    opop.theta[:] = SD.random_thetas(w, 80, 8, spread=0.05)
    g = pop_to_gpu(gm, opop, with_grad=True)
    S.smc_posterior_grad(gm, g, 300)
    got = g.grad.cpu().numpy().T
    want = np.array([O.loglik_grad(om, opop.theta[p], 300)[1] + O.logprior_grad(om, opop.theta[p])[1]
                     for p in range(80)])
    assert _grad_close(got, want, prec)


@pytest.mark.parametrize("name,prec", [("linreg", 0), ("egarch11", 0), ("egarch2t", 0),
                                       ("egarch2t", 1), ("egarch23", 0)])
def test_mala_step_matches_oracle(name, prec):
    w = SD.workload(name, T=250)
    gm, om = gpu_model(w, prec), ora_model(w)
    J, N = 4, 32
    opop = O.Pop(om, J, N)
    if name == "linreg":
        # exact posterior draws: the step is then on the posterior's own scale
        opop.theta[:] = CF.posterior_draws(w.y[:w.T], w.X[:w.T], J * N, np.random.default_rng(12))
    else:
        opop.theta[:] = SD.random_thetas(w, J * N, 12, spread=0.05)
    for p in range(J * N):
        opop.logprior[p] = O.logprior(om, opop.theta[p])
    opop.loglik[:], st = O.loglik_batch(om, opop.theta, w.T)
    if om.S:
        opop.state[:, :om.S] = st
    _, _, chol, rc = O.moments(opop)
    hl = {"linreg": 1.0, "egarch23": 1.5}.get(name, 0.3) * chol
    g = pop_to_gpu(gm, opop, with_grad=True)
    S.smc_posterior_grad(gm, g, w.T)
    before = (opop.theta.copy(), opop.logprior.copy(), opop.loglik.copy())
    g0 = g.grad.cpu().numpy().T.copy()
    acc_g = torch.zeros(J * N, dtype=torch.uint8, device="cuda")
    S.smc_mutate(gm, g, w.T, torch.from_numpy(hl).cuda(), seed=2, cycle=1, it=3,
                 kernel=S.SMC_KERNEL_MALA, accepted=acc_g)
    n_o, acc_o = O.mutate(om, opop, w.T, hl, seed=2, cycle=1, it=3, kernel=O.MALA)
    acc_g = acc_g.cpu().numpy()
    assert 0 < n_o < J * N
    if prec == S.SMC_FP64:
        assert np.array_equal(acc_g, acc_o)
        assert np.allclose(theta_np(g), opop.theta, rtol=1e-11, atol=1e-12)
    else:
        err, _ = accept_audit(gm, om, *before, w.T, hl, 2, 0, 1, 3, acc_g, acc_o,
                              kernel=S.SMC_KERNEL_MALA, g0_gpu=g0)
        assert err < 2e-2
        same = acc_g == acc_o
        assert np.allclose(theta_np(g)[same], opop.theta[same], rtol=1e-5, atol=1e-6)
    # the stored gradient follows the particle
    want = np.array([O.loglik_grad(om, theta_np(g)[p], w.T)[1] +
                     O.logprior_grad(om, theta_np(g)[p])[1] for p in range(J * N)])
    assert _grad_close(g.grad.cpu().numpy().T, want, prec)


def test_mala_run_linreg_log_ml_matches_closed_form():
    w = SD.workload("linreg")
    gm = gpu_model(w)
    exact = CF.log_ml(w.y, w.X)
    g = S.Population(gm, 16, 256, max_chunk=32, with_grad=True)
    rec = S.smc_run(gm, g, seed=3, check_every=1, force_every=20, kernel=S.SMC_KERNEL_MALA)
    s = rec.summary()
    assert abs(s["log_ml"] - exact) < 3.5 * s["nse"], (s["log_ml"], exact, s["nse"])


def test_mala_replay_of_oracle_design():
    w = SD.workload("egarch11", T=150)
    gm, om = gpu_model(w), ora_model(w)
    rc, orec, opop = O.run(om, 2, 64, 4, kernel=O.MALA, Lmax=200, RmaxRec=64)
    assert rc == 0
    L = orec.L
    g = S.Population(gm, 2, 64, max_chunk=32, with_grad=True)
    grec = S.Record(gm, 2, Lmax=200, RmaxRec=64)
    grec.t_end[:L] = orec.t_end[:L]
    grec.R[:L] = orec.R[:L]
    grec.hchol[:L].copy_(torch.from_numpy(orec.hchol[:L].copy()))
    S.smc_run(gm, g, seed=4, record=grec, replay=True, kernel=S.SMC_KERNEL_MALA)
    sg, so = grec.summary(), orec.summary()
    assert sg["L"] == so["L"]
    assert sg["log_ml"] == pytest.approx(so["log_ml"], rel=1e-9, abs=1e-8)
    assert np.allclose(theta_np(g), opop.theta, rtol=1e-8, atol=1e-9)


# --------------------------------------- the Langevin workload at full size --
# EGARCH(2) Student-t, FP32 recursion, 64 x 1,024 particles, T = 10,000: the
# adjoint's forward sweep keeps 157 checkpoints of 64 observations per
# particle.  Sampled particles are checked one by one against the oracle.

def _full_2t():
    w = SD.workload("egarch2t")
    gm, om = gpu_model(w, S.SMC_FP32), ora_model(w)
    P = w.P
    idx = np.concatenate([[0, 1, 63, 64, P - 64, P - 1],
                          np.random.default_rng(9).choice(np.arange(65, P - 64), 10, replace=False)])
    return w, gm, om, P, idx


def test_loglik_backward_full_size_sampled():
    w, gm, om, P, idx = _full_2t()
    assert (P, w.T, -(-w.T // 64)) == (65536, 10000, 157)
    th = SD.random_thetas(w, P, 51, spread=0.01)
    dl = np.random.default_rng(5).uniform(0.5, 2.0, P)
    got = S.smc_loglik_backward(gm, torch.from_numpy(th.T.copy()).cuda(), w.T,
                                torch.from_numpy(dl).cuda()).cpu().numpy().T
    want = np.array([dl[p] * O.loglik_grad(om, th[p], w.T)[1] for p in idx])
    rel = np.abs(got[idx] - want) / (np.linalg.norm(want, axis=1, keepdims=True))
    print(f"[fp32] gradient egarch2t T=10000 P=65536: max error {rel.max():.3e} of the norm")
    assert _grad_close(got[idx], want, S.SMC_FP32)


def test_mala_step_full_size_sampled():
    w, gm, om, P, idx = _full_2t()
    th = SD.random_thetas(w, P, 52, spread=0.01)
    g = S.Population(gm, w.J, w.N, max_chunk=16, with_grad=True)
    g.theta.copy_(torch.from_numpy(th.T.copy()))
    g.loglik.copy_(S.smc_loglik(gm, g.theta, w.T))
    lp_o = np.array([O.logprior(om, th[p]) for p in idx])
    ll_o = np.array([O.loglik(om, th[p], w.T)[0] for p in idx])
    for k, p in enumerate(idx):
        g.loglik[int(p)] = ll_o[k]
        g.logprior[int(p)] = lp_o[k]
    S.smc_posterior_grad(gm, g, w.T)
    g0 = g.grad.cpu().numpy().T[idx].copy()
    hl = np.linalg.cholesky(np.cov(th[::16].T)) * 0.3
    acc = torch.zeros(P, dtype=torch.uint8, device="cuda")
    S.smc_mutate(gm, g, w.T, torch.from_numpy(hl).cuda(), seed=6, run=0, cycle=4, it=2,
                 kernel=S.SMC_KERNEL_MALA, accepted=acc)
    acc = acc.cpu().numpy()[idx]
    th_g = theta_np(g)[idx]
    acc_o = np.zeros(len(idx), bool)
    for k, p in enumerate(idx):
        a, th_o, _, _, _ = O.mutate_particle(om, int(p), th[p], lp_o[k], ll_o[k], w.T, hl,
                                             seed=6, run=0, cycle=4, it=2, kernel=O.MALA)
        acc_o[k] = a
        if a == bool(acc[k]):
            # the proposal's drift uses the FP32 gradient
            assert np.allclose(th_g[k], th_o, rtol=1e-5, atol=1e-6), int(p)
    err, _ = accept_audit(gm, om, th[idx], lp_o, ll_o, w.T, hl, 6, 0, 4, 2, acc, acc_o,
                          pidx=idx, kernel=S.SMC_KERNEL_MALA, g0_gpu=g0)
    assert err < 0.5
    assert acc_o.sum() > 0
