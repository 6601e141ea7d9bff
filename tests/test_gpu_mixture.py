"""GPU parity of the egarch_KI family (normal-mixture shocks, Section 5.1)
against the oracle: prior draws with the truncated theta_8i, the likelihood
recursion in FP64 and FP32 over the whole (K, I) grid, the 32-wide MFMA
moments (d = 17 and 26), Metropolis decisions and a replayed run.

Tolerances as in the other parity tests: FP64 log-likelihoods 1e-10
relative, FP32 1e-4 relative to max(|value|, observations); accept
decisions in FP64 bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from tests.gpu_helpers import accept_audit, gpu_model, ora_model, pop_to_gpu, sync, theta_np
from tests.test_gpu_parity import _close

pytestmark = pytest.mark.gpu

GRID = [f"egarch{K}{I}" for K in (1, 2, 3, 4) for I in (2, 3, 4)]


def _thetas(w, P, seed):
    """Near the truth in the volatility part (0.05) and far from it in the
    mixture part (0.5), so the components' weights, means and scales vary."""
    th = SD.random_thetas(w, P, seed, spread=0.05)
    b = 2 + 3 * w.K
    th[:, b:] += 0.5 * np.random.default_rng(seed + 1).standard_normal((P, 3 * w.I))
    th[:, b + 2 * w.I:] = np.maximum(th[:, b + 2 * w.I:], -2.9)
    return th


def test_init_from_prior_with_truncation():
    w = SD.workload("egarch23", T=50)
    gm, om = gpu_model(w), ora_model(w)
    J, N = 8, 512
    g = S.Population(gm, J, N)
    S.smc_init_from_prior(gm, g, seed=5, run=1)
    sync()
    th = theta_np(g)
    d = w.d
    i8 = 2 + 3 * w.K + 2 * w.I
    # particles whose first draw of some theta_8i fell below -3 (rejection used)
    first = np.array([O.normals(5, 1, p, 0, 0, O.PRIOR, d)[i8:] for p in range(J * N)])
    redrawn = np.nonzero((first < -3.0).any(axis=1))[0]
    assert redrawn.size > 0
    idx = np.concatenate([redrawn, [0, 1, J * N - 1]])
    for p in idx:
        want = O.prior_draw(om, 5, 1, int(p))
        assert np.allclose(th[p], want, rtol=1e-13, atol=1e-13), (p, th[p], want)
        assert g.logprior[int(p)].item() == pytest.approx(O.logprior(om, want), rel=1e-13)
    assert th[:, i8:].min() >= -3.0


@pytest.mark.parametrize("name", GRID)
@pytest.mark.parametrize("prec", [S.SMC_FP64, S.SMC_FP32])
def test_loglik_matches_oracle(name, prec):
    w = SD.workload(name, T=203)  # unrolled blocks of 8 and a ragged tail
    gm, om = gpu_model(w, prec), ora_model(w)
    P = 96
    th = _thetas(w, P, 5)
    for t in (1, 8, 9, 203):
        st = torch.zeros((gm.S, P), dtype=gm.state_dtype, device="cuda")
        ll = S.smc_loglik(gm, torch.from_numpy(th.T.copy()).cuda(), t, state_out=st).cpu().numpy()
        want, wst = O.loglik_batch(om, th, t)
        assert _close(ll, want, prec, t), (t, np.max(np.abs(ll - want)))
        assert np.allclose(st.cpu().numpy().T, wst, rtol=1e-8 if prec == 0 else 2e-3,
                           atol=1e-9 if prec == 0 else 2e-3)


@pytest.mark.parametrize("prec", [S.SMC_FP32, S.SMC_FP64])
def test_loglik_full_size_sampled(prec):
    """egarch_23 at the paper's size (T = 5,100, 65,536 particles)."""
    w = SD.workload("egarch23")
    gm, om = gpu_model(w, prec), ora_model(w)
    P = w.P
    th = SD.random_thetas(w, P, 9, spread=0.02)
    ll = S.smc_loglik(gm, torch.from_numpy(th.T.copy()).cuda(), w.T).cpu().numpy()
    idx = np.concatenate([np.random.default_rng(1).choice(P, 16, replace=False), [0, P - 1]])
    want = O.loglik_batch(om, th[idx], w.T)[0]
    assert _close(ll[idx], want, prec, w.T)
    assert np.all(np.isfinite(ll))


@pytest.mark.parametrize("name,J,N", [("egarch23", 4, 64), ("egarch23", 64, 1024),
                                      ("egarch44", 16, 1024), ("egarch44", 3, 13)])
def test_moments_32_wide_match_oracle(name, J, N):
    w = SD.workload(name, T=10)
    gm, om = gpu_model(w), ora_model(w)
    d = w.d
    opop = O.Pop(om, J, N)
    rng = np.random.default_rng(J + N + d)
    A = rng.standard_normal((d, d)) + 3 * np.eye(d)
    opop.theta[:] = rng.standard_normal((J * N, d)) @ A + rng.standard_normal(d) * 3
    g = pop_to_gpu(gm, opop)
    mh = torch.tensor([4], dtype=torch.int32, device="cuda")
    mean = torch.zeros(d, dtype=torch.float64, device="cuda")
    cov = torch.zeros((d, d), dtype=torch.float64, device="cuda")
    hl = S.smc_particle_moments(gm, g, mh, mean=mean, cov=cov)
    m_o, c_o, l_o, rc = O.moments(opop)
    assert rc == 0
    assert np.allclose(mean.cpu().numpy(), m_o, rtol=1e-12, atol=1e-12)
    assert np.allclose(cov.cpu().numpy(), c_o, rtol=1e-10, atol=1e-12)
    assert np.allclose(hl.cpu().numpy(), 0.4 * l_o, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("name,prec", [("egarch12", 0), ("egarch23", 0), ("egarch44", 0),
                                       ("egarch23", 1)])
def test_mutate_matches_oracle(name, prec):
    w = SD.workload(name, T=250)
    gm, om = gpu_model(w, prec), ora_model(w)
    J, N = 4, 64
    opop = O.Pop(om, J, N)
    opop.theta[:] = _thetas(w, J * N, 12)
    for p in range(J * N):
        opop.logprior[p] = O.logprior(om, opop.theta[p])
    opop.loglik[:], st = O.loglik_batch(om, opop.theta, w.T)
    opop.state[:, :om.S] = st
    _, _, chol, rc = O.moments(opop)
    assert rc == 0
    hl = 0.5 * chol
    g = pop_to_gpu(gm, opop)
    before = (opop.theta.copy(), opop.logprior.copy(), opop.loglik.copy())
    acc_g = torch.zeros(J * N, dtype=torch.uint8, device="cuda")
    n_g = S.smc_mutate(gm, g, w.T, torch.from_numpy(hl).cuda(), seed=8, run=1, cycle=2, it=3,
                       accepted=acc_g)
    n_o, acc_o = O.mutate(om, opop, w.T, hl, seed=8, run=1, cycle=2, it=3)
    acc_g = acc_g.cpu().numpy()
    assert 0 < n_o < J * N
    if prec == S.SMC_FP64:
        assert np.array_equal(acc_g, acc_o)
        assert n_g.item() == n_o
        assert np.allclose(theta_np(g), opop.theta, rtol=1e-12, atol=1e-13)
        assert np.allclose(g.loglik.cpu().numpy(), opop.loglik, rtol=1e-10)
    else:
        err, _ = accept_audit(gm, om, *before, w.T, hl, 8, 1, 2, 3, acc_g, acc_o)
        assert err < 1e-2
        same = acc_g == acc_o
        assert np.allclose(theta_np(g)[same], opop.theta[same], rtol=1e-12, atol=1e-13)


def test_replay_of_oracle_design():
    """The GPU replays the oracle's adaptive egarch_23 run (t_l, hL, R_l)."""
    w = SD.workload("egarch23", T=160)
    gm, om = gpu_model(w), ora_model(w)
    rc, orec, opop = O.run(om, 4, 64, 6, check_every=1, Lmax=300, RmaxRec=64)
    assert rc == 0
    so = orec.summary()
    L = orec.L
    g = S.Population(gm, 4, 64, max_chunk=32)
    grec = S.Record(gm, 4, Lmax=300, RmaxRec=64)
    grec.t_end[:L] = orec.t_end[:L]
    grec.R[:L] = orec.R[:L]
    grec.hchol[:L].copy_(torch.from_numpy(orec.hchol[:L].copy()))
    S.smc_run(gm, g, seed=6, check_every=1, record=grec, replay=True)
    sg = grec.summary()
    assert sg["L"] == so["L"]
    assert sg["log_ml"] == pytest.approx(so["log_ml"], rel=1e-10, abs=1e-9)
    assert np.allclose(theta_np(g), opop.theta, rtol=1e-9, atol=1e-10)


def test_mala_run_replays_oracle_design():
    """The Langevin kernel on the mixture family: the GPU replays the oracle's
    adaptive MALA run of egarch_23 (gradients through eqs EGARCH_tran1/2)."""
    w = SD.workload("egarch23", T=120)
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


def test_mutate_full_size_sampled():
    """One M step of egarch_23 at the paper's size (65,536 particles, T =
    5,100, FP64): sampled particles replayed one by one by the oracle with
    their global Philox indices."""
    w = SD.workload("egarch23")
    gm, om = gpu_model(w), ora_model(w)
    P = w.P
    th = _thetas(w, P, 31)
    g = S.Population(gm, w.J, w.N, max_chunk=16)
    g.theta.copy_(torch.from_numpy(th.T.copy()))
    idx = np.concatenate([[0, 1, P - 1], np.random.default_rng(2).choice(P, 9, replace=False)])
    g.loglik.copy_(S.smc_loglik(gm, g.theta, w.T))
    lp_o = {int(p): O.logprior(om, th[p]) for p in idx}
    ll_o = {int(p): O.loglik(om, th[p], w.T)[0] for p in idx}
    for p in idx:
        g.loglik[int(p)] = ll_o[int(p)]
        g.logprior[int(p)] = lp_o[int(p)]
    hl = np.linalg.cholesky(np.cov(th[::16].T)) * 0.3
    acc = torch.zeros(P, dtype=torch.uint8, device="cuda")
    S.smc_mutate(gm, g, w.T, torch.from_numpy(hl).cuda(), seed=4, run=0, cycle=9, it=2,
                 accepted=acc)
    acc = acc.cpu().numpy()
    th_g = theta_np(g)
    for p in idx:
        p = int(p)
        a, th_o, _, ll1, _ = O.mutate_particle(om, p, th[p], lp_o[p], ll_o[p], w.T, hl, seed=4,
                                               run=0, cycle=9, it=2)
        assert a == bool(acc[p]), p
        assert np.allclose(th_g[p], th_o, rtol=1e-12, atol=1e-13)
        if a:
            assert g.loglik[p].item() == pytest.approx(ll1, rel=1e-10)
