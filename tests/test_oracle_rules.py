"""Pins for the two adaptive rules of Section 3.3 that the oracle's whole-run
checks do not see: where a C phase ends, and how the Metropolis step size
moves.

C phase termination (Section 3.3): the phase ends at the first observation
date s whose relative effective sample size RSS = ESS / (JN) is below
D1 = 0.5, the ESS being pooled over all J*N particles with the weights
accumulated since the phase began.  The tests rebuild every date's pooled
RSS in numpy from the log-likelihood increments p(y_s | y_{1:s-1}, theta)
(the oracle's likelihood over one date from the previous date's recursion
state, eq C_phase_compute) and require the oracle's end date to be that
first date, with every earlier checked date at or above D1.  The strictness of "below"
is pinned exactly: a population with half its particles dead and the rest
equally weighted has RSS = 1/2 to the bit, which must not end the phase,
while one slightly uneven live particle must.

Step size (Section 3.3, "Metropolis steps"): h starts at 0.5 in every M
phase and moves by 0.1 after each iteration, up if the acceptance rate
exceeded the target (0.25 for the random walk) and down otherwise, within
[0.1, 1].  The oracle keeps h in tenths; the test replays that rule from the
recorded accept counts and requires the recorded step of every iteration
and the scaled factor hL = h L of the recorded particle variance's Cholesky
factor L.
"""
import math

import numpy as np
import pytest

import oracle as O
import synthdata as SD


def _increments(m, theta, t_max):
    """[T, P] log p(y_s | y_{1:s-1}, theta_p) for s = 1..t_max: the oracle's
    likelihood over the single date s, from the recursion state at s - 1 (a
    non-finite term counts as -inf, a zero density)."""
    P = theta.shape[0]
    inc = np.zeros((t_max, P))
    for p in range(P):
        st = None
        for s in range(1, t_max + 1):
            v, st = O.loglik(m, theta[p], t=s, state=st, t0=s - 1)
            inc[s - 1, p] = v if not math.isnan(v) else -math.inf
    return inc


def _pooled_rss(logw):
    """(sum w)^2 / (P sum w^2) of each row of logw [dates, P]."""
    mx = logw.max(axis=1, keepdims=True)
    e = np.exp(logw - mx)
    return e.sum(axis=1) ** 2 / (logw.shape[1] * (e * e).sum(axis=1))


def _prior_pop(m, J, N, seed):
    pop = O.Pop(m, J, N)
    O.init(m, pop, seed)
    return pop


@pytest.mark.parametrize("name,J,N,seed", [("egarch11", 4, 64, 3), ("egarch11", 8, 32, 11),
                                           ("egarch2t", 4, 64, 5), ("linreg", 4, 64, 2)])
def test_c_phase_ends_at_first_pooled_rss_below_half(name, J, N, seed):
    w = SD.workload(name, T=120)
    m = O.Model.from_workload(w)
    pop = _prior_pop(m, J, N, seed)
    inc = _increments(m, pop.theta.copy(), w.T)
    ll0 = pop.loglik.copy()
    t_from = 0
    phases = 0
    while t_from < w.T and phases < 3:
        t, rss, glwb = O.correct(m, pop, t_from, w.T, check_every=1, rss_min=0.5)
        cum = np.cumsum(inc[t_from:], axis=0)  # log weights at dates t_from+1..T
        r = _pooled_rss(cum)
        below = np.nonzero(r < 0.5)[0]
        expect = t_from + 1 + below[0] if below.size else w.T
        assert t == expect, (t_from, t, expect)
        assert np.all(r[:t - t_from - 1] >= 0.5)
        assert rss == pytest.approx(r[t - t_from - 1], rel=1e-12)
        lw = cum[t - t_from - 1]
        assert np.allclose(pop.logw, lw, rtol=1e-12, atol=1e-9)
        # group log mean weights of the phase's end (Section 4.2)
        g = lw.reshape(J, N)
        gm = g.max(axis=1, keepdims=True)
        ref = gm[:, 0] + np.log(np.exp(g - gm).mean(axis=1))
        assert np.allclose(glwb, ref, rtol=1e-12, atol=1e-12)
        # the likelihood has advanced by the same terms
        assert np.allclose(pop.loglik - ll0, inc[:t].sum(axis=0), rtol=1e-11, atol=1e-8)
        t_from = t
        phases += 1
    assert phases >= 2  # the rule was exercised from a nonzero start too


def test_c_phase_pooled_not_per_group():
    """Groups whose own RSS stays high while the pooled RSS falls: the phase
    must follow the pooled value."""
    w = SD.workload("egarch11", T=80)
    m = O.Model.from_workload(w)
    J, N = 2, 64
    rng = np.random.default_rng(7)
    th = SD.random_thetas(w, J * N, 7, spread=0.0)
    # group 0 near the truth, group 1 shifted in the scale parameter: within
    # each group the weights stay even, between the groups they part fast
    th[:N, 1] += 0.02 * rng.standard_normal(N)
    th[N:, 1] += 0.8 + 0.02 * rng.standard_normal(N)
    pop = O.Pop(m, J, N)
    pop.theta[:] = th
    inc = _increments(m, th, w.T)
    cum = np.cumsum(inc, axis=0)
    pooled = _pooled_rss(cum)
    per_group = np.minimum(_pooled_rss(cum[:, :N]), _pooled_rss(cum[:, N:]))
    first_pooled = int(np.nonzero(pooled < 0.5)[0][0]) + 1
    assert np.all(per_group[:first_pooled] >= 0.5)  # a per-group rule would not stop here
    t, _, _ = O.correct(m, pop, 0, w.T, check_every=1, rss_min=0.5)
    assert t == first_pooled


def test_c_phase_checks_only_scheduled_dates():
    """With checks every k-th observation (and always at t_max) the phase
    ends at the first checked date below D1, never between checks."""
    w = SD.workload("egarch11", T=97)
    m = O.Model.from_workload(w)
    for seed, k in ((3, 5), (4, 7), (9, 13)):
        pop = _prior_pop(m, 4, 32, seed)
        inc = _increments(m, pop.theta.copy(), w.T)
        r = _pooled_rss(np.cumsum(inc, axis=0))
        dates = [s for s in range(1, w.T + 1) if s % k == 0 or s == w.T]
        hit = [s for s in dates if r[s - 1] < 0.5]
        expect = hit[0] if hit else w.T
        t, rss, _ = O.correct(m, pop, 0, w.T, check_every=k, rss_min=0.5)
        assert t == expect
        assert rss == pytest.approx(r[t - 1], rel=1e-12)


def _exact_half_pop(m, live_beta):
    """Regression population: particles with log s2 = +inf have log density
    -inf at every observation (zero weight); the live ones carry the given
    slopes."""
    n = len(live_beta)
    pop = O.Pop(m, 2, n)  # 2n particles: n live, n dead
    pop.theta[:n, 0] = live_beta
    pop.theta[:n, 1] = math.log(0.64)
    pop.theta[n:, 0] = 0.0
    pop.theta[n:, 1] = math.inf
    return pop


def test_c_phase_rss_test_is_strict():
    y, X = SD.linreg_series(T=12, k=1, beta=(1.0,))
    m = O.Model(O.LINREG, 12, y, nreg=1, X=X)
    # n equal live weights and n zero weights: RSS = n^2 / (2n * n) = 1/2
    # exactly at every date, so "below 1/2" never holds and the phase runs
    # to t_max
    pop = _exact_half_pop(m, [1.0, 1.0, 1.0, 1.0])
    t, rss, _ = O.correct(m, pop, 0, 12, check_every=1, rss_min=0.5)
    assert rss == 0.5
    assert t == 12
    # one live particle slightly different: RSS just below 1/2 at the first
    # date, which ends the phase there
    pop = _exact_half_pop(m, [1.0, 1.0, 1.0, 1.3])
    t, rss, _ = O.correct(m, pop, 0, 12, check_every=1, rss_min=0.5)
    assert rss < 0.5
    assert t == 1


def _replay_step_rule(s, P, target_permille, label):
    """Checks the recorded step sizes of every cycle against the rule."""
    saw_equal = False
    for l in range(s["L"]):
        R = int(s["R"][l])
        mh = s["mh"][l, :R]
        nacc = s["n_acc"][l, :R]
        assert mh[0] == 5, (label, l)  # h = 0.5 at the start of each M phase
        for r in range(1, R):
            up = 1000 * int(nacc[r - 1]) > target_permille * P
            saw_equal |= 1000 * int(nacc[r - 1]) == target_permille * P
            want = min(10, max(1, int(mh[r - 1]) + (1 if up else -1)))
            assert mh[r] == want, (label, l, r, mh[r - 1], nacc[r - 1])
        # the scale applied is h times the factor of the particle variance
        hl = s["hchol"][l, :R]
        ch = s["chol"][l, :R]
        assert np.array_equal(hl, (mh[:, None, None] / 10.0) * ch), (label, l)
    return saw_equal


def test_step_size_rule_random_walk():
    w = SD.workload("egarch11", T=300)
    m = O.Model.from_workload(w)
    J, N = 4, 64
    rc, rec, _ = O.run(m, J, N, 5, Lmax=200, RmaxRec=64)
    assert rc == 0
    s = rec.summary()
    _replay_step_rule(s, J * N, 250, "egarch11")
    # the run moved h away from 0.5 within phases, so a missing reset at the
    # start of a phase would show
    assert any(int(s["mh"][l, int(s["R"][l]) - 1]) != 5 for l in range(s["L"]))
    used = np.concatenate([s["mh"][l, :int(s["R"][l])] for l in range(s["L"])])
    assert used.min() >= 1 and used.max() <= 10 and used.max() > 5


def test_step_size_rule_boundary_is_strict():
    """Small populations reach an acceptance rate of exactly 1/4, which must
    lower h (the rule raises it only above the target)."""
    y, X = SD.linreg_series(T=40, k=1, beta=(1.0,))
    m = O.Model(O.LINREG, 40, y, nreg=1, X=X)
    equal_seen = 0
    for seed in range(1, 13):
        rc, rec, _ = O.run(m, 2, 4, seed, Lmax=64, RmaxRec=32, Rbar=4, kappa=2)
        if rc != 0:
            continue  # a collapsed particle variance (not positive definite)
        equal_seen += _replay_step_rule(rec.summary(), 8, 250, f"seed {seed}")
    assert equal_seen >= 1


def test_step_size_rule_langevin_target():
    """The Langevin kernel's rule moves h toward acceptance 0.574."""
    y, X = SD.linreg_series(T=60)
    m = O.Model(O.LINREG, 60, y, nreg=3, X=X)
    rc, rec, _ = O.run(m, 4, 32, 3, kernel=O.MALA, Lmax=64, RmaxRec=64)
    assert rc == 0
    _replay_step_rule(rec.summary(), 128, 574, "mala")
