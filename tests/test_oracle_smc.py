"""Pins for the oracle's C, S and M phases and its estimators.

Pins used here: hand-computed values on tiny inputs, numpy's covariance and
Cholesky, exact statistical properties (unbiased resampling counts, invariance
of the Metropolis kernel, Proposition 1's t(J-1) law of the standardised
error) and the closed-form marginal likelihood and posterior of the
conjugate regression.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import simpson

import oracle as O
import synthdata as SD
from oracle import closed_form as CF


# ------------------------------------------------------------- estimators ---

def test_rss_special_cases():
    assert O.rss(np.zeros(1000)) == pytest.approx(1.0, rel=1e-15)
    lw = np.full(1000, -np.inf)
    lw[17] = 3.0
    assert O.rss(lw) == pytest.approx(1e-3, rel=1e-15)
    # w = (1, 2, 3, 4): ESS = 10^2 / 30, RSS = ESS / 4
    assert O.rss(np.log([1.0, 2.0, 3.0, 4.0]) + 500.0) == pytest.approx(100 / 120, rel=1e-14)


def test_log_ml_hand_values():
    # one cycle, group mean weights 1 and 3: wbar = 2, NSE = sqrt(2/2)/2
    out = O.log_ml(np.log([[1.0, 3.0]]))
    assert out == pytest.approx([math.log(2.0), 0.5, math.log(2.0)], rel=1e-14)
    # two cycles: wbar_j = (2, 6), wbar = 4, NSE = sqrt(8/2)/4; wtilde = 2 * 2
    out = O.log_ml(np.log([[1.0, 3.0], [2.0, 2.0]]))
    assert out == pytest.approx([math.log(4.0), 0.5, math.log(4.0)], rel=1e-14)
    # equal groups: no numerical error
    out = O.log_ml(np.full((5, 8), -3.25))
    assert out[0] == pytest.approx(-16.25, rel=1e-15)
    assert out[1] == 0.0
    # shift invariance of the estimator in the log domain
    g = np.random.default_rng(0).normal(size=(4, 6))
    a, b = O.log_ml(g), O.log_ml(g + 1000.0)
    assert b[0] - a[0] == pytest.approx(4000.0, rel=1e-12)
    assert b[1] == pytest.approx(a[1], rel=1e-12)


def test_rne_hand_value_and_iid():
    y, X = SD.linreg_series(T=5)
    m = O.Model(O.LINREG, 5, y, nreg=3, X=X)
    pop = O.Pop(m, 2, 2)
    pop.theta[:] = np.array([[0.0], [2.0], [1.0], [3.0]]) * np.ones((1, 4))
    # gbar_j = (1, 2): vhat = 2 * 0.5 = 1; var-hat = 5/3
    assert O.rne_mean(pop) == pytest.approx(5.0 / 3.0, rel=1e-14)
    # iid draws: RNE near one (Condition 6)
    pop = O.Pop(m, 64, 256)
    pop.theta[:] = np.random.default_rng(3).standard_normal(pop.theta.shape)
    assert 0.6 < O.rne_mean(pop) < 1.6


# -------------------------------------------------------------- S phase -----

def test_resample_equal_weights_is_identity():
    # residual: one copy each; stratified / systematic: draw k lies in [k, k+1)
    for scheme in (O.RESIDUAL, O.STRATIFIED, O.SYSTEMATIC):
        anc, bad = O.resample(3, 64, np.full(192, -7.0), scheme, seed=4)
        assert bad == 0
        assert np.array_equal(anc, np.arange(192))


def test_resample_integer_copies_are_exact():
    # N W = (2, 1, 1, 0): residual resampling is deterministic
    lw = np.log([0.5, 0.25, 0.25, 1e-300])
    anc, bad = O.resample(1, 4, lw, O.RESIDUAL, seed=2)
    assert bad == 0
    assert anc.tolist() == [0, 0, 1, 2]
    # group offsets
    anc, _ = O.resample(2, 4, np.concatenate([lw, lw[::-1]]), O.RESIDUAL, seed=2)
    assert anc.tolist() == [0, 0, 1, 2, 5, 6, 7, 7]


def test_resample_dead_group_reported():
    lw = np.zeros(8)
    lw[4:] = -np.inf
    anc, bad = O.resample(2, 4, lw, O.RESIDUAL, seed=1)
    assert bad == 1
    assert anc[4:].tolist() == [4, 5, 6, 7]


@pytest.mark.parametrize("scheme", [O.RESIDUAL, O.MULTINOMIAL, O.STRATIFIED, O.SYSTEMATIC])
def test_resample_counts_unbiased(scheme):
    N = 16
    w = np.random.default_rng(8).gamma(0.7, size=N)
    W = w / w.sum()
    lw = np.log(w)
    counts = np.zeros(N)
    n_rep = 4000
    for seed in range(n_rep):
        anc, _ = O.resample(1, N, lw, scheme, seed=seed)
        assert np.all(np.diff(anc) >= 0)
        c = np.bincount(anc, minlength=N)
        assert c.sum() == N
        if scheme == O.RESIDUAL:
            assert np.all(c >= np.floor(N * W))
        if scheme in (O.STRATIFIED, O.SYSTEMATIC):
            # one draw per stratum [k, k+1) of the running sum N sum_{m<=n} W_m:
            # the running count sits in {floor, floor + 1} of it
            x = N * np.cumsum(W)
            cc = np.cumsum(c)
            assert np.all((cc >= np.floor(x - 1e-9)) & (cc <= np.floor(x + 1e-9) + 1))
        if scheme == O.SYSTEMATIC:
            # a common offset: every count is floor or ceil of N W_n
            assert np.all((c >= np.floor(N * W - 1e-9)) & (c <= np.ceil(N * W + 1e-9)))
        counts += c
    # E[count_n] = N W_n; multinomial variance bounds the residual one
    mean = counts / n_rep
    sd = np.sqrt(N * W * (1 - W) / n_rep)
    assert np.all(np.abs(mean - N * W) < 4.5 * sd + 1e-12)


def test_stratified_brute_force_tiny():
    """Ancestors from the definition: the k-th draw is the first n whose
    running sum of N W exceeds k + U_k (U_k the k-th uniform of the stream)."""
    N = 5
    lw = np.log(np.array([0.05, 0.4, 0.15, 0.3, 0.1]))
    for seed in range(50):
        # counter (group, cycle, k / 4, purpose 2 = resampling), key (seed, run)
        u = np.array([O.philox([0, 3, k // 4, 2], [seed, 0])[k % 4] for k in range(N)],
                     dtype=np.uint64)
        uf = (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        x = N * np.cumsum(np.exp(lw) / np.exp(lw).sum())
        for scheme, pts in ((O.STRATIFIED, np.arange(N) + uf),
                            (O.SYSTEMATIC, np.arange(N) + uf[0])):
            want = np.searchsorted(x, pts, side="right")
            anc, _ = O.resample(1, N, lw, scheme, seed=seed, cycle=3)
            assert anc.tolist() == want.tolist(), (seed, scheme)


# ---------------------------------------------------------------- moments ---

def test_moments_match_numpy():
    w = SD.workload("egarch2t", T=10)
    m = O.Model.from_workload(w)
    pop = O.Pop(m, 4, 100)
    rng = np.random.default_rng(1)
    A = rng.standard_normal((9, 9))
    pop.theta[:] = rng.standard_normal((400, 9)) @ A + 3.0
    mean, cov, chol, rc = O.moments(pop)
    assert rc == 0
    assert np.allclose(mean, pop.theta.mean(0), rtol=1e-13)
    assert np.allclose(cov, np.cov(pop.theta.T), rtol=1e-11, atol=1e-12)
    assert np.allclose(chol, np.linalg.cholesky(np.cov(pop.theta.T)), rtol=1e-9, atol=1e-10)
    pop.theta[:, 3] = 1.0  # singular
    assert O.moments(pop)[3] == -1


# ---------------------------------------------------------------- M phase ---

@pytest.mark.parametrize("kernel", [O.RW, O.MALA, O.INDEP])
def test_metropolis_leaves_posterior_invariant(kernel):
    """Start from exact posterior draws of the conjugate regression; after
    several Metropolis iterations the marginals are still the posterior.  The
    independent sampler gets a deliberately mismatched Gaussian (shifted by
    0.7 sd, scaled 1.3x), so only a correct proposal-density ratio keeps the
    posterior invariant."""
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    rng = np.random.default_rng(21)
    J, N = 8, 512
    pop = O.Pop(m, J, N)
    pop.theta[:] = CF.posterior_draws(w.y, w.X, J * N, rng)
    for p in range(J * N):
        pop.logprior[p] = O.logprior(m, pop.theta[p])
    pop.loglik[:] = O.loglik_batch(m, pop.theta)[0]
    start = pop.theta.copy()
    n_acc_tot = 0
    for it in range(1, 7):
        mean, cov, chol, rc = O.moments(pop)
        assert rc == 0
        arg = 0.5 * chol
        if kernel == O.INDEP:
            arg = np.concatenate([(1.3 * chol).ravel(), mean + 0.7 * np.sqrt(np.diag(cov))])
        n_acc, acc = O.mutate(m, pop, w.T, arg, seed=5, cycle=1, it=it, kernel=kernel)
        n_acc_tot += n_acc
    assert n_acc_tot > 0.2 * 6 * J * N
    assert np.mean(np.any(pop.theta != start, axis=1)) > 0.8
    fresh = CF.posterior_draws(w.y, w.X, J * N, np.random.default_rng(99))
    for i in range(4):
        assert stats.ks_2samp(pop.theta[:, i], fresh[:, i]).pvalue > 1e-3
    # the stored likelihood and prior follow the accepted particles
    ll = O.loglik_batch(m, pop.theta[:50])[0]
    assert np.allclose(ll, pop.loglik[:50], rtol=1e-13)


def test_mutate_accept_rule_extremes():
    w = SD.workload("egarch11", T=200)
    m = O.Model.from_workload(w)
    pop = O.Pop(m, 2, 8)
    O.init(m, pop, seed=3)
    pop.loglik[:] = O.loglik_batch(m, pop.theta, t=200)[0]
    # zero step: proposal equals current, Delta = 0 > log u whenever the
    # posterior kernel is finite (a non-finite one gives a NaN Delta: reject)
    finite = np.isfinite(pop.loglik)
    n, acc = O.mutate(m, pop, 200, np.zeros((5, 5)), seed=1)
    assert n == finite.sum() and np.array_equal(acc.astype(bool), finite)
    # a current state with infinite posterior mass is never left
    pop.loglik[:] = np.inf
    n, acc = O.mutate(m, pop, 200, 0.1 * np.eye(5), seed=1)
    assert n == 0


# ------------------------------------------------------------ end to end ----

def _linreg_run(J, N, seed, **kw):
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    rc, rec, pop = O.run(m, J, N, seed, check_every=1, force_every=20, **kw)
    assert rc == 0
    return w, rec, pop


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_linreg_log_ml_matches_closed_form(seed):
    w, rec, pop = _linreg_run(16, 256, seed)
    s = rec.summary()
    exact = CF.log_ml(w.y, w.X)
    assert abs(s["log_ml"] - exact) < 3.5 * s["nse"]
    assert abs(s["log_ml_tilde"] - exact) < 3.5 * s["nse"] + 0.05
    assert s["t_end"][-1] == w.T
    assert all(t % 20 == 0 or t == w.T or t < 20 * (t // 20 + 1) for t in s["t_end"])
    # dates of interest are cycle ends
    assert set(range(20, 201, 20)) <= set(s["t_end"].tolist())


def test_linreg_predictive_likelihoods_match_closed_form():
    w, rec, pop = _linreg_run(16, 256, 7)
    s = rec.summary()
    t_prev = 0
    for l in range(s["L"]):
        g = s["group_logwbar"][l]
        mx = g.max()
        r = np.exp(g - mx)
        est = mx + math.log(r.mean())
        nse = math.sqrt(((r - r.mean()) ** 2).sum() / (16 * 15)) / r.mean()
        exact = CF.log_predictive(w.y, w.X, t_prev, s["t_end"][l])
        assert abs(est - exact) < 4.5 * nse + 1e-3, (l, est, exact, nse)
        t_prev = s["t_end"][l]


def test_linreg_posterior_means_match_closed_form():
    w, rec, pop = _linreg_run(16, 256, 11)
    mb, es2, elog = CF.posterior_means(w.y, w.X)
    want = np.concatenate([mb, [elog]])
    gj = pop.theta.reshape(16, 256, 4).mean(1)
    nse = gj.std(0, ddof=1) / math.sqrt(16)
    assert np.all(np.abs(gj.mean(0) - want) < 4.5 * nse)


def test_replay_reproduces_and_new_seed_agrees():
    w, rec, pop = _linreg_run(8, 256, 5)
    s = rec.summary()
    m = O.Model.from_workload(w)
    rc, rec2, pop2 = O.run(m, 8, 256, 5, check_every=1, record=rec)
    assert rc == 0
    s2 = rec2.summary()
    assert np.array_equal(s2["t_end"], s["t_end"])
    assert s2["log_ml"] == s["log_ml"]
    assert np.array_equal(pop2.theta, pop.theta)
    rc, rec3, _ = O.run(m, 8, 256, 6, check_every=1, record=rec)
    s3 = rec3.summary()
    assert abs(s3["log_ml"] - s["log_ml"]) < 3.5 * math.hypot(s["nse"], s3["nse"])


def test_deterministic_m_phase_lengths():
    w, rec, pop = _linreg_run(4, 256, 3)
    s = rec.summary()
    for l in range(s["L"]):
        assert s["R"][l] == (21 if s["rss"][l] < 0.2 else 7)


def test_rne_stopping_rule():
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    rc, rec, pop = O.run(m, 8, 128, 2, check_every=1, force_every=20, stop_rule=1, E1=0.35,
                         Rmax=40)
    assert rc == 0
    s = rec.summary()
    assert np.all((s["R"] >= 1) & (s["R"] <= 40))
    assert O.rne_mean(pop) > 0.35 or s["R"][-1] == 40
    exact = CF.log_ml(w.y, w.X)
    assert abs(s["log_ml"] - exact) < 4.5 * s["nse"]


@pytest.mark.slow
def test_nse_calibration_proposition1():
    """(log-ML - exact) / NSE across independent runs follows t(J-1)."""
    w = SD.workload("linreg", T=100)
    m = O.Model.from_workload(w)
    exact = CF.log_ml(w.y, w.X)
    J = 8
    z = []
    for seed in range(1, 81):
        rc, rec, _ = O.run(m, J, 128, seed, check_every=1, force_every=20)
        assert rc == 0
        z.append((rec.c.log_ml - exact) / rec.c.nse)
    assert stats.kstest(z, "t", args=(J - 1,)).pvalue > 1e-3


# ------------------------------------------- functions of interest (f2) ---

def test_report_is_calibrated_on_iid_and_clustered_draws():
    """Section 2.3: for independent draws RNE is about 1 and the NSE matches
    the sampling sd of the grand mean; with every group made of copies of
    one draw (N copies), RNE is about 1/N."""
    J, N, G = 8, 64, 2
    rng = np.random.default_rng(0)
    nse2, rne, err2 = [], [], []
    for _ in range(300):
        g = rng.standard_normal((J * N, G)) * np.array([1.0, 3.0]) + np.array([0.5, -2.0])
        out = O.report(J, N, g)
        assert np.allclose(out[:, 0], g.mean(0), rtol=1e-12)
        nse2.append(out[:, 2] ** 2)
        rne.append(out[:, 3])
        err2.append((out[:, 0] - np.array([0.5, -2.0])) ** 2)
    sd_mean2 = np.array([1.0, 9.0]) / (J * N)
    assert np.allclose(np.mean(nse2, 0), sd_mean2, rtol=0.1)
    assert np.allclose(np.mean(err2, 0), sd_mean2, rtol=0.2)
    # v-hat / var-hat has expectation one (RNE itself is a ratio of them)
    assert np.allclose(np.mean(1.0 / np.array(rne), 0), 1.0, atol=0.06)
    # clustered: each group holds N identical values, so var-hat and v-hat
    # share the between-group sum of squares and RNE = (J - 1) / (NJ - 1)
    for _ in range(3):
        g = np.repeat(rng.standard_normal((J, 1)), N, axis=0)
        assert O.report(J, N, g)[0, 3] == pytest.approx((J - 1) / (N * J - 1), rel=1e-12)


def test_report_hand_values():
    # J = 2 groups of N = 2: group means 1 and 3, grand mean 2
    g = np.array([[0.0], [2.0], [3.0], [3.0]])
    out = O.report(2, 2, g)[0]
    var = ((0 - 2) ** 2 + 0 + 1 + 1) / 3.0
    assert out[0] == pytest.approx(2.0)
    assert out[1] == pytest.approx(math.sqrt(var))
    assert out[2] == pytest.approx(math.sqrt(((1 - 2) ** 2 + (3 - 2) ** 2) / 2.0))
    assert out[3] == pytest.approx(var / (2.0 / 1.0 * 2.0))


@pytest.mark.parametrize("name", ["egarch11", "egarch23"])
def test_log_volatility_is_the_simulated_path(name):
    """g1 at the generating parameters is log h_t of the data-generating
    process, at every date."""
    w = SD.workload(name, T=300)
    m = O.Model.from_workload(w)
    _, _, h = SD.egarch_series(w.theta_true, 300, w.K, w.shock,
                               SD.DATA_SEED_BASE + (2 if name == "egarch11" else 10 * w.K + w.I),
                               return_path=True)
    assert np.allclose(h[:300], np.abs(w.y - w.theta_true[0] / 1000) /
                       np.abs(SD.egarch_series(w.theta_true, 300, w.K, w.shock,
                                               SD.DATA_SEED_BASE + (2 if name == "egarch11" else 10 * w.K + w.I),
                                               return_path=True)[1]), rtol=1e-9)
    for t in (1, 2, 50, 300):
        _, st = O.loglik(m, w.theta_true, t=t)
        g = O.test_fns(m, w.theta_true, st, t)
        assert g[0] == pytest.approx(math.log(h[t - 1]), rel=1e-10)


@pytest.mark.parametrize("name", ["egarch11", "egarch23", "egarch2t"])
def test_loss_probability_and_skewness_by_quadrature(name):
    """g3 = P(Y_{t+1} < -0.03 | theta, y_{1:t}) from the conditional density
    of the next observation (the oracle's likelihood as a function of
    y_{t+1}, integrated), for Gaussian, mixture and Student-t shocks; g2 = its
    standardised third moment."""
    T = 41
    w = SD.workload(name, T=T)
    m = O.Model.from_workload(w)
    x = w.theta_true + 0.1 * np.random.default_rng(2).standard_normal(w.d)
    x[1] = math.log(0.02)  # a scale at which -3% is in the body of the density
    t = T - 1
    ll_prev, st = O.loglik(m, x, t=t)
    g = O.test_fns(m, x, st, t)
    # conditional density of y_T on a grid
    muY = x[0] / 1000
    grid = np.linspace(muY - 1.0, -0.03, 20001)
    dens = []
    for yv in grid:
        y2 = m.y.copy()
        y2[T - 1] = yv
        mm = O.Model(O.EGARCH, T, y2, K=w.K, shock=w.shock, I=w.I)
        dens.append(math.exp(O.loglik(mm, x)[0] - ll_prev))
    # Simpson's rule on the grid; the mass below mu_Y - 1 (50 scales) is
    # under 1e-10 of g3 even for the t shocks' heavier tail
    assert g[-1] == pytest.approx(simpson(dens, x=grid), rel=1e-8, abs=1e-12)
    assert 0.001 < g[-1] < 0.999
    if name == "egarch23":
        p, mu, sg = O.mixture_params(m, x)
        # third moment by quadrature of the mixture density
        z = np.linspace(-15, 15, 60001)
        f = sum(p[i] * stats.norm.pdf(z, mu[i], sg[i]) for i in range(len(p)))
        assert g[1] == pytest.approx(np.trapezoid(z ** 3 * f, z), rel=1e-6, abs=1e-9)


def test_student_t_loss_probability_matches_scipy():
    """g3 for Student-t shocks is the t_nu distribution function at the
    standardised point x sqrt(nu / (nu - 2)) (the shock has unit variance):
    checked against scipy over the tails, the centre and nu from near 2 to
    far beyond the prior's range.  With t = 0 and sigma_Y = 1, g3's argument
    x is set through mu_Y alone.  Dropping the standardisation, or taking the
    wrong side of the incomplete-beta symmetry, fails it.  Above nu = 1000 the
    log-gamma difference in 1/B(nu/2, 1/2) cancels to about a(log a)
    ulp-relative, a = nu/2, which sets the looser bar there."""
    w = SD.workload("egarch2t", T=50)
    m = O.Model.from_workload(w)
    assert O.num_test_fns(m) == 2
    th = w.theta_true.copy()
    th[1] = 0.0
    st = np.zeros(m.S)
    for nu in (2.05, 2.5, 3.0, 4.0, 7.3, 12.0, 30.0, 200.0, 1000.0, 1e4, 1e7):
        th[2 + 3 * w.K] = math.log(nu - 2.0)
        for x in (-80.0, -6.0, -1.5, -0.2, 0.0, 1e-3, 0.7, 3.0, 50.0):
            th[0] = -1000.0 * (x + 0.03)
            g = O.test_fns(m, th, st, 0)
            want = stats.t.cdf(x * math.sqrt(nu / (nu - 2.0)), nu)
            rel = 1e-11 if nu <= 1000.0 else 1e-7
            # relative in the lower tail, absolute near 1
            assert g[1] == pytest.approx(want, rel=rel, abs=1e-15 if x < 0 else rel), (nu, x)
    th[0] = -1000.0 * 0.03
    assert O.test_fns(m, th, st, 0)[1] == 0.5
    # textbook closed forms of the t distribution function, z = x sqrt(nu / (nu - 2)):
    # nu = 3: 1/2 + (z / (sqrt 3 (1 + z^2/3)) + atan(z / sqrt 3)) / pi;
    # nu = 4: 1/2 + z (z^2 + 6) / (2 (z^2 + 4)^(3/2))
    for nu, cdf in ((3.0, lambda z: 0.5 + (z / (math.sqrt(3.0) * (1.0 + z * z / 3.0))
                                           + math.atan(z / math.sqrt(3.0))) / math.pi),
                    (4.0, lambda z: 0.5 + z * (z * z + 6.0) / (2.0 * (z * z + 4.0) ** 1.5))):
        th[2 + 3 * w.K] = math.log(nu - 2.0)
        for x in (-7.0, -2.0, -0.4, 0.3, 1.1, 5.0):
            th[0] = -1000.0 * (x + 0.03)
            want = cdf(x * math.sqrt(nu / (nu - 2.0)))
            assert O.test_fns(m, th, st, 0)[1] == pytest.approx(want, rel=1e-12, abs=1e-15), (nu, x)
    # the limits: mu_Y = +inf puts x at -inf, mu_Y = -inf at +inf
    th[0] = math.inf
    assert O.test_fns(m, th, st, 0)[1] == 0.0
    th[0] = -math.inf
    assert O.test_fns(m, th, st, 0)[1] == 1.0


def test_log_score_matches_closed_form():
    """log p(y_{b+1:T} | y_{1:b}) with a burn-in b that is a date of interest."""
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    exact = CF.log_predictive(w.y, w.X, 100, w.T)
    hits = 0
    for seed in (1, 2, 3):
        rc, rec, _ = O.run(m, 16, 256, seed, check_every=1, burn_in=100)
        assert rc == 0
        s = rec.summary()
        assert 100 in s["t_end"].tolist()
        assert abs(s["log_score"] - exact) < 4.0 * s["log_score_nse"]
        assert s["log_score_nse"] < s["nse"]
        hits += abs(s["log_score"] - exact) < 2.5 * s["log_score_nse"]
    assert hits >= 2


def test_rne_rule_uses_e2_at_dates_of_interest():
    w = SD.workload("egarch23", T=120, J=8, N=64)
    m = O.Model.from_workload(w)
    rc, rec, _ = O.run(m, 8, 64, 3, check_every=1, force_every=40, stop_rule=1, E1=0.2,
                       E2=0.6, Rmax=30, test_fn=O.TEST_MODEL, moments=True)
    assert rc == 0
    s = rec.summary()
    for l in range(s["L"]):
        at_date = s["t_end"][l] % 40 == 0 or s["t_end"][l] == 120
        rne = s["moments"][l, :, 3].mean()
        if s["R"][l] < 30:
            assert rne > (0.6 if at_date else 0.2), (l, rne)
        if not at_date and s["R"][l] > 1:
            # one iteration fewer would not have passed E1 at the time (checked
            # only through the recorded R: the rule stops at the first pass)
            assert s["R"][l] <= 30
    assert any(s["t_end"][l] % 40 == 0 for l in range(s["L"]))


def test_hybrid_two_steps_agree_with_closed_form():
    """Algorithm 3: step 2 replays step 1's design with a new key; both
    estimate the regression's marginal likelihood and log score."""
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    rc, r1, r2, _ = O.run_hybrid(m, 16, 256, 11, 12, check_every=1, burn_in=100)
    assert rc == 0
    s1, s2 = r1.summary(), r2.summary()
    assert s1["L"] == s2["L"]
    assert np.array_equal(s1["t_end"], s2["t_end"]) and np.array_equal(s1["R"], s2["R"])
    assert s1["log_ml"] != s2["log_ml"]  # new particles
    exact = CF.log_ml(w.y, w.X)
    exact_ls = CF.log_predictive(w.y, w.X, 100, w.T)
    for s in (s1, s2):
        assert abs(s["log_ml"] - exact) < 3.5 * s["nse"]
        assert abs(s["log_score"] - exact_ls) < 3.5 * s["log_score_nse"]
    z = abs(s1["log_ml"] - s2["log_ml"]) / math.hypot(s1["nse"], s2["nse"])
    assert z < 4.0


def test_independent_sampler_run_matches_closed_form():
    """The independent Gaussian sampler (Section 3.3) inside the whole
    simulator: the regression's marginal likelihood within 3.5 NSE."""
    w = SD.workload("linreg")
    m = O.Model.from_workload(w)
    rc, rec, _ = O.run(m, 16, 256, 4, check_every=1, force_every=20, kernel=O.INDEP)
    assert rc == 0
    s = rec.summary()
    assert abs(s["log_ml"] - CF.log_ml(w.y, w.X)) < 3.5 * s["nse"]
    # the recorded means are the particle means that centred the proposals
    assert np.all(np.isfinite(rec.mean[:s["L"], 0]))
