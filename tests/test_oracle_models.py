"""Pins for the oracle's priors, per-observation densities and gradients.

Each check compares with something the oracle does not compute itself:
scipy's densities, the paper's Table 1 (golden fixture), the data-generating
process run forward, exact symmetries and finite differences.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O
import synthdata as SD

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    with open(os.path.join(GOLDEN, "table1_priors.json")) as f:
        return json.load(f)


def _egarch_model(K, shock, T=400, seed=11, theta=None):
    th = theta if theta is not None else (SD.egarch11_truth() if K == 1 else SD.egarch2t_truth())
    if K == 2 and shock == SD.GAUSS:
        th = th[:8]
    if K == 1 and shock == SD.STUDENT_T:
        th = np.concatenate([th, [math.log(6.0)]])
    y, z, h = SD.egarch_series(th, T, K, shock, seed, return_path=True)
    return O.Model(O.EGARCH, T, y, K=K, shock=shock), th, z, h


# ---------------------------------------------------------------- priors ---

@pytest.mark.parametrize("K,shock", [(1, 0), (2, 0), (2, 1)])
def test_egarch_logprior_is_table1(K, shock):
    t1 = _table1()
    m, th, _, _ = _egarch_model(K, shock, T=10)
    means = ([t1["theta1_mu"]["mean"], math.log(t1["theta2_sigma"]["mean_log_of"])]
             + [math.atanh(t1["theta3_alpha"]["mean_atanh_of"])] * K
             + [math.log(t1["theta4_beta"]["mean_log_of"])] * K
             + [t1["theta5_gamma"]["mean"]] * K)
    sds = ([t1["theta1_mu"]["sd"], t1["theta2_sigma"]["sd"]] + [t1["theta3_alpha"]["sd"]] * K
           + [t1["theta4_beta"]["sd"]] * K + [t1["theta5_gamma"]["sd"]] * K)
    if shock == SD.STUDENT_T:
        means.append(math.log(t1["theta9_nu"]["mean_log_of"]))
        sds.append(t1["theta9_nu"]["sd"])
    rng = np.random.default_rng(1)
    for _ in range(5):
        x = th + rng.standard_normal(th.size)
        want = stats.norm.logpdf(x, means, sds).sum()
        assert O.logprior(m, x) == pytest.approx(want, rel=1e-13, abs=1e-12)


def test_linreg_logprior_is_nig():
    y, X = SD.linreg_series(T=20)
    m = O.Model(O.LINREG, 20, y, nreg=3, X=X)
    rng = np.random.default_rng(2)
    for _ in range(5):
        th = rng.standard_normal(4)
        s2 = math.exp(th[3])
        want = (stats.invgamma.logpdf(s2, 2.0, scale=1.0) + th[3]
                + stats.norm.logpdf(th[:3], 0.0, math.sqrt(100.0 * s2)).sum())
        assert O.logprior(m, th) == pytest.approx(want, rel=1e-13)


def test_prior_draws_match_prior_distribution():
    w = SD.workload("egarch2t", T=10)
    m = O.Model.from_workload(w)
    draws = np.array([O.prior_draw(m, 9, 0, p) for p in range(3000)])
    t1 = _table1()
    assert stats.kstest(draws[:, 1], "norm", args=(math.log(0.01), 1.0)).pvalue > 1e-3
    assert stats.kstest(draws[:, 6], "norm", args=(0.0, t1["theta5_gamma"]["sd"])).pvalue > 1e-3
    assert stats.kstest(draws[:, 8], "norm", args=(math.log(10.0), 1.0)).pvalue > 1e-3
    # linreg: s2 ~ InvGamma(2, 1), beta | s2 ~ N(0, 100 s2)
    y, X = SD.linreg_series(T=5)
    ml = O.Model(O.LINREG, 5, y, nreg=3, X=X)
    d2 = np.array([O.prior_draw(ml, 9, 0, p) for p in range(3000)])
    s2 = np.exp(d2[:, 3])
    assert stats.kstest(s2, "invgamma", args=(2.0, 0, 1.0)).pvalue > 1e-3
    assert stats.kstest(d2[:, 0] / np.sqrt(100 * s2), "norm").pvalue > 1e-3


# -------------------------------------------------------------- densities ---

def test_linreg_loglik_is_gaussian_regression():
    y, X = SD.linreg_series(T=200)
    m = O.Model(O.LINREG, 200, y, nreg=3, X=X)
    th = np.array([0.9, -0.4, 0.3, math.log(0.5)])
    want = stats.norm.logpdf(y, X @ th[:3], math.sqrt(0.5)).sum()
    assert O.loglik(m, th)[0] == pytest.approx(want, rel=1e-13)
    want60 = stats.norm.logpdf(y[:60], X[:60] @ th[:3], math.sqrt(0.5)).sum()
    assert O.loglik(m, th, t=60)[0] == pytest.approx(want60, rel=1e-13)


@pytest.mark.parametrize("K,shock", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_egarch_without_volatility_dynamics_is_iid(K, shock):
    """beta_k = gamma_k = 0 leaves v = 0: returns iid with scale sigma_Y."""
    m, th, _, _ = _egarch_model(K, shock, T=300)
    th = th.copy()
    th[2 + K:2 + 2 * K] = -800.0   # beta = exp(-800) = 0
    th[2 + 2 * K:2 + 3 * K] = 0.0  # gamma = 0
    mu, sig = th[0] / 1000, math.exp(th[1])
    if shock == SD.GAUSS:
        want = stats.norm.logpdf(m.y, mu, sig).sum()
    else:
        nu = 2 + math.exp(th[2 + 3 * K])
        want = stats.t.logpdf(m.y, nu, mu, sig * math.sqrt((nu - 2) / nu)).sum()
    assert O.loglik(m, th)[0] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("K,shock", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_egarch_filter_recovers_simulated_shocks(K, shock):
    """At the parameters that generated the data the likelihood recursion
    inverts the data-generating process: eps_t equals the simulated shock and
    the log-likelihood is sum_t log f(z_t) - log h_t."""
    T = 500
    m, th, z, h = _egarch_model(K, shock, T=T)
    ll, st = O.loglik(m, th)
    assert st[K] == pytest.approx(z[-1], rel=1e-9)
    for t in (1, 2, 3, 17, 250):
        assert O.loglik(m, th, t=t)[1][K] == pytest.approx(z[t - 1], rel=1e-9, abs=1e-12)
    if shock == SD.GAUSS:
        want = (stats.norm.logpdf(z) - np.log(h)).sum()
    else:
        nu = 2 + math.exp(th[2 + 3 * K])
        sc = math.sqrt((nu - 2) / nu)
        want = (stats.t.logpdf(z, nu, 0, sc) - np.log(h)).sum()
    assert ll == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("K,shock,I", [(1, 0, 0), (2, 0, 0), (1, 1, 0), (2, 1, 0), (2, 2, 3),
                                     (1, 2, 2)])
def test_egarch_loglik_location_scale_equivariance(K, shock, I):
    """y -> a + c y with mu -> a + c mu and sigma_Y -> c sigma_Y leaves every
    standardised shock, hence the volatility recursion, unchanged, so the
    log-likelihood drops by exactly T log c (the Jacobian of the change of
    variables).  The parameters are moved well away from those that generated
    the data, so this pins the recursion where shock recovery cannot."""
    T = 300
    if shock == SD.MIXTURE:
        m, th, _, _ = _mix_model(K, I, T=T)
    else:
        m, th, _, _ = _egarch_model(K, shock, T=T)
    x = th + 0.3 * np.random.default_rng(K * 10 + shock + I).standard_normal(th.size)
    a, c = 0.37, 2.5
    y2 = a + c * m.y
    m2 = O.Model(O.EGARCH, T, y2, K=K, shock=shock, I=I) if shock == SD.MIXTURE else \
        O.Model(O.EGARCH, T, y2, K=K, shock=shock)
    x2 = x.copy()
    x2[0] = 1000.0 * a + c * x[0]   # mu = theta_0 / 1000
    x2[1] = x[1] + math.log(c)      # log sigma_Y
    base = O.loglik(m, x)[0]
    assert np.isfinite(base)
    assert O.loglik(m2, x2)[0] == pytest.approx(base - T * math.log(c), rel=1e-11)


@pytest.mark.parametrize("K,shock,I", [(1, 0, 0), (2, 0, 0), (2, 1, 0), (2, 2, 3)])
def test_egarch_loglik_reflection_symmetry(K, shock, I):
    """Reflecting the data about mu (y -> 2 mu - y) while negating the
    asymmetry coefficients gamma_k (and, for mixtures, the component
    locations) negates every standardised shock and leaves |eps|, gamma eps
    and hence the volatility path unchanged; with symmetric shock laws the
    log-likelihood is unchanged, at parameters away from the generating ones.
    Using eps where |eps| belongs (or the reverse) fails it."""
    T = 300
    if shock == SD.MIXTURE:
        m, th, _, _ = _mix_model(K, I, T=T)
    else:
        m, th, _, _ = _egarch_model(K, shock, T=T)
    x = th + 0.3 * np.random.default_rng(7 + K * 10 + shock + I).standard_normal(th.size)
    mu = x[0] / 1000.0
    y2 = 2.0 * mu - m.y
    m2 = O.Model(O.EGARCH, T, y2, K=K, shock=shock, I=I) if shock == SD.MIXTURE else \
        O.Model(O.EGARCH, T, y2, K=K, shock=shock)
    x2 = x.copy()
    x2[2 + 2 * K:2 + 3 * K] = -x[2 + 2 * K:2 + 3 * K]   # gamma_k
    if shock == SD.MIXTURE:
        b = 2 + 3 * K
        x2[b + I:b + 2 * I] = -x[b + I:b + 2 * I]         # component locations
    base = O.loglik(m, x)[0]
    assert np.isfinite(base)
    assert O.loglik(m2, x2)[0] == pytest.approx(base, rel=1e-11)


def test_egarch_factors_are_exchangeable():
    m, th, _, _ = _egarch_model(2, 1, T=400)
    sw = th.copy()
    for base in (2, 4, 6):
        sw[base], sw[base + 1] = th[base + 1], th[base]
    assert O.loglik(m, sw)[0] == pytest.approx(O.loglik(m, th)[0], rel=1e-13)
    assert O.logprior(m, sw) == pytest.approx(O.logprior(m, th), rel=1e-13)


@pytest.mark.parametrize("name", ["linreg", "egarch11", "egarch2t", "egarch23"])
def test_loglik_splits_over_dates(name):
    w = SD.workload(name, T=300)
    m = O.Model.from_workload(w)
    th = SD.random_thetas(w, 1, 3)[0]
    full, st_full = O.loglik(m, th)
    a, st = O.loglik(m, th, t=123)
    b, st2 = O.loglik(m, th, t=300, state=st if m.S else None, t0=123)
    assert a + b == pytest.approx(full, rel=1e-13)
    if m.S:
        assert np.allclose(st2, st_full, rtol=1e-14, atol=0)


# -------------------------------------------------------------- gradients ---

@pytest.mark.parametrize("name", ["linreg", "egarch11", "egarch2t", "egarch23", "egarch44"])
def test_gradient_matches_central_differences(name):
    w = SD.workload(name, T=250)
    m = O.Model.from_workload(w)
    rng = np.random.default_rng(4)
    for th in SD.random_thetas(w, 3, 7):
        ll, g = O.loglik_grad(m, th)
        assert ll == pytest.approx(O.loglik(m, th)[0], rel=1e-13)
        lp, gp = O.logprior_grad(m, th)
        assert lp == pytest.approx(O.logprior(m, th), rel=1e-13)
        for i in range(th.size):
            e = np.zeros_like(th)
            e[i] = 1e-5
            fd = (O.loglik(m, th + e)[0] - O.loglik(m, th - e)[0]) / 2e-5
            assert g[i] == pytest.approx(fd, rel=2e-6, abs=1e-4 * (1 + abs(fd)) * 1e-2)
            fdp = (O.logprior(m, th + e) - O.logprior(m, th - e)) / 2e-5
            assert gp[i] == pytest.approx(fdp, rel=1e-6, abs=1e-7)
    del rng


def test_linreg_gradient_closed_form():
    y, X = SD.linreg_series(T=200)
    m = O.Model(O.LINREG, 200, y, nreg=3, X=X)
    th = np.array([0.9, -0.4, 0.3, math.log(0.5)])
    _, g = O.loglik_grad(m, th)
    r = y - X @ th[:3]
    s2 = math.exp(th[3])
    assert np.allclose(g[:3], X.T @ r / s2, rtol=1e-12)
    assert g[3] == pytest.approx(-len(y) / 2 + (r @ r) / (2 * s2), rel=1e-12)


# -------------------------------------------------- normal-mixture shocks ---
# egarch_KI (Section 5.1): eq normal_mixture with the transforms of eqs
# EGARCH_tran1/2 and Table 1's theta_6..8 priors.

MIX = [(1, 2), (2, 3), (3, 4), (4, 4)]


def _mix_model(K, I, T=400, seed=5):
    th = SD.egarch_mixture_truth(K, I)
    y, z, h = SD.egarch_series(th, T, K, SD.MIXTURE, seed, return_path=True)
    return O.Model(O.EGARCH, T, y, K=K, shock=O.MIXTURE, I=I), th, z, h


def _mix_pdf(x, p, mu, sg):
    return sum(p[i] * stats.norm.pdf(x, mu[i], sg[i]) for i in range(len(p)))


@pytest.mark.parametrize("K,I", MIX)
def test_mixture_logprior_is_table1_with_truncation(K, I):
    """Table 1: all Gaussian, theta_8i truncated below at -3 (scipy's
    truncnorm carries the normalising constant)."""
    t1 = _table1()
    m, th, _, _ = _mix_model(K, I, T=10)
    means = ([t1["theta1_mu"]["mean"], math.log(t1["theta2_sigma"]["mean_log_of"])]
             + [math.atanh(t1["theta3_alpha"]["mean_atanh_of"])] * K
             + [math.log(t1["theta4_beta"]["mean_log_of"])] * K
             + [t1["theta5_gamma"]["mean"]] * K
             + [t1["theta6_p"]["mean"]] * I + [t1["theta7_mu"]["mean"]] * I)
    sds = ([t1["theta1_mu"]["sd"], t1["theta2_sigma"]["sd"]] + [t1["theta3_alpha"]["sd"]] * K
           + [t1["theta4_beta"]["sd"]] * K + [t1["theta5_gamma"]["sd"]] * K
           + [t1["theta6_p"]["sd"]] * I + [t1["theta7_mu"]["sd"]] * I)
    lo = t1["theta8_sigma"]["truncated_below"]
    rng = np.random.default_rng(K * 10 + I)
    n8 = 2 + 3 * K + 2 * I
    for _ in range(6):
        x = th + rng.standard_normal(th.size)
        x[n8:] = np.maximum(x[n8:], lo + 0.01)
        want = (stats.norm.logpdf(x[:n8], means, sds).sum()
                + stats.truncnorm.logpdf(x[n8:], lo, np.inf).sum())
        assert O.logprior(m, x) == pytest.approx(want, rel=1e-13, abs=1e-12)
    x = th.copy()
    x[n8 + I - 1] = lo - 1e-9
    assert O.logprior(m, x) == -math.inf


def test_mixture_prior_draws_respect_truncation():
    w = SD.workload("egarch23", T=10)
    m = O.Model.from_workload(w)
    draws = np.array([O.prior_draw(m, 4, 0, p) for p in range(4000)])
    n8 = 2 + 3 * 2 + 2 * 3
    assert draws[:, n8:].min() >= -3.0
    for i in range(3):
        assert stats.kstest(draws[:, n8 + i], stats.truncnorm(-3.0, np.inf).cdf).pvalue > 1e-3
        assert stats.kstest(draws[:, 2 + 6 + i], "norm").pvalue > 1e-3
    assert np.all(np.isfinite([O.logprior(m, d) for d in draws[:200]]))


@pytest.mark.parametrize("K,I", MIX)
def test_mixture_filter_recovers_simulated_shocks(K, I):
    """At the generating parameters (given in normalised form) eps_t is the
    simulated shock and log p = sum_t log f(z_t) - log h_t with f the mixture
    density evaluated by scipy."""
    T = 400
    m, th, z, h = _mix_model(K, I, T=T)
    p, mu, sg = SD.mixture_truth(I)
    ll, st = O.loglik(m, th)
    assert st[K] == pytest.approx(z[-1], rel=1e-9)
    want = (np.log(_mix_pdf(z, p, mu, sg)) - np.log(h)).sum()
    assert ll == pytest.approx(want, rel=1e-11)


def test_mixture_transforms_satisfy_normalisation():
    """eq EGARCH_normalization at arbitrary theta: mean 0, variance 1."""
    m, th, _, _ = _mix_model(2, 4, T=10)
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = th + rng.standard_normal(th.size)
        p, mu, sg = O.mixture_params(m, x)
        assert np.all(p > 0) and np.all(sg > 0)
        assert p.sum() == pytest.approx(1.0, abs=1e-14)
        assert (p * mu).sum() == pytest.approx(0.0, abs=1e-14)
        assert (p * (mu ** 2 + sg ** 2)).sum() == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("K,I", [(1, 2), (2, 3)])
def test_mixture_conditional_density_by_quadrature(K, I):
    """p(y_t | y_{1:t-1}, theta) at generic theta, as a function of y_t:
    integrates to one, has mean mu_Y, variance h_t^2 and third central
    moment h_t^3 sum p_i (mu_i^3 + 3 mu_i sigma_i^2)."""
    T = 60
    m, th, _, _ = _mix_model(K, I, T=T)
    x = th + 0.4 * np.random.default_rng(9).standard_normal(th.size)
    ll_prev, st = O.loglik(m, x, t=T - 1)
    vs = st[:K]
    eprev = st[K]
    alpha = np.tanh(x[2:2 + K])
    beta = np.exp(x[2 + K:2 + 2 * K])
    gamma = x[2 + 2 * K:2 + 3 * K]
    v = alpha * vs + beta * (abs(eprev) - math.sqrt(2 / math.pi)) + gamma * eprev
    h = math.exp(x[1]) * math.exp(0.5 * v.sum())
    muY = x[0] / 1000
    grid = muY + h * np.linspace(-14, 14, 8001)
    dens = []
    for yv in grid:
        y2 = m.y.copy()
        y2[T - 1] = yv
        mm = O.Model(O.EGARCH, T, y2, K=K, shock=O.MIXTURE, I=I)
        dens.append(math.exp(O.loglik(mm, x)[0] - ll_prev))
    dens = np.array(dens)
    mass = np.trapezoid(dens, grid)
    mean = np.trapezoid(grid * dens, grid)
    var = np.trapezoid((grid - muY) ** 2 * dens, grid)
    m3 = np.trapezoid((grid - muY) ** 3 * dens, grid)
    p, mu, sg = O.mixture_params(m, x)
    assert mass == pytest.approx(1.0, abs=1e-9)
    assert mean == pytest.approx(muY, abs=1e-9 * h)
    assert var == pytest.approx(h * h, rel=1e-8)
    assert m3 == pytest.approx(h ** 3 * (p * (mu ** 3 + 3 * mu * sg ** 2)).sum(), rel=1e-6, abs=1e-9 * h ** 3)


def test_mixture_with_equal_components_is_gaussian():
    """Identical components collapse to a standard normal shock: the
    likelihood equals the Gaussian-shock model's."""
    K, I = 2, 3
    m, th, _, _ = _mix_model(K, I, T=300)
    x = th.copy()
    b = 2 + 3 * K
    x[b:b + I] = 0.3
    x[b + I:b + 2 * I] = -0.7
    x[b + 2 * I:] = 0.2
    mg = O.Model(O.EGARCH, 300, m.y, K=K, shock=O.GAUSS)
    assert O.loglik(m, x)[0] == pytest.approx(O.loglik(mg, x[:b])[0], rel=1e-12)


def test_mixture_location_scale_and_label_invariance():
    """The normalisation removes the location and scale of (mu*, sigma*),
    and components are exchangeable (the label-switching symmetry of
    Section 5.1)."""
    K, I = 2, 3
    m, th, _, _ = _mix_model(K, I, T=300)
    x = th + 0.3 * np.random.default_rng(4).standard_normal(th.size)
    b = 2 + 3 * K
    base = O.loglik(m, x)[0]
    sh = x.copy()
    sh[b + I:b + 2 * I] += 0.37
    assert O.loglik(m, sh)[0] == pytest.approx(base, rel=1e-12)
    sc = x.copy()
    sc[b + I:b + 2 * I] *= 1.6
    sc[b + 2 * I:] += math.log(1.6)
    assert O.loglik(m, sc)[0] == pytest.approx(base, rel=1e-12)
    perm = [2, 0, 1]
    pm = x.copy()
    for r in range(3):
        pm[b + r * I:b + (r + 1) * I] = x[b + r * I:b + (r + 1) * I][perm]
    assert O.loglik(m, pm)[0] == pytest.approx(base, rel=1e-12)
