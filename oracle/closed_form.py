"""Closed forms for the conjugate Gaussian regression workload (test oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Model: y = X beta + e, e ~ N(0, s2 I_T); prior beta | s2 ~ N(0, c0 s2 I_k),
s2 ~ InvGamma(a0, b0) with (a0, b0, c0) = (2, 1, 100), so that the prior
variance of beta is c0 E[s2] = 100 = 10^2.  Normal-inverse-gamma updating:

    V_T = (I/c0 + X'X)^-1,  m_T = V_T X'y,  a_T = a0 + T/2,
    b_T = b0 + (y'y - m_T' V_T^-1 m_T) / 2,
    log p(y) = -T/2 log 2pi + 1/2 log|V_T| - k/2 log c0 + a0 log b0
               - a_T log b_T + lgamma(a_T) - lgamma(a0).

The predictive likelihood of a block y_{t+1:s} given y_{1:t} is the ratio of
two marginal likelihoods (the decomposition used in Section 4.2's proof).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import digamma, gammaln

A0, B0, C0 = 2.0, 1.0, 100.0


def nig_posterior(y, X):
    y = np.asarray(y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    T, k = X.shape
    prec = np.eye(k) / C0 + X.T @ X
    V = np.linalg.inv(prec)
    m = V @ (X.T @ y)
    aT = A0 + T / 2.0
    bT = B0 + 0.5 * (y @ y - m @ prec @ m)
    return m, V, aT, bT


def log_ml(y, X):
    """log p(y_{1:T}) under the NIG prior (0.0 for T = 0)."""
    y = np.asarray(y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    T, k = X.shape
    if T == 0:
        return 0.0
    m, V, aT, bT = nig_posterior(y, X)
    _, logdetV = np.linalg.slogdet(V)
    return (-0.5 * T * math.log(2.0 * math.pi) + 0.5 * logdetV - 0.5 * k * math.log(C0)
            + A0 * math.log(B0) - aT * math.log(bT) + gammaln(aT) - gammaln(A0))


def log_predictive(y, X, t, s):
    """log p(y_{t+1:s} | y_{1:t})."""
    return log_ml(y[:s], X[:s]) - log_ml(y[:t], X[:t])


def posterior_means(y, X):
    """E[beta | y], E[s2 | y], E[log s2 | y]."""
    m, V, aT, bT = nig_posterior(y, X)
    return m, bT / (aT - 1.0), math.log(bT) - digamma(aT)


def posterior_draws(y, X, n, rng):
    """Exact posterior draws in the sampler's coordinates (beta, log s2), [n, k+1]."""
    m, V, aT, bT = nig_posterior(y, X)
    s2 = bT / rng.gamma(aT, 1.0, size=n)
    L = np.linalg.cholesky(V)
    z = rng.standard_normal((n, m.size))
    beta = m[None, :] + np.sqrt(s2)[:, None] * (z @ L.T)
    return np.column_stack([beta, np.log(s2)])
