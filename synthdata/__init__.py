"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only *generates data*: it simulates the data-generating process of
each model forward (draw shocks, build the series) and lists the workload
shapes.  It evaluates no density, weight, resampling rule or Metropolis step,
so neither the HIP path nor the oracle depends on the other through it.

Workloads (the paper's application uses daily index returns, T = 5,100, with
2^16 particles in 2^6 groups of 2^10, Section 5.1-5.2; that series is not
available here, so seeded synthetic series of the same scalar layout stand in
for it):

* ``linreg``      Gaussian linear regression, k = 3 N(0,1) regressors,
                  beta = (1, -0.5, 0.25), sigma = 0.8, T = 200,
                  J = 4 x N = 256, data entering in blocks of 20.
* ``egarch11``    EGARCH with K = 1 factor and Gaussian shocks, T = 5,000,
                  J = 16 x N = 1,024 (Nelson-form truth mapped to Table 1's
                  parameterisation, see ``EGARCH11_TRUTH``).
* ``egarch2t``    EGARCH with K = 2 factors and standardised Student-t(8)
                  shocks, T = 10,000, J = 64 x N = 1,024.
* ``egarch23``    EGARCH with K = 2 factors and a 3-component normal-mixture
                  shock (the paper's featured specification), T = 5,100,
                  J = 64 x N = 1,024.  Other ``egarchKI`` names (K in 1..4,
                  I in 2..4) give the rest of the family at that size.
* ``batched``     32 independent runs mixing the two EGARCH forms with
                  T in [1,000, 20,000] and J*N in {4096 ... 65536}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DATA_SEED_BASE = 20130406

# Model kinds / shock kinds (mirrors the C-ABI enums by value, not by import).
LINREG = 1
EGARCH = 2
GAUSS = 0
STUDENT_T = 1
MIXTURE = 2

# Nelson (1991) form of the EGARCH(1,1) truth: log s2_t = omega + b log s2_{t-1}
#   + a (|z| - sqrt(2/pi)) + g z.  In the paper's form (EGARCH_mod1/2) the
# persistence is alpha_1 = b, the magnitude loading beta_1 = a, gamma_1 = g,
# mu_Y = mu and sigma_Y = exp(omega / (2 (1 - b))) (the unconditional level of
# the log variance folded into sigma_Y, so the factor has mean zero).
NELSON11 = dict(omega=-0.1, a=0.1, g=-0.05, b=0.97, mu=0.0003)


def egarch11_truth() -> np.ndarray:
    """theta_true for EGARCH(1,1)-N in Table 1's transformed coordinates."""
    n = NELSON11
    return np.array([
        n["mu"] * 1000.0,                      # theta_1: mu_Y = theta_1 / 1000
        n["omega"] / (2.0 * (1.0 - n["b"])),   # theta_2: sigma_Y = exp(theta_2)
        math.atanh(n["b"]),                    # theta_3: alpha = tanh(theta_3)
        math.log(n["a"]),                      # theta_4: beta = exp(theta_4)
        n["g"],                                # theta_5: gamma = theta_5
    ])


def egarch2t_truth() -> np.ndarray:
    """theta_true for EGARCH(2)-t: (th1, th2, th3_1, th3_2, th4_1, th4_2,
    th5_1, th5_2, th9 = log(nu - 2))."""
    return np.array([
        0.3, math.log(0.01),
        math.atanh(0.98), math.atanh(0.80),
        math.log(0.08), math.log(0.15),
        -0.04, -0.08,
        math.log(8.0 - 2.0),
    ])


# Mixture truth for the egarchKI workloads: a fat-tailed, slightly
# left-skewed shock built from I components, given directly in the
# normalised form (weights, means, scales with mean 0 and variance 1) and in
# Table 1's coordinates theta_6..8 with sum p* = 1 (th6 = atanh(p - 1)), sum
# p mu* = 0 (so mu** = mu*) and c = 1 (sum p (mu^2 + s^2) = 1).
def mixture_truth(I: int):
    if I == 2:
        p = np.array([0.85, 0.15])
        mu = np.array([0.06, -0.34])
    elif I == 3:
        p = np.array([0.6, 0.3, 0.1])
        mu = np.array([0.08, 0.02, -0.54])
    else:
        p = np.array([0.5, 0.25, 0.15, 0.1])
        mu = np.array([0.1, -0.02, 0.05, -0.525])
    mu = mu - (p * mu).sum()
    s_raw = np.linspace(0.7, 1.9, I)
    scale = math.sqrt((1.0 - (p * mu ** 2).sum()) / (p * s_raw ** 2).sum())
    sg = s_raw * scale
    return p, mu, sg


def egarch_mixture_truth(K: int, I: int) -> np.ndarray:
    """theta_true for egarchKI: the K-factor part from the 2-factor truth
    (factors beyond 2 get weaker persistence), then th6_i = atanh(p_i - 1),
    th7_i = mu_i, th8_i = log sigma_i for the normalised mixture above."""
    alphas = [0.98, 0.80, 0.6, 0.4][:K]
    betas = [0.08, 0.15, 0.1, 0.1][:K]
    gammas = [-0.04, -0.08, -0.02, -0.02][:K]
    p, mu, sg = mixture_truth(I)
    return np.concatenate([[0.3, math.log(0.01)], np.arctanh(alphas), np.log(betas), gammas,
                           np.arctanh(p - 1.0), mu, np.log(sg)])


def linreg_series(T: int = 200, k: int = 3, beta=(1.0, -0.5, 0.25),
                  sigma: float = 0.8, seed: int = DATA_SEED_BASE + 1):
    """y = X beta + sigma * eps with X, eps iid N(0, 1).  Returns (y[T], X[T,k])."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((T, k))
    eps = rng.standard_normal(T)
    y = X @ np.asarray(beta, dtype=np.float64) + sigma * eps
    return np.ascontiguousarray(y), np.ascontiguousarray(X)


def egarch_series(theta: np.ndarray, T: int, K: int, shock: int,
                  seed: int, return_path: bool = False):
    """Simulate the EGARCH data-generating process of eqs EGARCH_mod1/2.

    Factor states start at zero and take no innovation at t = 1 (so the
    first return has scale sigma_Y); from t = 2 on each factor follows
    v_kt = alpha_k v_k,t-1 + beta_k (|z_{t-1}| - sqrt(2/pi)) + gamma_k z_{t-1}.
    Shocks are N(0,1), Student-t(nu) rescaled to unit variance, or (for the
    mixture, whose truth is given with mean 0 and variance 1 already) a
    draw from component i with probability p_i.
    With ``return_path`` the shocks z and scales h are returned too.
    """
    theta = np.asarray(theta, dtype=np.float64)
    mu = theta[0] / 1000.0
    sig = math.exp(theta[1])
    alpha = np.tanh(theta[2:2 + K])
    beta = np.exp(theta[2 + K:2 + 2 * K])
    gamma = theta[2 + 2 * K:2 + 3 * K]
    rng = np.random.default_rng(seed)
    if shock == GAUSS:
        z = rng.standard_normal(T)
    elif shock == MIXTURE:
        I = (theta.size - 2 - 3 * K) // 3
        b = 2 + 3 * K
        p = np.tanh(theta[b:b + I]) + 1.0
        p = p / p.sum()
        comp = rng.choice(I, size=T, p=p)
        z = theta[b + I + comp] + np.exp(theta[b + 2 * I + comp]) * rng.standard_normal(T)
    else:
        nu = 2.0 + math.exp(theta[2 + 3 * K])
        z = rng.standard_t(nu, T) * math.sqrt((nu - 2.0) / nu)
    c = math.sqrt(2.0 / math.pi)
    v = np.zeros(K)
    y = np.empty(T)
    h = np.empty(T)
    for t in range(T):
        if t > 0:
            zp = z[t - 1]
            v = alpha * v + beta * (abs(zp) - c) + gamma * zp
        h[t] = sig * math.exp(0.5 * float(v.sum()))
        y[t] = mu + h[t] * z[t]
    if return_path:
        return y, z, h
    return y


@dataclass
class Workload:
    name: str
    kind: int
    K: int = 0
    shock: int = GAUSS
    nreg: int = 0
    T: int = 0
    J: int = 0
    N: int = 0
    check_every: int = 1
    I: int = 0
    y: np.ndarray = field(default=None, repr=False)
    X: np.ndarray = field(default=None, repr=False)
    theta_true: np.ndarray = field(default=None, repr=False)

    @property
    def P(self) -> int:
        return self.J * self.N

    @property
    def d(self) -> int:
        if self.kind == LINREG:
            return self.nreg + 1
        if self.shock == MIXTURE:
            return 2 + 3 * self.K + 3 * self.I
        return 2 + 3 * self.K + (1 if self.shock == STUDENT_T else 0)


def workload(name: str, T: int | None = None, J: int | None = None,
             N: int | None = None, seed_offset: int = 0) -> Workload:
    """Named workload at its full size, or shrunk via T/J/N overrides."""
    if name == "linreg":
        T = T or 200
        y, X = linreg_series(T=T, seed=DATA_SEED_BASE + 1 + seed_offset)
        return Workload(name, LINREG, nreg=3, T=T, J=J or 4, N=N or 256,
                        check_every=20, y=y, X=X)
    if name == "egarch11":
        T = T or 5000
        th = egarch11_truth()
        y = egarch_series(th, T, 1, GAUSS, DATA_SEED_BASE + 2 + seed_offset)
        return Workload(name, EGARCH, K=1, shock=GAUSS, T=T, J=J or 16,
                        N=N or 1024, y=y, theta_true=th)
    if name == "egarch2t":
        T = T or 10000
        th = egarch2t_truth()
        y = egarch_series(th, T, 2, STUDENT_T, DATA_SEED_BASE + 3 + seed_offset)
        return Workload(name, EGARCH, K=2, shock=STUDENT_T, T=T, J=J or 64,
                        N=N or 1024, y=y, theta_true=th)
    if len(name) == 8 and name.startswith("egarch") and name[6:].isdigit():
        K, I = int(name[6]), int(name[7])
        if 1 <= K <= 4 and 2 <= I <= 4:
            T = T or 5100
            th = egarch_mixture_truth(K, I)
            y = egarch_series(th, T, K, MIXTURE, DATA_SEED_BASE + 10 * K + I + seed_offset)
            return Workload(name, EGARCH, K=K, shock=MIXTURE, I=I, T=T, J=J or 64,
                            N=N or 1024, y=y, theta_true=th)
    raise KeyError(name)


def batched_specs(n_runs: int = 32, seed: int = DATA_SEED_BASE + 5):
    """Run list for the batched workload: model alternates EGARCH(1,1)-N and
    EGARCH(2)-t, T_r uniform on {1000..20000}, J = 16, N_r = 2^(8 + r mod 5)
    (so J*N_r runs over 4096 ... 65536)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_runs):
        T = int(rng.integers(1000, 20001))
        N = 2 ** (8 + (r % 5))
        if r % 2 == 0:
            th = egarch11_truth()
            y = egarch_series(th, T, 1, GAUSS, seed + 100 + r)
            out.append(Workload(f"run{r}", EGARCH, K=1, shock=GAUSS, T=T, J=16,
                                N=N, y=y, theta_true=th))
        else:
            th = egarch2t_truth()
            y = egarch_series(th, T, 2, STUDENT_T, seed + 100 + r)
            out.append(Workload(f"run{r}", EGARCH, K=2, shock=STUDENT_T, T=T,
                                J=16, N=N, y=y, theta_true=th))
    return out


def random_thetas(w: Workload, P: int, seed: int, spread: float = 0.05) -> np.ndarray:
    """Parameter draws near the truth (or near zero for linreg), [P, d].
    Used to exercise the likelihood at plausible points."""
    rng = np.random.default_rng(seed)
    if w.theta_true is not None:
        base = w.theta_true
    else:
        base = np.array([1.0, -0.5, 0.25, math.log(0.64)])
    return base[None, :] + spread * rng.standard_normal((P, base.size))
