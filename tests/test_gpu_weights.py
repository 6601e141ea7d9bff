"""The weight sums of the C phase as compiled: the pooled RSS of a weight
column (k_rss_cols for columns up to 16,384 particles, k_rss_slices and
k_rss_merge beyond), the adaptive path's RSS from the scan's per-wave sums
(k_cscan, k_rss_scan) and the group log mean weights (k_group_logwbar) on
crafted log-weight columns, against long double sums of the same values.

The columns come from one observation of a one-regressor Gaussian
regression: a particle with slope b and log variance 0 has log weight
-log(2 pi)/2 - r^2/2, r = y_1 - x_1 b, so choosing r places each weight
where wanted; a log variance of +inf gives a zero weight (log weight -inf).
The patterns put the arguments of the weights' exponentials, w - max w,
across [-1100, 0] (equal weights, one survivor, geometric ladders with
steps 0.01 to 2.2, uniform draws, a group entirely below -700 relative to
the pooled maximum) with dead particles mixed in.  Each exponential carries
at most 2 ulp of error, so the sums agree with long double to a few ulp
per term; a wrong polynomial, reduction or clamp does not.
"""
import math

import numpy as np
import pytest
import torch

import paper_1304_4334_amd as S
import synthdata as SD

pytestmark = pytest.mark.gpu


def _patterns(N, rng):
    k = np.arange(N, dtype=np.float64)
    dead = np.full(N, np.nan)
    one = dead.copy()
    one[N // 3] = 0.0
    half = k * 0.05
    half[::2] = np.nan
    return [np.zeros(N), one, k * 0.01, k * 0.5, k * 2.2, rng.uniform(0.0, 1100.0, N), half,
            700.0 + k * 0.001]


def _population(m, J, N, depth):
    """depth[P]: wanted -log weight above the best (NaN: a dead particle)."""
    y1, x1 = float(m.y[0].item()), float(m.X[0, 0].item())
    P = J * N
    r = np.sqrt(2.0 * np.nan_to_num(depth, nan=0.0))
    beta = (y1 - r) / x1
    eta = np.where(np.isnan(depth), np.inf, 0.0)
    g = S.Population(m, J, N, max_chunk=16)
    g.theta.copy_(torch.from_numpy(np.stack([beta, eta])))
    return g


def _ld_rss(lw):
    lw = lw.astype(np.longdouble)
    m = lw.max()
    e = np.exp(lw - m)
    return (e.sum() ** 2) / (len(lw) * (e * e).sum())


def _ld_lmw(lw):
    lw = lw.astype(np.longdouble)
    m = lw.max()
    if not np.isfinite(m):
        return -np.inf
    return m + np.log(np.exp(lw - m).sum() / len(lw))


@pytest.mark.parametrize("J,N", [(8, 512), (2, 16384), (4, 12288)])
def test_weight_sums_match_long_double(J, N):
    y, X = SD.linreg_series(T=4, k=1, beta=(1.0,))
    m = S.Model(S.SMC_MODEL_LINREG, y, X=X)
    rng = np.random.default_rng(J * N)
    pats = _patterns(N, rng)
    depth = np.concatenate([pats[(3 * j + J) % len(pats)] for j in range(J)])
    g = _population(m, J, N, depth)
    print(f"[weights] J={J} N={N}", flush=True)
    _, rss, glw = S.smc_correct(m, g, 0, 1, check_every=1, rss_min=0.0)
    lw = g.logw.cpu().numpy()
    assert np.isneginf(lw[np.isnan(depth)]).all()
    want = float(_ld_rss(lw))
    # 2 ulp per exponential plus the rounding of two sums reduced in a tree
    tol = (4 + 3 * math.log2(N * J)) * 4 * 2.0 ** -52
    print(f"[weights] RSS {rss!r} vs {want!r}: rel {abs(rss - want) / want:.2e} (bar {tol:.1e})")
    assert abs(rss - want) <= tol * want, (rss, want)
    got = glw.cpu().numpy()
    for j in range(J):
        ref = float(_ld_lmw(lw[j * N:(j + 1) * N]))
        if math.isinf(ref):
            assert got[j] == ref
        else:
            assert abs(got[j] - ref) <= 1e-13 + 4e-16 * abs(ref), (j, got[j], ref)
    # the adaptive path's RSS (per-wave sums in the scan, merged) agrees
    g2 = _population(m, J, N, depth)
    t, rss2, _ = S.smc_correct(m, g2, 0, 1, check_every=1, rss_min=0.5)
    assert t == 1 and rss2 == pytest.approx(want, rel=tol)


def test_equal_and_single_weights_are_exact():
    y, X = SD.linreg_series(T=4, k=1, beta=(1.0,))
    m = S.Model(S.SMC_MODEL_LINREG, y, X=X)
    J, N = 4, 256
    depth = np.zeros(J * N)
    g = _population(m, J, N, depth)
    _, rss, glw = S.smc_correct(m, g, 0, 1, check_every=1, rss_min=0.0)
    assert rss == 1.0
    lw0 = g.logw.cpu().numpy()[0]
    assert np.all(glw.cpu().numpy() == lw0)
    depth = np.full(J * N, np.nan)
    depth[[5, 300, 700, 1000]] = 0.0  # one survivor in each group
    g = _population(m, J, N, depth)
    _, rss, glw = S.smc_correct(m, g, 0, 1, check_every=1, rss_min=0.0)
    assert rss == pytest.approx(1.0 / N, rel=1e-15)
    assert np.allclose(glw.cpu().numpy(), lw0 - math.log(N), rtol=0, atol=1e-14)
