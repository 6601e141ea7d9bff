"""GPU parity of the simulator's reported outputs against the oracle: the
functions of interest and their posterior moments with NSE and RNE
(Sections 2.3, 5.2; the loss probability for every shock), the RNE stopping
rule with E2 at dates of interest (Section 3.3) and the log score over a
burn-in (Section 4.2).

Tolerances: moments 1e-9 relative (FP64 everywhere; the loss probability
goes through erfc, or the t's continued fraction, on both sides); adaptive decisions (cycle ends and M-phase
lengths) exact; log scores 1e-10 relative on a replayed design and within
3.5 NSE of the regression's closed form.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1304_4334_amd as S
import synthdata as SD
from oracle import closed_form as CF
from tests.gpu_helpers import gpu_model, ora_model, pop_to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,which", [("egarch11", 1), ("egarch23", 1), ("egarch2t", 1),
                                        ("linreg", 1), ("egarch23", 0), ("egarch34", 1)])
def test_test_moments_match_oracle(name, which):
    w = SD.workload(name, T=120)
    gm, om = gpu_model(w), ora_model(w)
    J, N = 8, 128
    opop = O.Pop(om, J, N)
    opop.theta[:] = SD.random_thetas(w, J * N, 4, spread=0.05)
    t = 97
    _, st = O.loglik_batch(om, opop.theta, t)
    if om.S:
        opop.state[:, :om.S] = st
    want = O.test_report(om, opop, t, which)
    g = pop_to_gpu(gm, opop)
    got = S.smc_test_moments(gm, g, t, which).cpu().numpy()
    assert got.shape == want.shape == (S.smc_num_test_functions(gm, which), 4)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-14), (got, want)


@pytest.mark.parametrize("nu", [2.05, 3.0, 12.0, 200.0, 1e4])
def test_student_t_loss_probability_matches_oracle(nu):
    """g3 with Student-t shocks against the oracle's, case by case: each
    (nu, x) is a population of identical particles at t = 0 with sigma_Y = 1,
    so g3's argument is x and the population mean is the particle's value.
    Both tails, the centre and x = 0, nu from near 2 to far beyond the
    prior's reach.  Both sides sum the same continued fraction to full
    precision, each with its own log-gamma: 1e-12 relative, and 1e-10 at
    nu = 1e4, where the oracle's difference of log-gamma values near 4e4
    cancels to about 1e-11."""
    w = SD.workload("egarch2t", T=50)
    gm, om = gpu_model(w), ora_model(w)
    th = w.theta_true.copy()
    th[1] = 0.0
    th[2 + 3 * w.K] = np.log(nu - 2.0)
    rel = 1e-12 if nu < 1000 else 1e-10
    for x in (-np.inf, -80.0, -6.0, -1.5, -0.2, 0.0, 1e-3, 0.7, 3.0, 50.0, np.inf):
        th[0] = -1000.0 * (x + 0.03)
        opop = O.Pop(om, 2, 64)
        opop.theta[:] = th
        want = O.test_fns(om, th, np.zeros(om.S), 0)
        got = S.smc_test_moments(gm, pop_to_gpu(gm, opop), 0, S.SMC_TEST_MODEL).cpu().numpy()
        assert got[0, 0] == want[0], x
        assert got[1, 0] == pytest.approx(want[1], rel=rel, abs=1e-300), (x, got[1, 0], want[1])
        assert got[1, 1] <= 1e-12 * max(want[1], 1e-300), x  # identical particles
    assert want[1] == 1.0  # the last case, x = +inf


@pytest.mark.parametrize("name", ["egarch23", "egarch2t"])
def test_rne_rule_with_e2_matches_oracle_run(name):
    """Adaptive run with the RNE rule over the model's functions of interest
    (for Student-t shocks g1 and the t loss probability), dates of interest
    every 40 observations: the same cycle ends, M-phase lengths, reports and
    log-ML as the oracle's run."""
    w = SD.workload(name, T=120)
    gm, om = gpu_model(w), ora_model(w)
    J, N = 8, 64
    rc, orec, _ = O.run(om, J, N, 3, check_every=1, force_every=40, stop_rule=1, E1=0.2, E2=0.6,
                        Rmax=30, test_fn=O.TEST_MODEL, moments=True, Lmax=300, RmaxRec=64)
    assert rc == 0
    so = orec.summary()
    g = S.Population(gm, J, N, max_chunk=32)
    rec = S.Record(gm, J, Lmax=300, RmaxRec=64, test_fn=S.SMC_TEST_MODEL)
    S.smc_run(gm, g, seed=3, check_every=1, force_every=40, stop_rule=1, E1=0.2, E2=0.6, Rmax=30,
              test_fn=S.SMC_TEST_MODEL, record=rec)
    sg = rec.summary()
    assert np.array_equal(sg["t_end"], so["t_end"])
    assert np.array_equal(sg["R"], so["R"])
    assert np.allclose(sg["moments"], so["moments"], rtol=1e-8, atol=1e-12)
    assert sg["log_ml"] == pytest.approx(so["log_ml"], rel=1e-9)


def test_log_score_replay_matches_oracle_and_closed_form():
    w = SD.workload("linreg")
    gm, om = gpu_model(w), ora_model(w)
    exact = CF.log_predictive(w.y, w.X, 100, w.T)
    rc, orec, _ = O.run(om, 16, 256, 2, check_every=1, burn_in=100, Lmax=300, RmaxRec=64)
    assert rc == 0
    so = orec.summary()
    L = orec.L
    g = S.Population(gm, 16, 256, max_chunk=32)
    rec = S.Record(gm, 16, Lmax=300, RmaxRec=64, test_fn=S.SMC_TEST_PARAMS)
    rec.t_end[:L] = orec.t_end[:L]
    rec.R[:L] = orec.R[:L]
    rec.hchol[:L].copy_(torch.from_numpy(orec.hchol[:L].copy()))
    S.smc_run(gm, g, seed=2, check_every=1, burn_in=100, record=rec, replay=True)
    ls = rec.summary()["log_score"]
    assert ls[0] == pytest.approx(so["log_score"], rel=1e-10)
    assert ls[1] == pytest.approx(so["log_score_nse"], rel=1e-7)
    # and an adaptive GPU run against the closed form
    rec2 = S.Record(gm, 16, Lmax=300, RmaxRec=64, test_fn=S.SMC_TEST_PARAMS)
    g2 = S.Population(gm, 16, 256, max_chunk=32)
    S.smc_run(gm, g2, seed=5, check_every=1, burn_in=100, record=rec2)
    s2 = rec2.summary()
    assert 100 in s2["t_end"].tolist()
    assert abs(s2["log_score"][0] - exact) < 3.5 * s2["log_score"][1]
    # the standalone call agrees with the driver's
    ls3 = S.smc_log_score(rec2.group_logwbar[:rec2.L], rec2.t_end, 100).cpu().numpy()
    assert np.allclose(ls3, s2["log_score"], rtol=1e-14)


@pytest.mark.parametrize("name,T,J,N", [("linreg", 200, 4, 256), ("egarch11", 300, 4, 128)])
def test_hybrid_matches_oracle_hybrid(name, T, J, N):
    """Algorithm 3 on the GPU (adaptive step, then its design replayed with a
    new key) against the oracle's two steps with the same keys."""
    w = SD.workload(name, T=T)
    gm, om = gpu_model(w), ora_model(w)
    fe = 20 if name == "linreg" else 0
    rc, o1, o2, opop = O.run_hybrid(om, J, N, 21, 22, check_every=1, force_every=fe, burn_in=100,
                                    Lmax=300, RmaxRec=64)
    assert rc == 0
    g = S.Population(gm, J, N, max_chunk=32)
    r1, r2, secs = S.smc_run_hybrid(gm, g, 21, 22, check_every=1, force_every=fe, burn_in=100,
                                    Lmax=300, RmaxRec=64, test_fn=S.SMC_TEST_PARAMS)
    for r, o in ((r1, o1), (r2, o2)):
        sg, so = r.summary(), o.summary()
        assert np.array_equal(sg["t_end"], so["t_end"]) and np.array_equal(sg["R"], so["R"])
        assert sg["log_ml"] == pytest.approx(so["log_ml"], rel=1e-9)
        assert sg["log_score"][0] == pytest.approx(so["log_score"], rel=1e-9)
    rep = S.hybrid_report(r1, r2, secs)
    assert rep["steps"][0]["cycles"] == rep["steps"][1]["cycles"]
    assert np.all(secs > 0)
    a, b = rep["steps"]
    assert rep["z_log_ml"] == pytest.approx(
        abs(a["log_ml"] - b["log_ml"]) / np.hypot(a["nse"], b["nse"]), rel=1e-15)
    if np.isnan(a["log_score"]):
        assert np.isnan(rep["z_log_score"])
    else:
        assert rep["z_log_score"] == pytest.approx(
            abs(a["log_score"] - b["log_score"]) / np.hypot(a["log_score_nse"],
                                                            b["log_score_nse"]), rel=1e-15)


@pytest.mark.parametrize("every", [1, 3])
@pytest.mark.parametrize("kernel", [S.SMC_KERNEL_RW, S.SMC_KERNEL_INDEPENDENT, S.SMC_KERNEL_MALA])
def test_mutation_timing_leaves_the_run_unchanged(kernel, every):
    """Timing mutation launches (events carried on the kernel's own dispatch,
    or around the Langevin step's kernels; every one, or every 3rd M step of
    the run) changes nothing the run computes, and yields one positive
    duration per timed M step and -1 for every other entry."""
    w = SD.workload("egarch11", T=300)
    gm = gpu_model(w)
    J, N = 4, 256
    out = []
    for timed in (False, True):
        g = S.Population(gm, J, N, max_chunk=64, with_grad=kernel == S.SMC_KERNEL_MALA)
        rec = S.Record(gm, J, Lmax=200, RmaxRec=32, time_mutate=timed, time_every=every)
        S.smc_run(gm, g, seed=11, kernel=kernel, record=rec)
        out.append((rec, rec.summary(), g.theta.cpu().numpy()))
    (_, a, th_a), (rec, b, th_b) = out
    assert np.array_equal(a["t_end"], b["t_end"]) and np.array_equal(a["R"], b["R"])
    assert a["log_ml"] == b["log_ml"] and a["nse"] == b["nse"]
    assert np.array_equal(th_a, th_b)
    step = 0  # the run's M steps in order
    for l in range(b["L"]):
        for r in range(b["R"][l]):
            ms = rec.mutate_ms[l, r]
            if step % every == 0:
                assert 0 < ms < 1e3, (l, r, ms)
            else:
                assert ms == -1, (l, r, ms)
            step += 1
        assert np.all(rec.mutate_ms[l, b["R"][l]:] == -1)
    assert np.all(rec.mutate_ms[b["L"]:] == -1)


def test_run_stops_on_numerical_flags():
    """An observation no parameter can explain (a NaN return) gives every
    particle zero weight: the S phase raises the dead-group flag, which the
    driver reads back with the next C phase's decision and turns into an
    error naming the cycle (the record keeps the cycles before it)."""
    w = SD.workload("egarch11", T=120)
    y = np.array(w.y[:120], dtype=np.float64)
    y[60] = np.nan                              # observation (date) 61
    m = S.Model(w.kind, y, K=w.K, shock=w.shock, precision=S.SMC_FP64)
    g = S.Population(m, 4, 64, max_chunk=64)
    rec = S.Record(m, 4, Lmax=200, RmaxRec=32)
    with pytest.raises(S.SmcError) as ei:
        S.smc_run(m, g, seed=5, record=rec)
    assert ei.value.status == S.SMC_E_NUMERIC
    assert "flags" in str(ei.value)
    L = rec.L
    assert L >= 1 and rec.t_end[L - 1] == 61


def test_run_stops_when_the_particle_variance_is_singular():
    """Two groups of 16 particles of the four-parameter regression: the
    oracle's run stops when the particle variance is no longer positive
    definite, and so does the GPU's, with a numerical error naming the flags
    and the same cycles recorded before it."""
    w = SD.workload("linreg", T=60)
    om = O.Model.from_workload(w)
    rc, orec, _ = O.run(om, 2, 16, 21, Lmax=62, RmaxRec=64)
    assert rc != 0
    m = S.Model.from_workload(w)
    g = S.Population(m, 2, 16, max_chunk=16)
    rec = S.Record(m, 2, Lmax=62, RmaxRec=64)
    with pytest.raises(S.SmcError) as ei:
        S.smc_run(m, g, seed=21, record=rec)
    assert ei.value.status == S.SMC_E_NUMERIC
    assert "flags" in str(ei.value)
    # the device raises the flag in the failing cycle; the driver reads it
    # back with the next decision, so the record may hold that cycle too
    assert orec.L <= rec.L <= orec.L + 1
    assert np.array_equal(rec.t_end[:orec.L], orec.t_end[:orec.L])
