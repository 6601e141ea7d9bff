"""Oracle: plain, slow FP64 CPU reference of the sequential posterior simulator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1304_4334_amd``) never imports, links or executes anything
here, and this package imports nothing from it.

``smc_oracle.c`` holds the algorithm (compiled by ``oracle/build.py`` with gcc);
this module is a ctypes binding over it with numpy arrays, plus
``closed_form`` (conjugate-regression marginal likelihood and posterior).

Layout convention here: parameters are ``[P, d]`` (particle-major rows), the
natural CPU layout; the HIP path stores ``[d, P]`` and tests transpose.

Parity-unpinned functions: the EGARCH log-likelihood for generic parameter
values has no external value to compare with beyond the special cases and
invariants in the tests (shock recovery on simulated data, the iid special
case, factor exchange, location-scale equivariance, finite-difference
gradients); see the test modules.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

RESIDUAL, MULTINOMIAL, STRATIFIED, SYSTEMATIC = 0, 1, 2, 3
RW, MALA, INDEP = 0, 1, 2
LINREG, EGARCH = 1, 2
GAUSS, STUDENT_T, MIXTURE = 0, 1, 2
PRIOR, RESAMPLE, PROPOSAL, ACCEPT = 1, 2, 3, 4
TEST_PARAMS, TEST_MODEL = 0, 1


class OrcModel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("K", C.c_int32), ("shock", C.c_int32),
                ("nreg", C.c_int32), ("T", C.c_int64),
                ("y", C.POINTER(C.c_double)), ("X", C.POINTER(C.c_double)),
                ("I", C.c_int32), ("pad", C.c_int32)]


class OrcPop(C.Structure):
    _fields_ = [("J", C.c_int32), ("N", C.c_int32), ("d", C.c_int32), ("S", C.c_int32),
                ("theta", C.POINTER(C.c_double)), ("logprior", C.POINTER(C.c_double)),
                ("loglik", C.POINTER(C.c_double)), ("state", C.POINTER(C.c_double)),
                ("logw", C.POINTER(C.c_double))]


class OrcCfg(C.Structure):
    _fields_ = [("J", C.c_int32), ("N", C.c_int32), ("seed", C.c_uint64), ("run", C.c_uint64),
                ("check_every", C.c_int32), ("force_every", C.c_int32), ("D1", C.c_double), ("D2", C.c_double),
                ("Rbar", C.c_int32), ("kappa", C.c_int32), ("stop_rule", C.c_int32),
                ("E1", C.c_double), ("Rmax", C.c_int32), ("scheme", C.c_int32),
                ("kernel", C.c_int32), ("replay", C.c_int32), ("Lmax", C.c_int32),
                ("RmaxRec", C.c_int32), ("test_fn", C.c_int32), ("pad", C.c_int32),
                ("E2", C.c_double), ("burn_in", C.c_int64)]


class OrcRecord(C.Structure):
    _fields_ = [("L", C.c_int32), ("t_end", C.POINTER(C.c_int64)), ("R", C.POINTER(C.c_int32)),
                ("hchol", C.POINTER(C.c_double)), ("rss", C.POINTER(C.c_double)),
                ("n_acc", C.POINTER(C.c_int64)), ("group_logwbar", C.POINTER(C.c_double)),
                ("log_ml", C.c_double), ("nse", C.c_double), ("log_ml_tilde", C.c_double),
                ("evals", C.c_int64), ("moments", C.POINTER(C.c_double)),
                ("mean", C.POINTER(C.c_double)), ("log_score", C.c_double), ("log_score_nse", C.c_double),
                ("log_score_tilde", C.c_double), ("mh", C.POINTER(C.c_int32)),
                ("chol", C.POINTER(C.c_double))]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_loglik_range.restype = C.c_double
        L.orc_logprior.restype = C.c_double
        L.orc_loglik_grad.restype = C.c_double
        L.orc_logprior_grad.restype = C.c_double
        L.orc_rss.restype = C.c_double
        L.orc_rss.argtypes = [dp, C.c_int64]
        L.orc_rne_mean.restype = C.c_double
        L.orc_correct.restype = C.c_int64
        L.orc_mutate.restype = C.c_int64
        L.orc_resample.restype = C.c_int
        L.orc_moments.restype = C.c_int
        L.orc_run.restype = C.c_int
        L.orc_dim.restype = C.c_int
        L.orc_state_dim.restype = C.c_int
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Model:
    """Holds the numpy data alive for the C struct."""

    def __init__(self, kind, T, y, K=0, shock=GAUSS, nreg=0, X=None, I=0):
        self.y = _f64(y)
        self.X = _f64(X) if X is not None else None
        self.c = OrcModel(kind, K, shock, nreg, T, _dp(self.y),
                          _dp(self.X) if self.X is not None else C.POINTER(C.c_double)(), I, 0)
        self.kind, self.K, self.shock, self.nreg, self.T, self.I = kind, K, shock, nreg, T, I

    @classmethod
    def from_workload(cls, w, T=None):
        T = T or w.T
        return cls(w.kind, T, w.y[:T], K=w.K, shock=w.shock, nreg=w.nreg,
                   X=None if w.X is None else w.X[:T], I=w.I)

    @property
    def d(self):
        return lib().orc_dim(C.byref(self.c))

    @property
    def S(self):
        return lib().orc_state_dim(C.byref(self.c))


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's particle loops (timing only)."""
    lib().orc_set_num_threads(C.c_int(int(n)))


def run_hybrid(m: Model, J, N, seed, seed2, **kw):
    """Algorithm 3: an adaptive run (key (seed, run)), then Algorithm 1 on its
    design {t_l, hL_lr, R_l} with the new key (seed2, run).  Returns
    (rc, record1, record2, population after step 2)."""
    rc, r1, _ = run(m, J, N, seed, **kw)
    if rc:
        return rc, r1, None, None
    kw = {k: v for k, v in kw.items() if k not in ("Lmax", "RmaxRec")}
    rc, r2, pop = run(m, J, N, seed2, record=r1, **kw)
    return rc, r1, r2, pop


def philox(ctr, key):
    out = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10((C.c_uint64 * 4)(*ctr), (C.c_uint64 * 2)(*key), out)
    return [int(v) for v in out]


def normals(seed, run, c0, c1, c2, purpose, n):
    z = np.zeros(n)
    lib().orc_normals(C.c_uint64(seed), C.c_uint64(run), C.c_uint64(c0), C.c_uint64(c1),
                      C.c_uint64(c2), C.c_uint64(purpose), C.c_int(n), _dp(z))
    return z


def mixture_params(m: Model, theta):
    """(p, mu, sigma) of the shock mixture at theta (eqs EGARCH_tran1/2)."""
    p, mu, sg = np.zeros(m.I), np.zeros(m.I), np.zeros(m.I)
    th = _f64(theta)
    lib().orc_mixture_params(C.byref(m.c), _dp(th), _dp(p), _dp(mu), _dp(sg))
    return p, mu, sg


def num_test_fns(m: Model, which=TEST_MODEL):
    return int(lib().orc_num_test_fns(C.byref(m.c), C.c_int(which)))


def test_fns(m: Model, theta, state, t, which=TEST_MODEL):
    """Test functions at one particle (Section 5.2's g1..g3 for EGARCH)."""
    g = np.zeros(num_test_fns(m, which))
    th, st = _f64(theta), _f64(state if state is not None and len(state) else np.zeros(8))
    lib().orc_test_fns(C.byref(m.c), C.c_int(which), _dp(th), _dp(st), C.c_int64(t), _dp(g))
    return g


def report(J, N, g):
    """Posterior moment report of g[P, G]: rows (mean, sd, NSE, RNE)."""
    g = _f64(g)
    G = g.shape[1]
    out = np.zeros((G, 4))
    lib().orc_report(C.c_int32(J), C.c_int32(N), C.c_int(G), _dp(g), _dp(out))
    return out


def test_report(m: Model, pop, t, which=TEST_MODEL):
    out = np.zeros((num_test_fns(m, which), 4))
    lib().orc_test_report(C.byref(m.c), C.byref(pop.c), C.c_int(which), C.c_int64(t), _dp(out))
    return out


def logprior(m: Model, theta):
    th = _f64(theta)
    return lib().orc_logprior(C.byref(m.c), _dp(th))


def prior_draw(m: Model, seed, run, p):
    th = np.zeros(m.d)
    lib().orc_prior_draw(C.byref(m.c), C.c_uint64(seed), C.c_uint64(run), C.c_int64(p), _dp(th))
    return th


def loglik(m: Model, theta, t=None, state=None, t0=0):
    """log p(y_{t0+1:t} | theta) for one parameter vector (state at t0 given or s0)."""
    t = m.T if t is None else t
    st = np.zeros(max(m.S, 1)) if state is None else _f64(state).copy()
    th = _f64(theta)
    ll = lib().orc_loglik_range(C.byref(m.c), _dp(th), C.c_int64(t0), C.c_int64(t), _dp(st))
    return ll, st[:m.S]


def loglik_batch(m: Model, theta, t=None):
    th = _f64(theta)
    P = th.shape[0]
    t = m.T if t is None else t
    ll = np.zeros(P)
    st = np.zeros((P, max(m.S, 1)))
    lib().orc_loglik_batch(C.byref(m.c), C.c_int64(P), _dp(th), C.c_int64(t), _dp(ll),
                           _dp(st) if m.S else C.POINTER(C.c_double)())
    return ll, st[:, :m.S] if m.S else np.zeros((P, 0))


def loglik_grad(m: Model, theta, t=None):
    t = m.T if t is None else t
    g = np.zeros(m.d)
    ll = lib().orc_loglik_grad(C.byref(m.c), _dp(_f64(theta)), C.c_int64(t), _dp(g))
    return ll, g


def logprior_grad(m: Model, theta):
    g = np.zeros(m.d)
    lp = lib().orc_logprior_grad(C.byref(m.c), _dp(_f64(theta)), _dp(g))
    return lp, g


class Pop:
    """Particle population in the oracle's [P, d] layout."""

    def __init__(self, m: Model, J, N):
        self.J, self.N, self.d, self.S = J, N, m.d, m.S
        P = J * N
        self.theta = np.zeros((P, self.d))
        self.logprior = np.zeros(P)
        self.loglik = np.zeros(P)
        self.state = np.zeros((P, max(self.S, 1)))
        self.logw = np.zeros(P)
        self._sync()

    def _sync(self):
        for name in ("theta", "logprior", "loglik", "state", "logw"):
            a = getattr(self, name)
            if not (a.flags.c_contiguous and a.dtype == np.float64):
                setattr(self, name, _f64(a))
        self.c = OrcPop(self.J, self.N, self.d, self.S, _dp(self.theta), _dp(self.logprior),
                        _dp(self.loglik), _dp(self.state), _dp(self.logw))

    def copy(self):
        q = Pop.__new__(Pop)
        q.J, q.N, q.d, q.S = self.J, self.N, self.d, self.S
        for name in ("theta", "logprior", "loglik", "state", "logw"):
            setattr(q, name, getattr(self, name).copy())
        q._sync()
        return q


def init(m: Model, pop: Pop, seed, run=0):
    pop._sync()
    lib().orc_init(C.byref(m.c), C.byref(pop.c), C.c_uint64(seed), C.c_uint64(run))


def correct(m: Model, pop: Pop, t_from, t_max, check_every=1, rss_min=0.5):
    pop._sync()
    rss = C.c_double(0)
    glwb = np.zeros(pop.J)
    t = lib().orc_correct(C.byref(m.c), C.byref(pop.c), C.c_int64(t_from), C.c_int64(t_max),
                          C.c_int64(check_every), C.c_double(rss_min), C.byref(rss), _dp(glwb))
    return int(t), rss.value, glwb


def rss(logw):
    lw = _f64(logw)
    return lib().orc_rss(_dp(lw), C.c_int64(lw.size))


def resample(J, N, logw, scheme=RESIDUAL, seed=1, run=0, cycle=1, with_margin=False):
    lw = _f64(logw)
    anc = np.zeros(J * N, dtype=np.int32)
    mrg = np.zeros(J)
    bad = lib().orc_resample(C.c_int32(J), C.c_int32(N), _dp(lw), C.c_int(scheme),
                             C.c_uint64(seed), C.c_uint64(run), C.c_uint64(cycle),
                             anc.ctypes.data_as(C.POINTER(C.c_int32)), _dp(mrg))
    if with_margin:
        return anc, bad, mrg
    return anc, bad


def gather(pop: Pop, anc):
    pop._sync()
    a = np.ascontiguousarray(anc, dtype=np.int32)
    lib().orc_gather(C.byref(pop.c), a.ctypes.data_as(C.POINTER(C.c_int32)))


def moments(pop: Pop):
    pop._sync()
    d = pop.d
    mean, cov, chol = np.zeros(d), np.zeros((d, d)), np.zeros((d, d))
    rc = lib().orc_moments(C.byref(pop.c), _dp(mean), _dp(cov), _dp(chol))
    return mean, cov, chol, rc


def mutate(m: Model, pop: Pop, t, hchol, seed, run=0, cycle=1, it=1, kernel=RW):
    pop._sync()
    hl = _f64(hchol)
    acc = np.zeros(pop.J * pop.N, dtype=np.uint8)
    n = lib().orc_mutate(C.byref(m.c), C.byref(pop.c), C.c_int64(t), C.c_int(kernel), _dp(hl),
                         C.c_uint64(seed), C.c_uint64(run), C.c_uint64(cycle), C.c_uint64(it),
                         acc.ctypes.data_as(C.POINTER(C.c_uint8)))
    return int(n), acc


def mutate_particle(m: Model, p, theta, lp, ll, t, hchol, seed, run=0, cycle=1, it=1,
                    kernel=RW):
    """M step of the single particle with global index p; returns
    (accepted, theta, lp, ll, state)."""
    th = _f64(theta).copy()
    lpv, llv = C.c_double(lp), C.c_double(ll)
    st = np.zeros(max(m.S, 1))
    acc = lib().orc_mutate_particle(C.byref(m.c), C.c_int64(p), _dp(th), C.byref(lpv),
                                    C.byref(llv), _dp(st), C.c_int64(t), C.c_int(kernel),
                                    _dp(_f64(hchol)), C.c_uint64(seed), C.c_uint64(run),
                                    C.c_uint64(cycle), C.c_uint64(it))
    return bool(acc), th, lpv.value, llv.value, st[:m.S]


def rne_mean(pop: Pop):
    pop._sync()
    return lib().orc_rne_mean(C.byref(pop.c))


def log_ml(group_logwbar):
    g = _f64(group_logwbar)
    L, J = g.shape
    out = np.zeros(3)
    lib().orc_log_ml(C.c_int32(L), C.c_int32(J), _dp(g), _dp(out))
    return out


class Record:
    def __init__(self, J, d, Lmax=400, RmaxRec=128, G=0):
        self.Lmax, self.RmaxRec, self.J, self.d, self.G = Lmax, RmaxRec, J, d, G
        self.t_end = np.zeros(Lmax, dtype=np.int64)
        self.R = np.zeros(Lmax, dtype=np.int32)
        self.hchol = np.zeros((Lmax, RmaxRec, d, d))
        self.rss = np.zeros(Lmax)
        self.n_acc = np.zeros((Lmax, RmaxRec), dtype=np.int64)
        self.group_logwbar = np.zeros((Lmax, J))
        self.moments = np.zeros((Lmax, max(G, 1), 4))
        self.mean = np.zeros((Lmax, RmaxRec, d))
        self.mh = np.zeros((Lmax, RmaxRec), dtype=np.int32)
        self.chol = np.zeros((Lmax, RmaxRec, d, d))
        self.c = OrcRecord(0, self.t_end.ctypes.data_as(C.POINTER(C.c_int64)),
                           self.R.ctypes.data_as(C.POINTER(C.c_int32)), _dp(self.hchol),
                           _dp(self.rss), self.n_acc.ctypes.data_as(C.POINTER(C.c_int64)),
                           _dp(self.group_logwbar), 0.0, 0.0, 0.0, 0,
                           _dp(self.moments) if G else C.POINTER(C.c_double)(),
                           _dp(self.mean), float("nan"), float("nan"), float("nan"),
                           self.mh.ctypes.data_as(C.POINTER(C.c_int32)), _dp(self.chol))

    @property
    def L(self):
        return self.c.L

    def summary(self):
        L = self.L
        return dict(L=L, t_end=self.t_end[:L].copy(), R=self.R[:L].copy(),
                    rss=self.rss[:L].copy(), log_ml=self.c.log_ml, nse=self.c.nse,
                    log_ml_tilde=self.c.log_ml_tilde, evals=self.c.evals,
                    group_logwbar=self.group_logwbar[:L].copy(),
                    moments=self.moments[:L, :self.G].copy() if self.G else None,
                    log_score=self.c.log_score, log_score_nse=self.c.log_score_nse,
                    log_score_tilde=self.c.log_score_tilde,
                    n_acc=self.n_acc[:L].copy(), mh=self.mh[:L].copy(),
                    chol=self.chol[:L].copy(), hchol=self.hchol[:L].copy())


def run(m: Model, J, N, seed, run_id=0, check_every=1, force_every=0, D1=0.5, D2=0.2, Rbar=7, kappa=3,
        stop_rule=0, E1=0.35, Rmax=100, scheme=RESIDUAL, kernel=RW, record=None,
        Lmax=400, RmaxRec=128, test_fn=TEST_PARAMS, E2=0.90, burn_in=0, moments=False):
    """Whole simulator.  With ``record`` given (a Record filled by an earlier
    run) the design {t_l, hL_lr, R_l} is replayed (Algorithm 1).  With
    ``moments`` the record keeps the test-function report of every cycle."""
    replay = record is not None
    G = num_test_fns(m, test_fn) if moments else 0
    rec = record if replay else Record(J, m.d, Lmax, RmaxRec, G)
    cfg = OrcCfg(J, N, seed, run_id, check_every, force_every, D1, D2, Rbar, kappa, stop_rule, E1, Rmax,
                 scheme, kernel, 1 if replay else 0, rec.Lmax, rec.RmaxRec, test_fn, 0, E2, burn_in)
    pop = Pop(m, J, N)
    if replay:
        # replay writes into a fresh record that shares the design arrays
        out = Record(J, m.d, rec.Lmax, rec.RmaxRec, G)
        out.t_end[:] = rec.t_end
        out.R[:] = rec.R
        out.hchol[:] = rec.hchol
        out.mean[:] = rec.mean
        rec = out
    rc = lib().orc_run(C.byref(m.c), C.byref(cfg), C.byref(pop.c), C.byref(rec.c))
    return rc, rec, pop
