"""ctypes binding of libsmc.so (include/smc.h): argument marshalling only.

Every computation runs in the HIP library.  torch supplies device memory and
the stream; nothing here falls back to the CPU.  If the library is missing
the import of a call raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmc.so")

# Enums (values fixed by include/smc.h).
SMC_OK = 0
SMC_E_INVALID_ARG, SMC_E_UNSUPPORTED, SMC_E_DEVICE, SMC_E_NUMERIC, SMC_E_WORKSPACE = -1, -2, -3, -4, -5
SMC_MODEL_LINREG, SMC_MODEL_EGARCH = 1, 2
SMC_SHOCK_GAUSS, SMC_SHOCK_STUDENT_T, SMC_SHOCK_MIXTURE = 0, 1, 2
SMC_FP64, SMC_FP32 = 0, 1
SMC_TEST_PARAMS, SMC_TEST_MODEL = 0, 1
SMC_RESAMPLE_RESIDUAL, SMC_RESAMPLE_MULTINOMIAL = 0, 1
SMC_RESAMPLE_STRATIFIED, SMC_RESAMPLE_SYSTEMATIC = 2, 3
SMC_KERNEL_RW, SMC_KERNEL_MALA, SMC_KERNEL_INDEPENDENT = 0, 1, 2
SMC_FLAG_DEAD_GROUP, SMC_FLAG_NOT_PD = 1, 2

_vp = C.c_void_p


class ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("K", C.c_int32), ("shock", C.c_int32),
                ("nreg", C.c_int32), ("precision", C.c_int32), ("ncomp", C.c_int32),
                ("T", C.c_int64), ("y", _vp), ("y32", _vp), ("X", _vp)]


class Particles(C.Structure):
    _fields_ = [("J", C.c_int32), ("N", C.c_int32), ("theta", _vp), ("logprior", _vp),
                ("loglik", _vp), ("state", _vp), ("logw", _vp), ("grad", _vp),
                ("ancestor", _vp), ("ws", _vp), ("ws_bytes", C.c_size_t)]


class Rng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("run", C.c_uint64)]


class RunConfig(C.Structure):
    _fields_ = [("J", C.c_int32), ("N", C.c_int32), ("rng", Rng),
                ("check_every", C.c_int32), ("force_every", C.c_int32),
                ("D1", C.c_double), ("D2", C.c_double), ("Rbar", C.c_int32),
                ("kappa", C.c_int32), ("stop_rule", C.c_int32), ("E1", C.c_double),
                ("Rmax", C.c_int32), ("scheme", C.c_int32), ("kernel", C.c_int32),
                ("replay", C.c_int32), ("Lmax", C.c_int32), ("RmaxRec", C.c_int32),
                ("max_chunk", C.c_int64), ("test_fn", C.c_int32), ("graph", C.c_int32),
                ("E2", C.c_double), ("burn_in", C.c_int64)]


class RunRecord(C.Structure):
    _fields_ = [("L", C.c_int32), ("time_every", C.c_int32), ("t_end", _vp), ("R", _vp),
                ("rss", _vp), ("n_accept", _vp), ("hchol", _vp), ("group_logwbar", _vp),
                ("log_ml", _vp), ("evals", C.c_int64), ("mh_steps", C.c_int64),
                ("mutate_ms", _vp), ("moments", _vp), ("log_score", _vp), ("mean", _vp)]


class BatchTiming(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("launches", C.c_int32), ("ms", _vp), ("evals", _vp)]


_L = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        st = C.c_int32
        P = C.POINTER
        L.smc_status_string.restype = C.c_char_p
        L.smc_status_string.argtypes = [st]
        L.smc_last_error.restype = C.c_char_p
        L.smc_last_error.argtypes = []
        L.smc_model_create.restype = st
        L.smc_model_create.argtypes = [P(ModelDesc), P(_vp)]
        L.smc_model_destroy.restype = st
        L.smc_model_destroy.argtypes = [_vp]
        L.smc_model_set_launch.restype = st
        L.smc_model_set_launch.argtypes = [_vp, C.c_int32, C.c_int32]
        L.smc_model_dim.restype = C.c_int32
        L.smc_model_dim.argtypes = [_vp]
        L.smc_model_state_dim.restype = C.c_int32
        L.smc_model_state_dim.argtypes = [_vp]
        L.smc_workspace_bytes.restype = C.c_size_t
        L.smc_workspace_bytes.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int64]
        L.smc_backward_ws_bytes.restype = C.c_size_t
        L.smc_backward_ws_bytes.argtypes = [_vp, C.c_int64, C.c_int64]
        L.smc_mala_workspace_bytes.restype = C.c_size_t
        L.smc_mala_workspace_bytes.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int64]
        L.smc_posterior_grad.restype = st
        L.smc_posterior_grad.argtypes = [_vp, P(Particles), C.c_int64, _vp]
        L.smc_init_from_prior.restype = st
        L.smc_init_from_prior.argtypes = [_vp, P(Particles), Rng, _vp]
        L.smc_correct.restype = st
        L.smc_correct.argtypes = [_vp, P(Particles), C.c_int64, C.c_int64, C.c_int64,
                                  C.c_double, _vp, P(C.c_int64), P(C.c_double), _vp]
        L.smc_correct_async.restype = st
        L.smc_correct_async.argtypes = [_vp, P(Particles), C.c_int64, C.c_int64, C.c_int64,
                                        C.c_double, _vp, _vp, _vp, _vp]
        L.smc_resample.restype = st
        L.smc_resample.argtypes = [_vp, P(Particles), C.c_int32, Rng, C.c_int32, _vp]
        L.smc_particle_moments.restype = st
        L.smc_particle_moments.argtypes = [_vp, P(Particles), _vp, _vp, _vp, _vp, _vp]
        L.smc_particle_moments_noalloc.restype = st
        L.smc_particle_moments_noalloc.argtypes = [_vp, P(Particles), _vp, _vp, _vp, _vp, _vp]
        L.smc_mutate.restype = st
        L.smc_mutate.argtypes = [_vp, P(Particles), C.c_int64, C.c_int32, _vp, Rng,
                                 C.c_int32, C.c_int32, _vp, _vp, _vp]
        L.smc_loglik.restype = st
        L.smc_loglik.argtypes = [_vp, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp]
        L.smc_loglik_backward.restype = st
        L.smc_loglik_backward.argtypes = [_vp, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp,
                                          C.c_size_t, _vp]
        L.smc_log_ml.restype = st
        L.smc_log_ml.argtypes = [C.c_int32, C.c_int32, _vp, _vp, _vp]
        L.smc_adapt_scale.restype = st
        L.smc_adapt_scale.argtypes = [_vp, C.c_int64, C.c_int32, _vp, _vp]
        L.smc_rne.restype = st
        L.smc_rne.argtypes = [_vp, P(Particles), _vp, _vp]
        L.smc_flags.restype = st
        L.smc_flags.argtypes = [P(Particles), P(C.c_int32), _vp]
        L.smc_batch_ws_bytes.restype = C.c_size_t
        L.smc_batch_ws_bytes.argtypes = [C.c_int32]
        L.smc_run_batch.restype = st
        L.smc_run_batch.argtypes = [C.c_int32, P(_vp), P(P(Particles)), P(RunConfig), P(RunRecord),
                                    _vp, C.c_size_t, C.c_int32, P(BatchTiming), _vp]
        L.smc_run.restype = st
        L.smc_run.argtypes = [_vp, P(Particles), P(RunConfig), P(RunRecord), _vp]
        L.smc_run_hybrid.restype = st
        L.smc_run_hybrid.argtypes = [_vp, P(Particles), P(RunConfig), C.c_uint64, P(RunRecord),
                                     P(RunRecord), _vp, _vp]
        L.smc_hybrid_report.restype = st
        L.smc_hybrid_report.argtypes = [P(RunRecord), P(RunRecord), _vp, _vp]
        L.smc_num_test_functions.restype = C.c_int32
        L.smc_num_test_functions.argtypes = [_vp, C.c_int32]
        L.smc_test_moments.restype = st
        L.smc_test_moments.argtypes = [_vp, P(Particles), C.c_int64, C.c_int32, _vp, _vp]
        L.smc_log_score.restype = st
        L.smc_log_score.argtypes = [C.c_int32, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp]
        _L = L
    return _L


class SmcError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.smc_status_string(status).decode()
        detail = L.smc_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")
        self.status = status


def _check(status, where):
    if status != SMC_OK:
        raise SmcError(status, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Model:
    """A model handle plus the device copies of its data."""

    def __init__(self, kind, y, X=None, K=1, shock=SMC_SHOCK_GAUSS, precision=SMC_FP64,
                 device="cuda", I=0):
        self.y = torch.as_tensor(y, dtype=torch.float64).to(device).contiguous()
        self.y32 = self.y.float().contiguous() if precision == SMC_FP32 else None
        self.X = (torch.as_tensor(X, dtype=torch.float64).to(device).contiguous()
                  if X is not None else None)
        nreg = int(self.X.shape[1]) if self.X is not None else 0
        self.kind, self.K, self.shock, self.precision, self.I = kind, K, shock, precision, I
        self.T = int(self.y.numel())
        self.device = device
        self.desc = ModelDesc(kind, K, shock, nreg, precision, I, self.T, _ptr(self.y),
                              _ptr(self.y32), _ptr(self.X))
        h = C.c_void_p()
        _check(lib().smc_model_create(C.byref(self.desc), C.byref(h)), "smc_model_create")
        self.h = h

    @classmethod
    def from_workload(cls, w, precision=SMC_FP64, device="cuda"):
        return cls(w.kind, w.y, X=w.X, K=w.K, shock=w.shock, precision=precision,
                   device=device, I=w.I)

    def set_launch(self, block=0, unroll=0):
        """Launch shape of the random-walk step (smc_model_set_launch)."""
        _check(lib().smc_model_set_launch(self.h, block, unroll), "smc_model_set_launch")
        self.launch = (block, unroll)

    @property
    def d(self):
        return lib().smc_model_dim(self.h)

    @property
    def S(self):
        return lib().smc_model_state_dim(self.h)

    @property
    def state_dtype(self):
        return torch.float32 if self.precision == SMC_FP32 else torch.float64

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().smc_model_destroy(self.h)
                self.h = None
        except Exception:
            pass


class Population:
    """Device buffers of J x N particles ([d][P] layouts) and a workspace."""

    def __init__(self, model: Model, J, N, max_chunk=256, with_grad=False):
        dev = model.device
        P = J * N
        self.model, self.J, self.N, self.P = model, J, N, P
        f64 = dict(dtype=torch.float64, device=dev)
        self.theta = torch.zeros((model.d, P), **f64)
        self.logprior = torch.zeros(P, **f64)
        self.loglik = torch.zeros(P, **f64)
        self.state = (torch.zeros((model.S, P), dtype=model.state_dtype, device=dev)
                      if model.S > 0 else None)
        self.logw = torch.zeros(P, **f64)
        self.grad = torch.zeros((model.d, P), **f64) if with_grad else None
        self.ancestor = torch.zeros(P, dtype=torch.int32, device=dev)
        self.max_chunk = max_chunk
        nb = (lib().smc_mala_workspace_bytes(model.h, J, N, max_chunk) if with_grad
              else lib().smc_workspace_bytes(model.h, J, N, max_chunk))
        if nb == 0:
            raise SmcError(-1, "smc_workspace_bytes")
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + nb]
        self.c = Particles(J, N, _ptr(self.theta), _ptr(self.logprior), _ptr(self.loglik),
                           _ptr(self.state), _ptr(self.logw), _ptr(self.grad),
                           _ptr(self.ancestor), _ptr(self.ws_view), nb)


# --- the calls, same names as the C ABI ----------------------------------

def smc_init_from_prior(model: Model, pop: Population, seed, run=0, stream=None):
    _check(lib().smc_init_from_prior(model.h, C.byref(pop.c), Rng(seed, run), _stream(stream)),
           "smc_init_from_prior")


def smc_correct(model, pop, t_from, t_max, check_every=1, rss_min=0.5, group_logwbar=None,
                want_rss=True, stream=None):
    """Returns (t_to, rss or None, group_logwbar tensor [J])."""
    glwb = group_logwbar if group_logwbar is not None else torch.empty(
        pop.J, dtype=torch.float64, device=model.device)
    t_to = C.c_int64(0)
    rss = C.c_double(0.0)
    _check(lib().smc_correct(model.h, C.byref(pop.c), t_from, t_max, check_every, rss_min,
                             _ptr(glwb), C.byref(t_to), C.byref(rss) if want_rss else None,
                             _stream(stream)), "smc_correct")
    return t_to.value, (rss.value if want_rss else None), glwb


def smc_correct_async(model, pop, t_from, t_max, check_every=1, rss_min=0.5,
                      group_logwbar=None, t_to=None, rss=None, want_rss=True, stream=None):
    """smc_correct with device outputs and no host synchronisation (capturable).
    Returns (t_to int64 tensor [1], rss float64 tensor [1] or None,
    group_logwbar tensor [J])."""
    dev = model.device
    glwb = group_logwbar if group_logwbar is not None else torch.empty(
        pop.J, dtype=torch.float64, device=dev)
    t_to = t_to if t_to is not None else torch.empty(1, dtype=torch.int64, device=dev)
    if want_rss and rss is None:
        rss = torch.empty(1, dtype=torch.float64, device=dev)
    _check(lib().smc_correct_async(model.h, C.byref(pop.c), t_from, t_max, check_every, rss_min,
                                   _ptr(glwb), _ptr(t_to), _ptr(rss) if want_rss else None,
                                   _stream(stream)), "smc_correct_async")
    return t_to, (rss if want_rss else None), glwb


def smc_resample(model, pop, scheme=SMC_RESAMPLE_RESIDUAL, seed=1, run=0, cycle=1,
                 stream=None):
    _check(lib().smc_resample(model.h, C.byref(pop.c), scheme, Rng(seed, run), cycle,
                              _stream(stream)), "smc_resample")


def smc_particle_moments(model, pop, mh, mean=None, cov=None, hchol=None, stream=None):
    if hchol is None:
        hchol = torch.zeros((model.d, model.d), dtype=torch.float64, device=model.device)
    _check(lib().smc_particle_moments(model.h, C.byref(pop.c), _ptr(mh), _ptr(mean), _ptr(cov),
                                      _ptr(hchol), _stream(stream)), "smc_particle_moments")
    return hchol


def smc_particle_moments_noalloc(model, pop, mh, mean=None, cov=None, hchol=None, stream=None):
    """smc_particle_moments without the population's workspace (its scratch
    is the library's static device array)."""
    if hchol is None:
        hchol = torch.zeros((model.d, model.d), dtype=torch.float64, device=model.device)
    _check(lib().smc_particle_moments_noalloc(model.h, C.byref(pop.c), _ptr(mh), _ptr(mean),
                                              _ptr(cov), _ptr(hchol), _stream(stream)),
           "smc_particle_moments_noalloc")
    return hchol


def smc_mutate(model, pop, t, hchol, seed, run=0, cycle=1, it=1, kernel=SMC_KERNEL_RW,
               n_accept=None, accepted=None, stream=None):
    if n_accept is None:
        n_accept = torch.zeros(1, dtype=torch.int64, device=model.device)
    _check(lib().smc_mutate(model.h, C.byref(pop.c), t, kernel, _ptr(hchol), Rng(seed, run),
                            cycle, it, _ptr(n_accept), _ptr(accepted), _stream(stream)),
           "smc_mutate")
    return n_accept


def smc_loglik(model, theta, t, state_out=None, stream=None):
    P = int(theta.shape[1])
    out = torch.empty(P, dtype=torch.float64, device=model.device)
    _check(lib().smc_loglik(model.h, P, _ptr(theta), t, _ptr(out), _ptr(state_out),
                            _stream(stream)), "smc_loglik")
    return out


def smc_loglik_backward(model, theta, t, dloglik, stream=None):
    P = int(theta.shape[1])
    dtheta = torch.empty_like(theta)
    nb = lib().smc_backward_ws_bytes(model.h, P, t)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=model.device)
    _check(lib().smc_loglik_backward(model.h, P, _ptr(theta), t, _ptr(dloglik), _ptr(dtheta),
                                     _ptr(ws), nb, _stream(stream)), "smc_loglik_backward")
    return dtheta


def smc_posterior_grad(model, pop, t, stream=None):
    """pop.grad <- gradient of log prior + log likelihood over 1..t."""
    _check(lib().smc_posterior_grad(model.h, C.byref(pop.c), t, _stream(stream)),
           "smc_posterior_grad")
    return pop.grad


def smc_log_ml(group_logwbar, stream=None):
    g = group_logwbar.contiguous()
    L, J = g.shape
    out = torch.empty(3, dtype=torch.float64, device=g.device)
    _check(lib().smc_log_ml(L, J, _ptr(g), _ptr(out), _stream(stream)), "smc_log_ml")
    return out


def smc_adapt_scale(n_accept, P, target_permille, mh, stream=None):
    _check(lib().smc_adapt_scale(_ptr(n_accept), P, target_permille, _ptr(mh), _stream(stream)),
           "smc_adapt_scale")


def smc_rne(model, pop, stream=None):
    out = torch.empty(1, dtype=torch.float64, device=model.device)
    _check(lib().smc_rne(model.h, C.byref(pop.c), _ptr(out), _stream(stream)), "smc_rne")
    return out


def smc_flags(pop, stream=None):
    f = C.c_int32(0)
    _check(lib().smc_flags(C.byref(pop.c), C.byref(f), _stream(stream)), "smc_flags")
    return f.value


class Record:
    """Host and device arrays of a run's design and outputs."""

    def __init__(self, model, J, Lmax=512, RmaxRec=128, time_mutate=False, test_fn=None,
                 time_every=1):
        """``test_fn`` (SMC_TEST_*) also keeps the moment report of every cycle
        and the log score; with ``time_mutate`` every ``time_every``-th
        Metropolis iteration is timed (the others' entries are -1)."""
        import numpy as np
        d, dev = model.d, model.device
        self.Lmax, self.RmaxRec, self.J, self.d = Lmax, RmaxRec, J, d
        self.test_fn = test_fn
        self.G = smc_num_test_functions(model, test_fn) if test_fn is not None else 0
        self.t_end = np.zeros(Lmax, dtype=np.int64)
        self.R = np.zeros(Lmax, dtype=np.int32)
        self.rss = np.zeros(Lmax, dtype=np.float64)
        self.n_accept = torch.zeros((Lmax, RmaxRec), dtype=torch.int64, device=dev)
        self.hchol = torch.zeros((Lmax, RmaxRec, d, d), dtype=torch.float64, device=dev)
        self.group_logwbar = torch.zeros((Lmax, J), dtype=torch.float64, device=dev)
        self.log_ml = torch.zeros(3, dtype=torch.float64, device=dev)
        self.mutate_ms = np.zeros((Lmax, RmaxRec), dtype=np.float32) if time_mutate else None
        self.moments = (torch.zeros((Lmax, self.G, 4), dtype=torch.float64, device=dev)
                        if self.G else None)
        self.log_score = (torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
                          if self.G else None)
        self.mean = torch.zeros((Lmax, RmaxRec, d), dtype=torch.float64, device=dev)
        self.c = RunRecord(0, time_every, self.t_end.ctypes.data, self.R.ctypes.data,
                           self.rss.ctypes.data,
                           _ptr(self.n_accept), _ptr(self.hchol), _ptr(self.group_logwbar),
                           _ptr(self.log_ml), 0, 0,
                           self.mutate_ms.ctypes.data if time_mutate else None,
                           _ptr(self.moments), _ptr(self.log_score), _ptr(self.mean))

    @property
    def L(self):
        return self.c.L

    def summary(self):
        L = self.L
        lm = self.log_ml.cpu().numpy()
        return dict(L=L, t_end=self.t_end[:L].copy(), R=self.R[:L].copy(), rss=self.rss[:L].copy(),
                    log_ml=float(lm[0]), nse=float(lm[1]), log_ml_tilde=float(lm[2]),
                    evals=self.c.evals, mh_steps=self.c.mh_steps,
                    group_logwbar=self.group_logwbar[:L].cpu().numpy(),
                    n_accept=self.n_accept[:L].cpu().numpy(),
                    moments=self.moments[:L].cpu().numpy() if self.G else None,
                    log_score=(self.log_score.cpu().numpy().tolist() if self.G
                               else [float("nan")] * 3))


def smc_num_test_functions(model, which=SMC_TEST_MODEL):
    return int(lib().smc_num_test_functions(model.h, which))


def smc_test_moments(model, pop, t, which=SMC_TEST_MODEL, out=None, stream=None):
    """Posterior moments of the test functions at date t: [G, 4] device
    tensor of (mean, sd, NSE, RNE)."""
    G = smc_num_test_functions(model, which)
    if G < 1:
        raise SmcError(SMC_E_INVALID_ARG, "smc_test_moments")
    out = out if out is not None else torch.empty((G, 4), dtype=torch.float64, device=model.device)
    _check(lib().smc_test_moments(model.h, C.byref(pop.c), C.c_int64(t), which, _ptr(out),
                                  _stream(stream)), "smc_test_moments")
    return out


def smc_log_score(group_logwbar, t_end, burn_in, out=None, stream=None):
    """Log score over (burn_in, T] from a record's group weights (device [L, J])
    and cycle dates (host int64 [L])."""
    import numpy as np
    L, J = group_logwbar.shape
    te = np.ascontiguousarray(t_end[:L], dtype=np.int64)
    out = out if out is not None else torch.empty(3, dtype=torch.float64,
                                                  device=group_logwbar.device)
    _check(lib().smc_log_score(L, J, _ptr(group_logwbar.contiguous()), te.ctypes.data,
                               C.c_int64(burn_in), _ptr(out), _stream(stream)), "smc_log_score")
    return out


def smc_run(model, pop, seed, run=0, check_every=1, force_every=0, D1=0.5, D2=0.2, Rbar=7,
            kappa=3, stop_rule=0, E1=0.35, Rmax=100, scheme=SMC_RESAMPLE_RESIDUAL,
            kernel=SMC_KERNEL_RW, record=None, replay=False, Lmax=512, RmaxRec=128,
            test_fn=SMC_TEST_PARAMS, E2=0.90, burn_in=0, graph=False, stream=None):
    """Whole simulator (adaptive, or replay of ``record``'s design).  The RNE
    rule (stop_rule=1) uses ``test_fn``'s functions, with E2 after a C phase
    that ends at a date of interest; a record made with ``test_fn`` also
    receives the moment reports and the log score over ``burn_in``.  With
    ``graph`` the adaptive random-walk run is driven on the device (one
    captured step graph launched until the run ends; same results)."""
    rec = record if record is not None else Record(model, pop.J, Lmax, RmaxRec)
    if rec.G and rec.test_fn != test_fn:
        raise ValueError("the record's test functions differ from test_fn")
    cfg = RunConfig(pop.J, pop.N, Rng(seed, run), check_every, force_every, D1, D2, Rbar, kappa,
                    stop_rule, E1, Rmax, scheme, kernel, 1 if replay else 0, rec.Lmax,
                    rec.RmaxRec, pop.max_chunk, test_fn, 1 if graph else 0, E2, burn_in)
    _check(lib().smc_run(model.h, C.byref(pop.c), C.byref(cfg), C.byref(rec.c), _stream(stream)),
           "smc_run")
    return rec


def smc_run_hybrid(model, pop, seed, seed2, run=0, check_every=1, force_every=0, D1=0.5, D2=0.2,
                   Rbar=7, kappa=3, stop_rule=0, E1=0.35, Rmax=100,
                   scheme=SMC_RESAMPLE_RESIDUAL, kernel=SMC_KERNEL_RW, Lmax=512, RmaxRec=128,
                   test_fn=None, E2=0.90, burn_in=0, stream=None):
    """Algorithm 3: an adaptive run with key (seed, run), then its design
    replayed with key (seed2, run).  Returns (record1, record2, seconds[2])."""
    import numpy as np
    tf = SMC_TEST_PARAMS if test_fn is None else test_fn
    r1 = Record(model, pop.J, Lmax, RmaxRec, test_fn=test_fn)
    r2 = Record(model, pop.J, Lmax, RmaxRec, test_fn=test_fn)
    cfg = RunConfig(pop.J, pop.N, Rng(seed, run), check_every, force_every, D1, D2, Rbar, kappa,
                    stop_rule, E1, Rmax, scheme, kernel, 0, Lmax, RmaxRec, pop.max_chunk, tf, 0,
                    E2, burn_in)
    secs = np.zeros(2)
    _check(lib().smc_run_hybrid(model.h, C.byref(pop.c), C.byref(cfg), C.c_uint64(seed2),
                                C.byref(r1.c), C.byref(r2.c), secs.ctypes.data, _stream(stream)),
           "smc_run_hybrid")
    return r1, r2, secs


def hybrid_report(r1, r2, secs=None, stream=None):
    """Table 2's rows for the two steps, and the standardised differences of
    their log-ML (and log score) estimates, |a - b| / sqrt(NSE_a^2 + NSE_b^2)
    (smc_hybrid_report)."""
    import numpy as np
    z = np.zeros(2)
    _check(lib().smc_hybrid_report(C.byref(r1.c), C.byref(r2.c), z.ctypes.data, _stream(stream)),
           "smc_hybrid_report")
    rows = []
    for k, r in enumerate((r1, r2)):
        s = r.summary()
        rows.append(dict(step=k + 1, seconds=None if secs is None else float(secs[k]),
                         cycles=s["L"], metropolis_steps=s["mh_steps"], log_ml=s["log_ml"],
                         nse=s["nse"], log_score=s["log_score"][0],
                         log_score_nse=s["log_score"][1]))
    return dict(steps=rows, z_log_ml=float(z[0]), z_log_score=float(z[1]))


def smc_run_batch(models, pops, seeds, runs=None, records=None, replay=False, waves=0,
                  Rbar=7, kappa=3, D1=0.5, D2=0.2, Lmax=1024, RmaxRec=64, bws=None,
                  timing=0, kernel=SMC_KERNEL_RW, stream=None):
    """Many runs together (see smc_run_batch in include/smc.h); returns the
    records.  With replay=True the records' designs are replayed.  `bws`
    (a device uint8 tensor of smc_batch_ws_bytes(n) + 256 bytes) may be
    given to keep the batch workspace alive, e.g. across graph replays.
    With timing = k > 0 the first k persistent M-step launches are timed;
    then (records, dict(ms=[...], evals=[[egarch1, egarch2t], ...])) is
    returned."""
    import numpy as np
    n = len(models)
    runs = runs if runs is not None else [0] * n
    if records is None:
        records = [Record(m, p.J, Lmax, RmaxRec) for m, p in zip(models, pops)]
    cfgs = (RunConfig * n)()
    recs = (RunRecord * n)()
    for i in range(n):
        r = records[i]
        cfgs[i] = RunConfig(pops[i].J, pops[i].N, Rng(seeds[i], runs[i]), 1, 0, D1, D2, Rbar,
                            kappa, 0, 0.35, 100, SMC_RESAMPLE_RESIDUAL, kernel,
                            1 if replay else 0, r.Lmax, r.RmaxRec, pops[i].max_chunk,
                            SMC_TEST_PARAMS, 0, 0.90, 0)
        recs[i] = r.c
    hs = (_vp * n)(*[m.h.value for m in models])
    ps = (C.POINTER(Particles) * n)(*[C.pointer(p.c) for p in pops])
    nb = lib().smc_batch_ws_bytes(n)
    if bws is None:
        bws = torch.empty(nb + 256, dtype=torch.uint8, device=models[0].device)
    off = (-bws.data_ptr()) % 256
    tms = np.zeros(max(timing, 1), dtype=np.float32)
    tev = np.zeros((max(timing, 1), 2), dtype=np.int64)
    tim = BatchTiming(timing, 0, tms.ctypes.data, tev.ctypes.data) if timing > 0 else None
    _check(lib().smc_run_batch(n, hs, ps, cfgs, recs, C.c_void_p(bws.data_ptr() + off), nb, waves,
                               C.byref(tim) if tim is not None else None, _stream(stream)),
           "smc_run_batch")
    for i in range(n):
        records[i].c = recs[i]
        records[i].batch_ws = bws  # the stream may still read it
    if tim is not None:
        k = tim.launches
        return records, dict(ms=tms[:k].astype(np.float64).tolist(), evals=tev[:k].tolist())
    return records
