"""CPU checks of the C ABI: the library loads, exports every function the
header declares, validates arguments on the host, and the Python structs
match the C layout.  No call here reaches the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1304_4334_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = S._lib.lib()
    names = _declared()
    assert "smc_init_from_prior" in names and "smc_log_ml" in names
    for n in ["smc_init_from_prior", "smc_correct", "smc_resample", "smc_mutate", "smc_loglik",
              "smc_loglik_backward", "smc_log_ml"]:
        assert n in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_sizes_match_header_layout():
    assert C.sizeof(S._lib.ModelDesc) == 6 * 4 + 8 + 3 * 8
    assert C.sizeof(S._lib.Particles) == 8 + 8 * 8 + 8
    assert C.sizeof(S._lib.Rng) == 16
    assert S._lib.RunConfig.max_chunk.offset % 8 == 0
    assert S._lib.RunConfig.burn_in.offset == C.sizeof(S._lib.RunConfig) - 8
    assert S._lib.RunRecord.mean.offset == C.sizeof(S._lib.RunRecord) - 8


def _desc(**kw):
    base = dict(kind=S.SMC_MODEL_EGARCH, K=1, shock=0, nreg=0, precision=0, ncomp=0, T=10,
                y=C.c_void_p(0x1000), y32=None, X=None)
    base.update(kw)
    return S._lib.ModelDesc(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(T=0), -1), (dict(y=None), -1), (dict(kind=7), -1), (dict(K=3), -2),
    (dict(precision=1), -1), (dict(ncomp=1), -1), (dict(shock=5), -1),
    (dict(shock=2, ncomp=1), -2), (dict(shock=2, ncomp=5), -2), (dict(shock=2, K=5, ncomp=3), -2),
    (dict(kind=1, nreg=3, X=C.c_void_p(0x1000), ncomp=2), -1),
    (dict(kind=1, nreg=3, X=None), -1), (dict(kind=1, nreg=9, X=C.c_void_p(0x1000)), -2),
    (dict(kind=1, nreg=3, X=C.c_void_p(0x1000), precision=1), -2),
])
def test_model_create_validates(kw, status):
    L = S._lib.lib()
    h = C.c_void_p()
    assert L.smc_model_create(C.byref(_desc(**kw)), C.byref(h)) == status
    assert L.smc_last_error()


def test_model_dims_and_workspace():
    L = S._lib.lib()
    for kw, d, s in [(dict(), 5, 2), (dict(K=2, shock=1), 9, 3),
                     (dict(K=2, shock=2, ncomp=3), 17, 3), (dict(K=4, shock=2, ncomp=4), 26, 5),
                     (dict(kind=1, nreg=3, X=C.c_void_p(0x1000)), 4, 0)]:
        h = C.c_void_p()
        assert L.smc_model_create(C.byref(_desc(**kw)), C.byref(h)) == 0
        assert L.smc_model_dim(h) == d and L.smc_model_state_dim(h) == s
        w1 = L.smc_workspace_bytes(h, 4, 256, 16)
        w2 = L.smc_workspace_bytes(h, 4, 256, 32)
        assert w2 - w1 == 16 * 1024 * 8
        assert L.smc_workspace_bytes(h, 0, 256, 16) == 0
        L.smc_model_destroy(h)
    assert L.smc_model_dim(None) == -1


def test_number_of_test_functions():
    L = S._lib.lib()
    for kw, want in [(dict(), 2), (dict(K=2, shock=1), 2), (dict(K=2, shock=2, ncomp=3), 3),
                     (dict(kind=1, nreg=3, X=C.c_void_p(0x1000)), 4)]:
        h = C.c_void_p()
        assert L.smc_model_create(C.byref(_desc(**kw)), C.byref(h)) == 0
        assert L.smc_num_test_functions(h, S.SMC_TEST_MODEL) == want
        assert L.smc_num_test_functions(h, S.SMC_TEST_PARAMS) == L.smc_model_dim(h)
        assert L.smc_num_test_functions(h, 7) == -1
        L.smc_model_destroy(h)
    assert L.smc_num_test_functions(None, 0) == -1


def test_log_score_needs_a_cycle_ending_at_the_burn_in():
    L = S._lib.lib()
    t_end = (C.c_int64 * 3)(40, 100, 200)
    fake = C.c_void_p(0x1000)
    assert L.smc_log_score(3, 4, fake, t_end, 70, fake, None) == -1
    assert L.smc_log_score(3, 4, fake, t_end, 200, fake, None) == -1
    assert L.smc_log_score(0, 4, fake, t_end, 40, fake, None) == -1


def test_host_side_argument_errors():
    L = S._lib.lib()
    assert L.smc_log_ml(0, 4, C.c_void_p(0x1000), C.c_void_p(0x1000), None) == -1
    assert L.smc_log_ml(2, 1, C.c_void_p(0x1000), C.c_void_p(0x1000), None) == -1
    assert L.smc_adapt_scale(None, 10, 250, C.c_void_p(0x1000), None) == -1
    h = C.c_void_p()
    assert L.smc_model_create(C.byref(_desc()), C.byref(h)) == 0
    pop = S._lib.Particles(1, 8, *([C.c_void_p(0x1000)] * 8), 1 << 20)
    assert L.smc_init_from_prior(h, C.byref(pop), S._lib.Rng(1, 0), None) == -1  # J < 2
    pop.J = 2
    pop.ws = C.c_void_p(0x1001)
    assert L.smc_resample(h, C.byref(pop), 0, S._lib.Rng(1, 0), 1, None) == -1  # misaligned
    pop.ws = C.c_void_p(0x1000)
    pop.ws_bytes = 16
    assert L.smc_resample(h, C.byref(pop), 0, S._lib.Rng(1, 0), 1, None) == -5  # too small
    assert L.smc_mutate(h, C.byref(pop), 5, 1, C.c_void_p(0x1000), S._lib.Rng(1, 0), 1, 1,
                        C.c_void_p(0x1000), None, None) == -5  # no room for checkpoints
    pop.grad = None
    assert L.smc_mutate(h, C.byref(pop), 5, 1, C.c_void_p(0x1000), S._lib.Rng(1, 0), 1, 1,
                        C.c_void_p(0x1000), None, None) == -1  # Langevin needs the gradient
    assert L.smc_mutate(h, C.byref(pop), 5, 7, C.c_void_p(0x1000), S._lib.Rng(1, 0), 1, 1,
                        C.c_void_p(0x1000), None, None) == -1  # unknown kernel
    assert L.smc_loglik(h, 4, C.c_void_p(0x1000), 11, C.c_void_p(0x1000), None, None) == -1
    assert L.smc_status_string(-4) == b"numerical failure"
    L.smc_model_destroy(h)
