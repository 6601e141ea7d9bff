"""The allocation-free particle moments (smc_particle_moments_noalloc) against
smc_particle_moments, which runs the same kernels on the population's
workspace: mean, variance and h L equal to the bit, on two calls in a row
(the second with a smaller, ragged population, so stale partials of the
first call in the static scratch would show), for 16-wide (d = 9) and
32-wide (d = 17) moment matrices, with the population's workspace pointer
NULL for the allocation-free call.
"""
import ctypes as C

import pytest
import torch

import paper_1304_4334_amd as S
import synthdata as SD
from paper_1304_4334_amd import _lib

pytestmark = pytest.mark.gpu


def _moments(fn, m, pop, pc, mh0):
    d = m.d
    mh = torch.full((1,), mh0, dtype=torch.int32, device="cuda")
    mean = torch.full((d,), float("nan"), dtype=torch.float64, device="cuda")
    cov = torch.full((d, d), float("nan"), dtype=torch.float64, device="cuda")
    hl = torch.full((d, d), float("nan"), dtype=torch.float64, device="cuda")
    st = fn(m.h, C.byref(pc), C.c_void_p(mh.data_ptr()), C.c_void_p(mean.data_ptr()),
            C.c_void_p(cov.data_ptr()), C.c_void_p(hl.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == S.SMC_OK, _lib.lib().smc_last_error().decode()
    torch.cuda.synchronize()
    return mean, cov, hl, mh


@pytest.mark.parametrize("name", ["egarch2t", "egarch23"])
def test_noalloc_moments_equal_workspace_moments(name):
    L = _lib.lib()
    w = SD.workload(name, T=64)
    m = S.Model.from_workload(w)
    print(f"[noalloc] {name} d={m.d}", flush=True)
    for call, (J, N, seed, mh0) in enumerate(((64, 1024, 3, 5), (5, 333, 4, 7))):
        pop = S.Population(m, J, N)
        S.smc_init_from_prior(m, pop, seed)
        torch.cuda.synchronize()
        ref = _moments(L.smc_particle_moments, m, pop, pop.c, mh0)
        bare = _lib.Particles.from_buffer_copy(pop.c)
        bare.ws = None
        bare.ws_bytes = 0
        got = _moments(L.smc_particle_moments_noalloc, m, pop, bare, mh0)
        for a, b, what in zip(ref, got, ("mean", "cov", "hchol", "mh")):
            assert torch.equal(a, b), (name, call, what)
        assert torch.isfinite(got[2]).all() and got[2][0, 0] > 0
        assert int(got[3].item()) == mh0


def test_noalloc_moments_reject_bad_arguments():
    L = _lib.lib()
    w = SD.workload("egarch11", T=32)
    m = S.Model.from_workload(w)
    pop = S.Population(m, 4, 64)
    bare = _lib.Particles.from_buffer_copy(pop.c)
    bare.J = 1
    mh = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    hl = torch.zeros((m.d, m.d), dtype=torch.float64, device="cuda")
    st = L.smc_particle_moments_noalloc(m.h, C.byref(bare), C.c_void_p(mh.data_ptr()), None, None,
                                        C.c_void_p(hl.data_ptr()), None)
    assert st == S.SMC_E_INVALID_ARG
