"""Constants compiled into the HIP kernels, checked on the CPU against the
mathematics they stand for.

kExp2Coef (model.h): the FP64 base-2 exponential's polynomial on
[-1/2, 1/2]; its relative error against 2^f (50-digit arithmetic) must stay
below 4e-17, a third of an ulp, and it must be exact at f = 0.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL_H = os.path.join(ROOT, "paper_1304_4334_amd", "csrc", "model.h")


def _exp2_coefficients():
    src = open(MODEL_H).read()
    m = re.search(r"kExp2Coef\[(\d+)\]\s*=\s*\{([^}]*)\}", src)
    assert m, "kExp2Coef not found"
    vals = [float.fromhex(v.strip()) for v in m.group(2).split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return vals


def test_exp2_polynomial_error_below_a_third_of_an_ulp():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    c = [mp.mpf(x) for x in _exp2_coefficients()]
    assert c[0] == 1
    worst = 0
    for k in range(4001):
        f = mp.mpf(-0.5) + mp.mpf(k) / 4000
        worst = max(worst, abs(mp.polyval(c[::-1], f) / mp.power(2, f) - 1))
    assert worst < 4e-17, worst


def test_exp2_coefficients_near_taylor():
    # the minimax polynomial stays close to the series of 2^f = e^(f ln 2),
    # the more so the lower the degree: a misplaced or mistyped coefficient
    # shows here
    import math
    c = _exp2_coefficients()
    bound = [1e-15, 1e-15, 1e-14, 1e-13, 1e-11, 1e-10, 1e-8, 1e-7, 1e-5, 1e-4, 1e-2, 1e-2]
    for k, ck in enumerate(c):
        taylor = math.log(2) ** k / math.factorial(k)
        assert abs(ck / taylor - 1) < bound[k], (k, ck, taylor)
