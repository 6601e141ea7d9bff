"""Constants compiled into the HIP kernels, checked on the CPU against the
mathematics they stand for.

kExp2Coef (model.h): the FP64 base-2 exponential's polynomial on
[-1/2, 1/2]; its relative error against 2^f (50-digit arithmetic) must stay
below 4e-17, a third of an ulp, and it must be exact at f = 0.

kLn2Hi / kLn2Lo (model.h): ln 2 split over two doubles for the weights'
exponential, whose arithmetic is replayed here against long double.

kLgHalf and t_log_const (model.h): the Student-t density's constant
log Gamma((nu+1)/2) - log Gamma(nu/2) - log(pi (nu - 2))/2 by an upward shift
and Stirling's series.  The coefficients must be the series' own (Bernoulli
numbers, rounded to double), and the device's double arithmetic, replayed
here in the same order, must stay within 4e-15 of the exact constant
(100-digit arithmetic) from nu just above 2 to nu = 1e40.
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


KERNELS_HIP = MODEL_H  # the weights' exponential sits beside the recursion's


def _ln2_split():
    src = open(KERNELS_HIP).read()
    m = re.search(r"kLn2Hi\s*=\s*([0-9a-fA-Fx.p+-]+)\s*,\s*kLn2Lo\s*=\s*([0-9a-fA-Fx.p+-]+)\s*;", src)
    assert m, "kLn2Hi / kLn2Lo not found"
    return float.fromhex(m.group(1)), float.fromhex(m.group(2))


def test_ln2_split_sums_to_ln2():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    hi, lo = _ln2_split()
    assert hi == float(mp.log(2))
    assert abs(mp.mpf(hi) + mp.mpf(lo) - mp.log(2)) < mp.mpf(2) ** -105


def test_exp_nonpos_error_within_two_ulp(tmp_path):
    """The weights' exponential (model.h, exp_nonpos), replayed on the CPU
    with the same constants and fused multiply-adds, against long double
    expl on [-708, 0]; -inf gives 0 and 0 gives 1."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    hi, lo = _ln2_split()
    m = re.search(r"kLog2e\s*=\s*([0-9.]+)\s*;", open(MODEL_H).read())
    assert m, "kLog2e not found"
    log2e = float(m.group(1)).hex()
    coef = ", ".join(c.hex() for c in _exp2_coefficients())
    src = f"""
#include <math.h>
#include <stdio.h>
static const double C[12] = {{{coef}}};
static double e_np(double x) {{
  double xc = fmax(x, -1100.0);
  double n = rint(xc * {log2e});
  double r = fma(-n, {lo.hex()}, fma(-n, {hi.hex()}, xc));
  double f = r * {log2e};
  double p = fma(C[11], f, C[10]);
  for (int k = 9; k >= 0; --k) p = fma(p, f, C[k]);
  return x < -1100.0 ? 0.0 : ldexp(p, (int)n);
}}
int main(void) {{
  double worst = 0.0;
  unsigned long long s = 12345;
  for (int i = 0; i < 2000000; ++i) {{
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    double u = (double)(s >> 11) * 0x1.0p-53;
    double x = (i & 3) ? -708.0 * u : -2.0 * u;
    long double ref = expl((long double)x);
    double y = e_np(x);
    double ulp = nextafter((double)ref, INFINITY) - (double)ref;
    double err = fabs((double)((long double)y - ref)) / ulp;
    if (err > worst) worst = err;
  }}
  printf("%.6f %.17g %.17g\\n", worst, e_np(-INFINITY), e_np(0.0));
  return 0;
}}
"""
    c_file = tmp_path / "e.c"
    c_file.write_text(src)
    exe = tmp_path / "e"
    subprocess.run(["gcc", "-O2", "-o", str(exe), str(c_file), "-lm"], check=True)
    worst, at_neg_inf, at_zero = map(float, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.split())
    assert worst < 2.0, worst
    assert at_neg_inf == 0.0 and at_zero == 1.0


def _lghalf_coefficients():
    src = open(MODEL_H).read()
    m = re.search(r"kLgHalf\[(\d+)\]\s*=\s*\{([^}]*)\}", src)
    assert m, "kLgHalf not found"
    vals = [float.fromhex(v.strip()) for v in m.group(2).split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return vals


def test_t_constant_series_coefficients_are_the_bernoulli_terms():
    from fractions import Fraction as F
    bern = {2: F(1, 6), 4: F(-1, 30), 6: F(1, 42), 8: F(-1, 30), 10: F(5, 66),
            12: F(-691, 2730), 14: F(7, 6), 16: F(-3617, 510)}
    got = _lghalf_coefficients()
    for j, k in enumerate(range(1, 17, 2)):
        want = (F(1, 2 ** k) - 2) * bern[k + 1] / (k * (k + 1))
        assert got[j] == float(want), (k, got[j], float(want))


def _t_log_const_replayed(nu):
    """t_log_const's double arithmetic in the device's order (libm's log)."""
    import math
    c = _lghalf_coefficients()
    x = 0.5 * nu
    xs = min(x, 2.0 ** 100)
    num, den = xs + 0.5, xs
    for k in range(1, 8):
        num *= xs + (k + 0.5)
        den *= xs + k
    y = x + 8.0
    iy = 1.0 / y
    w = iy * iy
    s = c[7]
    for j in range(6, -1, -1):
        s = math.fma(s, w, c[j]) if hasattr(math, "fma") else s * w + c[j]
    r = den / num
    v = 0.5 * math.log(y * r * r / (math.pi * (nu - 2.0)))
    return s * iy + v


def test_t_constant_within_4e15_of_the_exact_value():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 100  # the two log-gammas reach 1e42 at nu = 1e40
    worst = 0.0
    nus = [2.0 + 10.0 ** e for e in range(-12, 41)]
    nus += [2.0 + 0.37 * k for k in range(1, 400)]
    for nu in nus:
        n = mp.mpf(nu)
        exact = mp.loggamma((n + 1) / 2) - mp.loggamma(n / 2) - mp.log(mp.pi * (n - 2)) / 2
        worst = max(worst, abs(float(exact - mp.mpf(_t_log_const_replayed(nu)))))
    assert worst < 4e-15, worst
