// Device-side models: priors, prior simulation and the per-observation
// likelihood recursion (Section 5.1 for EGARCH; the conjugate Gaussian
// regression as the closed-form test model).
//
// A model type M provides
//   M::D, M::S           parameter and state dimensions (compile time)
//   M::R, M::Y           recursion arithmetic and observation type
//   M::Par               per-particle constants prepared once per evaluation
//   M::params(th)        transform theta (FP64) to Par
//   M::logprior(th)      log prior density of theta (FP64)
//   M::prior_draw(...)   theta ~ p(theta) from the particle's Philox stream
//   M::advance(...)      sum over s = t0+1..t1 of log p(y_s | y_{1:s-1}, theta),
//                        advancing the state held in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "common.h"
#include "rng.h"

namespace smc {

constexpr double kLog2Pi = 1.8378770664093453390819;
constexpr double kSqrt2OverPi = 0.79788456080286535588;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2e = 1.4426950408889634074;
// Per-observation terms are summed in the recursion's precision over groups
// of kAcc observations before each group's sum is added to FP64
// accumulators.  kUnroll is the default number of observations whose loads
// are issued together; the loads of the next batch are in flight while the
// current one is processed.  The batch size does not change the arithmetic.
constexpr int kAcc = 8;
constexpr int kUnroll = 8;

// 2^x.  FP32: the hardware base-2 exponential.  FP64: x = n + f with
// n = rint(x), |f| <= 1/2, 2^f by the degree-11 minimax polynomial of
// kExp2Coef (relative error 3.4e-17 on [-1/2, 1/2] with the coefficients
// rounded to double; written by gen_exp2_coef.py), then scaled by 2^n.
// Arguments beyond the double range give 0 or inf through the final scaling.
//
// exp2_fast evaluates the polynomial as two Horner chains in f^2 (even and
// odd coefficients) joined by one fma: 12 operations, 7 deep, for values on
// a loop-carried dependency chain.  exp2_lean is plain Horner (11 fmas, 11
// deep) for independent values whose latencies overlap.
__device__ constexpr double kExp2Coef[12] = {
  0x1.0000000000000p+0,
  0x1.62e42fefa39efp-1,
  0x1.ebfbdff82c5adp-3,
  0x1.c6b08d7049fd1p-5,
  0x1.3b2ab6fb9f413p-7,
  0x1.5d87fe78cf26dp-10,
  0x1.43091310bf6b0p-13,
  0x1.ffcbfba7b89b6p-17,
  0x1.62bfc3c1c8a7cp-20,
  0x1.b526788b3b73dp-24,
  0x1.e620fb765be15p-28,
  0x1.e7aa0f6005d3cp-32,
};
// e^x for x <= 0 or -inf (weights relative to their maximum; -inf gives 0): x =
// n ln 2 + r with n = rint(x log2 e) and r reduced against ln 2 split in two
// doubles (|r| <= ln2/2, the first fma exact to one rounding of r), then
// 2^(r log2 e) by the minimax polynomial of kExp2Coef and the scaling by 2^n.
// About 20 operations against the library's 45; error within 2 ulp.
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;
__device__ __forceinline__ double exp_nonpos(double x) {
  const double xc = fmax(x, -1100.0);  // keeps -inf out of the reduction
  const double n = __builtin_rint(xc * kLog2e);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, xc));
  const double f = r * kLog2e;
  double p = fma(kExp2Coef[11], f, kExp2Coef[10]);
#pragma unroll
  for (int k = 9; k >= 0; --k) p = fma(p, f, kExp2Coef[k]);
  return x < -1100.0 ? 0.0 : __builtin_ldexp(p, (int)n);
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float exp2_lean(float x) { return __builtin_amdgcn_exp2f(x); }
// 2^(x - n) with n = rint(x) returned through n_out, so that callers can fold
// the exact scaling by 2^n into another operand off the dependency chain.
__device__ __forceinline__ double exp2_frac(double x, int &n_out) {
  const double n = __builtin_rint(x);
  const double f = x - n;
  const double u = f * f;
  double e = fma(kExp2Coef[10], u, kExp2Coef[8]), o = fma(kExp2Coef[11], u, kExp2Coef[9]);
  e = fma(e, u, kExp2Coef[6]);
  o = fma(o, u, kExp2Coef[7]);
  e = fma(e, u, kExp2Coef[4]);
  o = fma(o, u, kExp2Coef[5]);
  e = fma(e, u, kExp2Coef[2]);
  o = fma(o, u, kExp2Coef[3]);
  e = fma(e, u, kExp2Coef[0]);
  o = fma(o, u, kExp2Coef[1]);
  n_out = (int)n;
  return fma(o, f, e);
}
__device__ __forceinline__ double exp2_fast(double x) {
  int n;
  const double p = exp2_frac(x, n);
  return __builtin_ldexp(p, n);
}
__device__ __forceinline__ double exp2_lean(double x) {
  const double n = __builtin_rint(x);
  const double f = x - n;
  double p = fma(kExp2Coef[11], f, kExp2Coef[10]);
#pragma unroll
  for (int k = 9; k >= 0; --k) p = fma(p, f, kExp2Coef[k]);
  return __builtin_ldexp(p, (int)n);
}

// log2 x.  FP32: the hardware base-2 logarithm; FP64: the library's.
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double log2_fast(double x) { return log2(x); }

// Student-t kernel term log(1 + e^2/(nu - 2)): FP64 log1p; FP32 log2 (scaled
// by ln 2 at the end).
__device__ __forceinline__ double t_term(double e2, double inu2) { return log1p(e2 * inu2); }
__device__ __forceinline__ float t_term(float e2, float inu2) {
  return __builtin_amdgcn_logf(fmaf(e2, inu2, 1.0f));
}
template <typename R>
__device__ __forceinline__ double t_scale();
template <>
__device__ __forceinline__ double t_scale<double>() { return 1.0; }
template <>
__device__ __forceinline__ double t_scale<float>() { return kLn2; }

__device__ __forceinline__ double normal_logpdf_std(double z) { return -0.5 * kLog2Pi - 0.5 * z * z; }

// The Student-t density's per-observation constant
//   log Gamma((nu + 1)/2) - log Gamma(nu/2) - log(pi (nu - 2)) / 2,   nu > 2,
// without the library's branchy lgamma.  With x = nu/2 >= 1, the recurrence
// log Gamma(z + 1) = log Gamma(z) + log z moves both arguments up by 8:
//   D(x) = D(x + 8) - log prod_{k<8} (x + k + 1/2) / (x + k),
// D(z) = log Gamma(z + 1/2) - log Gamma(z).  At y = x + 8 >= 9 Stirling's
// series, with the Bernoulli polynomials at 1/2 and at 0, gives
//   D(y) = log(y)/2 + sum over odd k of (2^-k - 2) B_{k+1} / (k (k+1) y^k);
// kLgHalf holds those coefficients for k = 1, 3, ..., 15 (the first omitted
// term is below 3e-17 at y = 9).  All logarithms are taken at once, of
// y r^2 / (pi (nu - 2)) with r the products' ratio.  Beyond x = 2^100 the
// ratio is 1 to rounding (and its products would overflow), so the
// products use min(x, 2^100).
__device__ constexpr double kLgHalf[8] = {
  -0x1.0000000000000p-3,
  0x1.5555555555555p-8,
  -0x1.999999999999ap-10,
  0x1.36db6db6db6dbp-10,
  -0x1.b8e38e38e38e4p-10,
  0x1.f68ba2e8ba2e9p-9,
  -0x1.a413b13b13b14p-7,
  0x1.e426888888889p-5,
};
__device__ __forceinline__ double t_log_const(double nu) {
  const double x = 0.5 * nu;
  const double xs = fmin(x, 0x1p100);
  double num = xs + 0.5, den = xs;
#pragma unroll
  for (int k = 1; k < 8; ++k) {
    num *= xs + (k + 0.5);
    den *= xs + k;
  }
  const double y = x + 8.0, iy = 1.0 / y, w = iy * iy;
  double s = kLgHalf[7];
#pragma unroll
  for (int j = 6; j >= 0; --j) s = fma(s, w, kLgHalf[j]);
  const double r = den / num;
  return fma(s, iy, 0.5 * log(y * r * r / (M_PI * (nu - 2.0))));
}

// Distribution function of the unit-variance Student-t shock at x, with
// nu2 = nu - 2.  The shock is z sqrt(nu2 / nu) with z ~ t_nu, and
// P(t_nu < z) = I_w(nu/2, 1/2) / 2 for z < 0 with w = nu / (nu + z^2)
// (DLMF 8.17.22's relation); in terms of x, w = nu2 / (nu2 + x^2), and
// symmetry gives x >= 0.  The regularised incomplete beta function is the
// continued fraction of DLMF 8.17.22 summed by the modified Lentz method, at
// (nu/2, 1/2, w) or, where that converges slowly (w > (a + 1) / (a + b + 2)),
// at (1/2, nu/2, 1 - w) through I_w(a, b) = 1 - I_{1-w}(b, a).  Both share
// the prefactor w^(nu/2) (1 - w)^(1/2) / B(nu/2, 1/2), whose log-beta is the
// t density's constant plus log(nu2)/2.  log w and log(1 - w) are formed
// from nu2, x^2 and their sum, so neither cancels.  At most 4,096 terms: a
// few hundred suffice for any nu the prior reaches.
__device__ inline double t_unit_cdf(double x, double nu2) {
  if (isinf(x)) return x < 0.0 ? 0.0 : 1.0;
  const double r = nu2 + x * x, lr = log(r);
  const double lw = log(nu2) - lr, l1w = 2.0 * log(fabs(x)) - lr;
  const double ha = 0.5 * (nu2 + 2.0);
  const bool swap = nu2 * (ha + 2.5) > (ha + 1.0) * r;
  const double a = swap ? 0.5 : ha, b = swap ? ha : 0.5;
  const double xw = swap ? x * x / r : nu2 / r;
  double f = 1.0, c = 1.0, dd = 0.0;
  for (int j = 1; j <= 4096; ++j) {
    const double m = (double)(j >> 1), a2m = a + 2.0 * m;
    const double dj = (j & 1) ? -(a + m) * (a + b + m) * xw / (a2m * (a2m + 1.0))
                              : m * (b - m) * xw / ((a2m - 1.0) * a2m);
    dd = fma(dj, dd, 1.0);
    if (fabs(dd) < 1e-300) dd = 1e-300;
    c = 1.0 + dj / c;
    if (fabs(c) < 1e-300) c = 1e-300;
    dd = 1.0 / dd;
    f *= c * dd;
    if (fabs(c * dd - 1.0) < 1e-16) break;
  }
  const double lib = t_log_const(nu2 + 2.0) + 0.5 * log(nu2);
  const double I = exp(fma(ha, lw, 0.5 * l1w) + lib) / (a * f);
  const double tail = 0.5 * (swap ? 1.0 - I : I);
  return x < 0.0 ? tail : 1.0 - tail;
}

// ---------------------------------------------------------------- EGARCH --
// theta = (th1, th2, th3_1..K, th4_1..K, th5_1..K, then th9 = log(nu - 2) for
// Student-t shocks or th6_1..I, th7_1..I, th8_1..I for normal-mixture shocks),
// mu_Y = th1/1000, sigma_Y = exp(th2), alpha_k = tanh(th3k), beta_k = exp(th4k),
// gamma_k = th5k (Table 1), nu = 2 + exp(th9) (an extension), and the mixture
// from p*_i = tanh(th6i) + 1, mu*_i = th7i, sigma*_i = exp(th8i) through the
// normalisation of eqs EGARCH_tran1/2.
constexpr double kMixTrunc = -3.0;  // Table 1: th8i truncated below here
// log P(Z >= -3) for a standard normal Z (correctly rounded).
constexpr double kLogMixMass = -0x1.621b527ca016fp-10;

template <int K_, int SHOCK_, typename R_, int I_ = 1>
struct Egarch {
  static constexpr int K = K_;
  static constexpr int I = I_;
  static constexpr bool kT = (SHOCK_ == SMC_SHOCK_STUDENT_T);
  static constexpr bool kMix = (SHOCK_ == SMC_SHOCK_MIXTURE);
  static_assert(!kMix || (I_ >= 2 && I_ <= 4), "mixtures of 2..4 components");
  static constexpr int D = 2 + 3 * K + (kT ? 1 : 0) + (kMix ? 3 * I : 0);
  static constexpr int S = K + 1;
  static constexpr int kNM = kMix ? I : 1;  // component arrays (unused if no mixture)
  // FP32 Student-t shocks: the factors 1 + eps^2/(nu - 2) of four
  // consecutive observations are multiplied before one log2 is taken (the
  // log2 runs at a quarter of the FP32 rate; four to a log2 measured 2% less
  // time per observation than two).  A group whose product exceeds the float
  // range (four shocks in a row beyond about 6.6e4 (nu - 2)^(1/2) standard
  // deviations) counts as a zero density.
  static constexpr bool kTProd = kT && sizeof(R_) == 4;
  static constexpr int kTGroup = 4;  // observations per log2 (divides kAcc)
  static_assert(kAcc % kTGroup == 0, "log2 groups inside accumulation groups");
  static constexpr bool kEps = sizeof(R_) == 4;  // the FP32 form of the step (see Par)
  using R = R_;
  using Y = R_;

  // Exponent form of the recursion.  With kappa = -log2(e)/2 and
  // w_k = kappa v_k, the scale factor is E_s = sigma_Y / h_s = 2^(sum_k w_ks),
  // the standardised shock is eps_s = z_s E_s with z_s = (y_s - mu_Y)/sigma_Y,
  // and since E_s > 0, |eps_s| = |z_s| E_s.  So eq EGARCH_mod1 reads
  //   w_k,s+1 = alpha_k w_ks - kappa beta_k sqrt(2/pi)
  //             + kappa (beta_k |z_s| + gamma_k z_s) E_s,
  // whose loop-carried chain is one exp2 and one fma; z_s and the bracket do
  // not depend on the recursion.  log h_s = log sigma_Y - ln2 sum_k w_ks.
  //
  // Mixture shocks: log2 of p_i phi(eps; mu_i, sigma_i^2) sqrt(2 pi) is
  // x_i = lw_i + nb_i (eps - mu_i)^2 with lw_i = log2(p_i / sigma_i) and
  // nb_i = -log2(e) / (2 sigma_i^2); the density's log2 is
  // m + log2 sum_i 2^(x_i - m), m = max_i x_i.  The sums are multiplied
  // over each block of observations (each lies in [1, I]) and one log2 is
  // taken per block.
  //
  // FP32 (kEps): the loop is bound by instruction issue rather than by its
  // chain, so each factor adds the shock terms directly,
  //   w_k,s+1 = (alpha_k w_ks - kappa beta_k c) + kappa gamma_k eps_s
  //             + kappa beta_k |eps_s|,
  // three fmas instead of four, with eps_s = z_s E_s formed once; and for
  // Student-t shocks z_s, hence eps_s, is scaled by q = (nu - 2)^(-1/2) (the
  // factor coefficients by 1/q), so 1 + eps^2/(nu - 2) is one fma.
  struct Par {
    R a[K], c0[K], kb[K], kg[K];  // alpha, -kappa beta c, kappa beta, kappa gamma
    R isig, mus;                  // 1/sigma_Y, mu_Y/sigma_Y
    R inu2;                       // 1/(nu - 2)
    R kbe[K], kge[K], isige, muse, uzs;  // kEps: kb/q, kg/q, q/sigma_Y, q mu_Y/sigma_Y, 1/q
    R lw[kNM], nb[kNM], mu[kNM];  // mixture components (see above)
    double lsig;                  // log sigma_Y
    double cst;                   // per-observation log-density constant
    double hnu1;                  // (nu + 1)/2
  };
  static constexpr double kKappa = -0.72134752044448170368;  // -log2(e)/2

  __device__ static const Y *ydata(const DevModel &m) {
    if constexpr (sizeof(R) == 4) return m.y32;
    else return m.y;
  }

  // Normalised mixture components (eqs EGARCH_tran1/2): weights p_i, means
  // mu_i and scales sigma_i, with mean 0 and variance 1.
  __device__ static void mixture(const double *th, double *pw, double *mu, double *sg) {
    constexpr int b = 2 + 3 * K;
    double ps = 0.0, pm = 0.0, q = 0.0;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      pw[i] = tanh(th[b + i]) + 1.0;
      ps += pw[i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      pw[i] /= ps;
      pm += pw[i] * th[b + I + i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      mu[i] = th[b + I + i] - pm;
      sg[i] = exp(th[b + 2 * I + i]);
      q += pw[i] * (mu[i] * mu[i] + sg[i] * sg[i]);
    }
    const double c = 1.0 / sqrt(q);
#pragma unroll
    for (int i = 0; i < I; ++i) {
      mu[i] *= c;
      sg[i] *= c;
    }
  }

  // Functions of interest of Section 5.2 at date t, from theta and the state
  // (v_1..v_K, eps_t): g1 = log sigma_Y + sum_k v_kt / 2 (log volatility);
  // for mixtures g2 = E(eps^3) = sum_i p_i (mu_i^3 + 3 mu_i sigma_i^2); and
  // g3 = P(Y_{t+1} < -0.03 | theta, y_{1:t}) = F((-0.03 - mu_Y) / h_{t+1})
  // with h_{t+1} one step of eq EGARCH_mod1 ahead (no innovation when t = 0)
  // and F the shock's distribution function.
  static constexpr int kTests = kMix ? 3 : 2;
  __device__ static void test_fns(const double *th, const R (&st)[S], int64_t t, double *g) {
    double vs = 0.0, vn = 0.0;
    const double e = (double)st[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double v = (double)st[k];
      vs += v;
      if (t >= 1)
        vn += tanh(th[2 + k]) * v + exp(th[2 + K + k]) * (fabs(e) - kSqrt2OverPi) +
              th[2 + 2 * K + k] * e;
    }
    int q = 0;
    g[q++] = th[1] + 0.5 * vs;
    const double x = (-0.03 - th[0] * 1e-3) / (exp(th[1]) * exp(0.5 * vn));
    if constexpr (kMix) {
      double pw[I], mu[I], sg[I];
      mixture(th, pw, mu, sg);
      double m3 = 0.0, F = 0.0;
#pragma unroll
      for (int i = 0; i < I; ++i) {
        m3 += pw[i] * (mu[i] * mu[i] * mu[i] + 3.0 * mu[i] * sg[i] * sg[i]);
        F += pw[i] * (0.5 * erfc(-(x - mu[i]) / (sg[i] * M_SQRT2)));
      }
      g[q++] = m3;
      g[q++] = F;
    } else if constexpr (kT) {
      g[q++] = t_unit_cdf(x, exp(th[2 + 3 * K]));
    } else {
      g[q++] = 0.5 * erfc(-x / M_SQRT2);
    }
  }

  __device__ static Par params(const double *th) {
    if constexpr (kEps) return params_f32(th);
    Par p;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double b = exp(th[2 + K + k]);
      p.a[k] = (R)tanh(th[2 + k]);
      p.c0[k] = (R)(-kKappa * b * kSqrt2OverPi);
      p.kb[k] = (R)(kKappa * b);
      p.kg[k] = (R)(kKappa * th[2 + 2 * K + k]);
    }
    const double isig = exp(-th[1]);
    p.isig = (R)isig;
    p.mus = (R)(th[0] * 1e-3 * isig);
    p.lsig = th[1];
    {
      const double q = kT ? exp(-0.5 * th[2 + 3 * K]) : 1.0;  // (nu - 2)^(-1/2)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        p.kbe[k] = (R)(kKappa * exp(th[2 + K + k]) / q);
        p.kge[k] = (R)(kKappa * th[2 + 2 * K + k] / q);
      }
      p.isige = (R)(isig * q);
      p.muse = (R)(th[0] * 1e-3 * isig * q);
      p.uzs = (R)(1.0 / q);
    }
    if constexpr (kT) {
      const double nu = 2.0 + exp(th[2 + 3 * K]);
      p.inu2 = (R)exp(-th[2 + 3 * K]);
      p.hnu1 = 0.5 * (nu + 1.0);
      p.cst = t_log_const(nu);
    } else if constexpr (kMix) {
      double pw[I], mu[I], sg[I];
      mixture(th, pw, mu, sg);
#pragma unroll
      for (int i = 0; i < I; ++i) {
        p.mu[i] = (R)mu[i];
        p.lw[i] = (R)(log2(pw[i]) - log2(sg[i]));
        p.nb[i] = (R)(-kLog2e / (2.0 * sg[i] * sg[i]));
      }
      p.inu2 = (R)0;
      p.hnu1 = 0.5;
      p.cst = -0.5 * kLog2Pi;
    } else {
      p.inu2 = (R)0;
      p.hnu1 = 0.5;
      p.cst = -0.5 * kLog2Pi;
    }
    return p;
  }
  // FP32 models: the coefficients that enter the float recursion are
  // computed in float (their float roundings were all that reached the
  // recursion anyway); the per-observation log-density constant, log sigma_Y
  // and (nu + 1)/2 stay FP64.
  __device__ static Par params_f32(const double *th) {
    Par p;
    const float kap = (float)kKappa;
    const float q = kT ? __expf(-0.5f * (float)th[2 + 3 * K]) : 1.0f;  // (nu - 2)^(-1/2)
    const float iq = 1.0f / q;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float b = __expf((float)th[2 + K + k]);
      const float x = (float)th[2 + k];  // tanh x = 1 - 2 / (e^(2x) + 1)
      p.a[k] = (R)(1.0f - 2.0f / (__expf(2.0f * x) + 1.0f));
      p.c0[k] = (R)(-kap * b * (float)kSqrt2OverPi);
      p.kb[k] = (R)(kap * b);
      p.kg[k] = (R)(kap * (float)th[2 + 2 * K + k]);
      p.kbe[k] = p.kb[k] * iq;
      p.kge[k] = p.kg[k] * iq;
    }
    const float isig = __expf(-(float)th[1]);
    p.isig = (R)isig;
    p.mus = (R)((float)(th[0] * 1e-3) * isig);
    p.isige = (R)(isig * q);
    p.muse = p.mus * q;
    p.uzs = iq;
    p.lsig = th[1];
    if constexpr (kT) {
      const double nu = 2.0 + exp(th[2 + 3 * K]);
      p.inu2 = (R)(q * q);
      p.hnu1 = 0.5 * (nu + 1.0);
      p.cst = t_log_const(nu);
    } else if constexpr (kMix) {
      double pw[I], mu[I], sg[I];
      mixture(th, pw, mu, sg);
#pragma unroll
      for (int i = 0; i < I; ++i) {
        p.mu[i] = (R)mu[i];
        p.lw[i] = (R)(log2(pw[i]) - log2(sg[i]));
        p.nb[i] = (R)(-kLog2e / (2.0 * sg[i] * sg[i]));
      }
      p.inu2 = (R)0;
      p.hnu1 = 0.5;
      p.cst = -0.5 * kLog2Pi;
    } else {
      p.inu2 = (R)0;
      p.hnu1 = 0.5;
      p.cst = -0.5 * kLog2Pi;
    }
    return p;
  }


  // Table 1 (and the nu extension): prior mean, standard deviation and its
  // logarithm of parameter i.  Hexadecimal literals are the correctly rounded
  // log(0.01), atanh(0.95), log(0.10), log(10) and log(0.2).
  __device__ __forceinline__ static void prior_moments(int i, double &mean, double &sd,
                                                       double &lsd) {
    sd = 1.0;
    lsd = 0.0;
    if (i == 0) mean = 0.0;
    else if (i == 1) mean = -0x1.26bb1bbb55515p+2;
    else if (i < 2 + K) mean = 0x1.d4ef968880dd4p+0;
    else if (i < 2 + 2 * K) mean = -0x1.26bb1bbb55515p+1;
    else if (i < 2 + 3 * K) { mean = 0.0; sd = 0.2; lsd = -0x1.9c041f7ed8d33p+0; }
    else if (kT) mean = 0x1.26bb1bbb55516p+1;
    else mean = 0.0;  // th6i, th7i, th8i
  }

  __device__ static double logprior(const double *th) {
    double lp = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double m, sd, lsd;
      prior_moments(i, m, sd, lsd);
      const double z = (th[i] - m) / sd;
      lp += normal_logpdf_std(z) - lsd;
    }
    if constexpr (kMix) {
#pragma unroll
      for (int i = 2 + 3 * K + 2 * I; i < D; ++i) {
        if (th[i] < kMixTrunc) return -INFINITY;
        lp -= kLogMixMass;
      }
    }
    return lp;
  }

  __device__ static void prior_draw(uint64_t seed, uint64_t run, uint64_t p, double *th) {
    double z[D];
    normals<D>(seed, run, p, 0, 0, kPrior, z, D);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double m, sd, lsd;
      prior_moments(i, m, sd, lsd);
      th[i] = m + sd * z[i];
    }
    if constexpr (kMix) {
      // Truncated th8i by rejection: attempt a redraws the normal vector on
      // counter (p, 0, a, PRIOR | block) and takes this parameter's entry;
      // after 32 failures the truncation point itself.
      for (int i = 2 + 3 * K + 2 * I; i < D; ++i) {
        for (uint64_t a = 1; th[i] < kMixTrunc && a <= 32; ++a) {
          normals<D>(seed, run, p, 0, a, kPrior, z, D);
          th[i] = z[i];
        }
        if (th[i] < kMixTrunc) th[i] = kMixTrunc;
      }
    }
  }

  // Loop state: the exponents w_k of the observation about to be processed
  // and their sum.
  struct Run {
    R w[K];
    R sw;
  };

  // The shock eps = z E of an observation from step()'s E and z (z scaled
  // by q in the kEps form).
  __device__ __forceinline__ static R shock(const Par &p, R z, R E) {
    if constexpr (kEps) return z * E * p.uzs;
    else return z * E;
  }

  // One observation: returns the exponent sum used (for log h), adds eps^2
  // (Gaussian), the Student-t term or the mixture's largest log2 term m to
  // ae (and multiplies the mixture's sum of 2^(x_i - m) into pm), reports E
  // and z (see shock()), and advances r to the next observation's exponents.
  __device__ __forceinline__ static R step(const Par &p, R y, Run &r, R &ae, R &pm, R &E_out,
                                           R &z_out) {
    const R sw = r.sw;
    if constexpr (kEps) {
      const R Ef = exp2_fast(sw);
      const R zq = fma(y, p.isige, -p.muse);
      const R e = zq * Ef;  // eps q
#pragma unroll
      for (int k = 0; k < K; ++k)
        r.w[k] = fma(p.kbe[k], fabs(e), fma(p.kge[k], e, fma(p.a[k], r.w[k], p.c0[k])));
      R sw1 = r.w[0];
#pragma unroll
      for (int k = 1; k < K; ++k) sw1 += r.w[k];
      r.sw = sw1;
      if constexpr (kTProd) {
        pm *= fma(e, e, (R)1);  // 1 + eps^2/(nu - 2); the caller takes the log2
      } else if constexpr (kMix) {
        R x[I];
#pragma unroll
        for (int i = 0; i < I; ++i) {
          const R dd = e - p.mu[i];
          x[i] = fma(p.nb[i] * dd, dd, p.lw[i]);
        }
        R mx = x[0];
#pragma unroll
        for (int i = 1; i < I; ++i) mx = fmax(mx, x[i]);
        R sm = exp2_lean(x[0] - mx);
#pragma unroll
        for (int i = 1; i < I; ++i) sm += exp2_lean(x[i] - mx);
        ae += mx;
        pm *= sm;
      } else {
        ae = fma(e, e, ae);
      }
      E_out = Ef;
      z_out = zq;
      return sw;
    } else {
      return step_chain(p, y, r, ae, pm, E_out, z_out);
    }
  }

  // FP64: the form whose loop-carried chain is one exp2 and one fma.
  __device__ __forceinline__ static R step_chain(const Par &p, R y, Run &r, R &ae, R &pm,
                                                 R &E_out, R &z_out) {
    const R sw = r.sw;
    // E = 2^sw.  For FP64 mixtures it is kept as Ef * 2^n: the exact scaling
    // by 2^n goes into the other factor of each product (off the
    // loop-carried chain, which then ends at the polynomial), giving the
    // same products.  Measured on the likelihood kernel at t = T, this is 3%
    // faster for egarch_23 and 3% slower for EGARCH(1,1), whose loop has
    // less to overlap the two extra scalings with.
    constexpr bool kSplit = std::is_same<R, double>::value && kMix;
    R Ef;
    int n = 0;
    if constexpr (kSplit) {
      Ef = exp2_frac(sw, n);
    } else {
      Ef = exp2_fast(sw);
    }
    const auto scaled = [&](R v) -> R {
      if constexpr (kSplit) return __builtin_ldexp(v, n);
      else return v;
    };
    const R z = fma(y, p.isig, -p.mus);
    // The next exponent sum.  FP64 forms it as one fma from the factors'
    // bracket and constant sums, which keeps the loop-carried chain at an
    // exp2 and an fma.  The FP32 loop is bound by instruction issue (the
    // exp2 and log2 run at a quarter of the rate), so it adds the new
    // exponents instead: K - 1 additions in place of 2K - 1 operations, at
    // the cost of one more dependent addition on the chain.  (The sums
    // start from the first factor's terms; an added zero would cost an
    // instruction.)
    constexpr bool kSumW = sizeof(R) == 4;
    R kk, AA;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R A = fma(p.a[k], r.w[k], p.c0[k]);
      const R kz = fma(p.kb[k], fabs(z), p.kg[k] * z);
      r.w[k] = fma(scaled(kz), Ef, A);
      if constexpr (!kSumW) {
        if (k == 0) {
          kk = kz;
          AA = A;
        } else {
          kk += kz;
          AA += A;
        }
      }
    }
    if constexpr (K == 1) {
      r.sw = r.w[0];
    } else if constexpr (kSumW) {
      R sw1 = r.w[0];
#pragma unroll
      for (int k = 1; k < K; ++k) sw1 += r.w[k];
      r.sw = sw1;
    } else {
      r.sw = fma(scaled(kk), Ef, AA);
    }
    const R e = scaled(z) * Ef;
    const R E = scaled(Ef);
    if constexpr (kTProd) {
      pm *= fma(e * e, p.inu2, (R)1);  // the caller takes the log2 (see kTProd)
    } else if constexpr (kT) {
      ae += t_term(e * e, p.inu2);
    } else if constexpr (kMix) {
      R x[I];
#pragma unroll
      for (int i = 0; i < I; ++i) {
        const R dd = e - p.mu[i];
        x[i] = fma(p.nb[i] * dd, dd, p.lw[i]);
      }
      R mx = x[0];
#pragma unroll
      for (int i = 1; i < I; ++i) mx = fmax(mx, x[i]);
      R sm = exp2_lean(x[0] - mx);
#pragma unroll
      for (int i = 1; i < I; ++i) sm += exp2_lean(x[i] - mx);
      ae += mx;
      pm *= sm;
    } else {
      ae = fma(e, e, ae);
    }
    E_out = E;
    z_out = z;
    return sw;
  }

  // Exponents of observation t0+1 from the state at t0 in the API's units,
  // (v_1..v_K, eps_t0).  The factors take no innovation at s = 1.
  __device__ __forceinline__ static void start(const Par &p, const R (&st)[S], int64_t t0,
                                               Run &r) {
    const R kap = (R)kKappa;
    if (t0 == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) r.w[k] = (R)0;
    } else {
      // w_k at t0+1 from (v_k, eps) at t0, in the model's own form
      const R e = st[K];
#pragma unroll
      for (int k = 0; k < K; ++k)
        r.w[k] = fma(p.kb[k], fabs(e), fma(p.kg[k], e, fma(p.a[k], kap * st[k], p.c0[k])));
    }
    R sw0 = r.w[0];
#pragma unroll
    for (int k = 1; k < K; ++k) sw0 += r.w[k];
    r.sw = sw0;
  }

  // Observation by observation: f(s, log p(y_s | y_{1:s-1}, theta)) for
  // s = t0+1..t1 (the C phase records running weights at check dates), with
  // the recursion kept in registers; g() after every 16 observations of the
  // batched loop (the C phase reduces its recorded weights there); st
  // receives the state at t1.
  template <class F, class G>
  __device__ static void scan(const Par &p, R (&st)[S], int64_t t0, int64_t t1,
                              const Y *__restrict__ y, F &&f, G &&g) {
    if (t1 <= t0) return;
    Run r;
    start(p, st, t0, r);
    const double base = p.cst - p.lsig;
    R wl[K], E = (R)1, z = (R)0;
    auto one = [&](int64_t s, R yv) {
#pragma unroll
      for (int k = 0; k < K; ++k) wl[k] = r.w[k];
      R ae = (R)0, pm = (R)1;
      const R sw = step(p, yv, r, ae, pm, E, z);
      if constexpr (kTProd) ae = log2_fast(pm);
      double ld;
      if constexpr (kT) ld = base + kLn2 * (double)sw - p.hnu1 * t_scale<R>() * (double)ae;
      else if constexpr (kMix) ld = base + kLn2 * ((double)sw + (double)ae + (double)log2_fast(pm));
      else ld = base + kLn2 * (double)sw - 0.5 * (double)ae;
      f(s, ld);
    };
    // Observations in batches of kUnroll whose loads are issued together,
    // the next batch's while the current one is processed.
    int64_t s = t0 + 1;
    const int64_t nbat = (t1 - t0) / kUnroll;
    if (nbat > 0) {
      // two buffers filled alternately, each batch's loads issued before the
      // previous batch is processed (see advance)
      R ya[kUnroll], yc[kUnroll];
#pragma unroll
      for (int i = 0; i < kUnroll; ++i) ya[i] = y[s - 1 + i];
      __asm__ volatile("" ::"s"(ya[0]), "s"(ya[kUnroll - 1]));
      int64_t b = 0;
      for (; b + 1 < nbat; b += 2, s += 2 * kUnroll) {
        __asm__ volatile("" ::"s"(ya[0]), "s"(ya[kUnroll - 1]));
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) yc[i] = y[s - 1 + kUnroll + i];
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) one(s + i, ya[i]);
        __asm__ volatile("" ::"s"(yc[0]), "s"(yc[kUnroll - 1]));
        const Y *pn = y + (s - 1) + (b + 2 < nbat ? 2 * kUnroll : kUnroll);
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) ya[i] = pn[i];
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) one(s + kUnroll + i, yc[i]);
        g();
      }
      if (b < nbat) {
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) one(s + i, ya[i]);
        s += kUnroll;
      }
    }
    for (; s <= t1; ++s) one(s, y[s - 1]);
    const R kap = (R)kKappa;
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = wl[k] / kap;
    st[K] = shock(p, z, E);
  }

  // Sum of log p(y_s | y_{1:s-1}, theta) over s = t0+1..t1.  st holds the
  // state at t0 in the API's units, (v_1..v_K, eps_t0), and receives the
  // state at t1.  The terms are summed in groups of kAcc; the observations
  // are loaded U at a time (U = 4, 8 or 16), each batch's loads issued
  // while the previous batch is processed.  U changes the schedule only:
  // every U gives the same operations in the same order.
  template <int U = kUnroll>
  __device__ static double advance(const Par &p, R (&st)[S], int64_t t0, int64_t t1,
                                   const Y *__restrict__ y) {
    static_assert(U == 4 || U == 8 || U == 16, "batches of 4, 8 or 16 observations");
    if (t1 <= t0) return 0.0;
    Run r;
    const R kap = (R)kKappa;
    start(p, st, t0, r);
    double sv = 0.0, se = 0.0;
    const Y *yp = y + t0;
    const int n = (int)(t1 - t0);
    const int nm = n - 1;  // all but the last observation
    const int nb = nm / kAcc;  // whole groups
    // group sums (carried across the two batches of a group when U = 4).
    // FP32 recursions carry them over two groups (kF) before adding them
    // to the FP64 totals: groups 2j and 2j + 1 form one span, the same for
    // every U, which halves the conversions and FP64 additions.
    constexpr int kF = sizeof(R) == 4 ? 2 : 1;  // groups per FP64 flush
    R av = (R)0, ae = (R)0, pm = (R)1;
    auto flush = [&]() {
      sv += (double)av;
      se += (double)ae;
      if constexpr (kMix) se += (double)log2_fast(pm);
      ae = (R)0;
      pm = (R)1;
    };
    constexpr int G = U < kAcc ? kAcc / U : 1;  // batches per group
    constexpr int Q = U > kAcc ? U / kAcc : 1;  // groups per batch
    const int nbat = nb * G / Q;  // whole batches (U = 16 may leave one group)
    // Batch b of observations; bp = b % 2 (with U = 4 a group spans batches
    // b and b + 1, b even, and godd is the parity of its group b / 2).
    auto batch = [&](const R(&yv)[U], int bp, int godd) {
#pragma unroll
      for (int i = 0; i < U; ++i) {
        R Ed, zd;
        const R sw = step(p, yv[i], r, ae, pm, Ed, zd);
        // position in the group, and the group's parity: batches of 16
        // hold groups 2j and 2j + 1, batches of 8 are groups (b even in
        // the first call of a pair), batches of 4 are told
        const int pos = (G > 1 ? bp * U : 0) + (i % kAcc);
        const int odd = Q > 1 ? (i / kAcc) & 1 : (G > 1 ? godd : bp);
        // the first term of a flush span starts its sum
        if (pos == 0 && (kF == 1 || !odd)) av = sw;
        else av += sw;
        if constexpr (kTProd) {
          if (pos % kTGroup == kTGroup - 1) {
            ae += log2_fast(pm);
            pm = (R)1;
          }
        }
        if (pos == kAcc - 1 && (kF == 1 || odd)) flush();
      }
    };
    static_assert(G <= 2, "a group spans at most two batches");
    if (nbat > 0) {
      // Two buffers of observations, filled alternately, so no copies
      // between batches.  Each batch's loads are issued before the previous
      // batch is processed (the observations are read-only, so the compiler
      // would otherwise place them just before their use).
      R ya[U], yc[U];
#pragma unroll
      for (int i = 0; i < U; ++i) ya[i] = yp[i];
      // the first batch is waited for here, so that the waits inside the
      // loop cover only what the loop itself loads
      __asm__ volatile("" ::"s"(ya[0]), "s"(ya[U - 1]));
      // A batch is waited for before the next one's loads are issued (a
      // wait covers every scalar load in flight), i.e. after a whole batch
      // of work since its own loads.
      int b = 0;
      for (; b + 1 < nbat; b += 2, yp += 2 * U) {
        __asm__ volatile("" ::"s"(ya[0]), "s"(ya[U - 1]));
#pragma unroll
        for (int i = 0; i < U; ++i) yc[i] = yp[U + i];
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        batch(ya, 0, (b >> 1) & 1);
        __asm__ volatile("" ::"s"(yc[0]), "s"(yc[U - 1]));
        // batch b + 2, or batch b + 1 again when there is none (not used)
        const Y *pn = yp + (b + 2 < nbat ? 2 * U : U);
#pragma unroll
        for (int i = 0; i < U; ++i) ya[i] = pn[i];
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        batch(yc, 1, (b >> 1) & 1);
      }
      if (b < nbat) {
        batch(ya, 0, (b >> 1) & 1);
        yp += U;
      }
    }
    // a group left over by batches of 16 (group 2j, as nbat batches of 16
    // hold an even number of groups)
    for (int g = nbat * Q / G; g < nb; ++g, yp += kAcc) {
      R yb[kAcc];
#pragma unroll
      for (int i = 0; i < kAcc; ++i) yb[i] = yp[i];
#pragma unroll
      for (int i = 0; i < kAcc; ++i) {
        R Ed, zd;
        const R sw = step(p, yb[i], r, ae, pm, Ed, zd);
        if (i == 0 && (kF == 1 || !(g & 1))) av = sw;
        else av += sw;
        if constexpr (kTProd) {
          if (i % kTGroup == kTGroup - 1) {
            ae += log2_fast(pm);
            pm = (R)1;
          }
        }
      }
      if (kF == 1 || (g & 1)) flush();
    }
    // an odd number of groups leaves the last one's span open
    if (kF == 2 && (nb & 1)) flush();
    for (int i = nb * kAcc; i < nm; ++i, ++yp) {
      R ae1 = (R)0, pm1 = (R)1, Ed, zd;
      const R av1 = step(p, *yp, r, ae1, pm1, Ed, zd);
      if constexpr (kTProd) ae1 = log2_fast(pm1);
      sv += (double)av1;
      se += (double)ae1;
      if constexpr (kMix) se += (double)log2_fast(pm1);
    }
    // The last observation: keep its exponents and shock for the state.
    R wl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wl[k] = r.w[k];
    R ae1 = (R)0, pm1 = (R)1, E, z;
    const R av1 = step(p, *yp, r, ae1, pm1, E, z);
    if constexpr (kTProd) ae1 = log2_fast(pm1);
    sv += (double)av1;
    se += (double)ae1;
    if constexpr (kMix) se += (double)log2_fast(pm1);
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = wl[k] / kap;
    st[K] = shock(p, z, E);
    const double nd = (double)n;
    // log h_s = log sigma_Y - ln2 * sum_k w_ks
    if constexpr (kT) return nd * (p.cst - p.lsig) + kLn2 * sv - p.hnu1 * t_scale<R>() * se;
    else if constexpr (kMix) return nd * (p.cst - p.lsig) + kLn2 * (sv + se);
    else return nd * (p.cst - p.lsig) + kLn2 * sv - 0.5 * se;
  }
};

// ------------------------------------------------------ linear regression --
// theta = (beta_1..beta_k, eta = log s2); prior beta | s2 ~ N(0, c0 s2 I),
// s2 ~ InvGamma(a0, b0) with (a0, b0, c0) = (2, 1, 100).
template <int NREG>
struct Linreg {
  static constexpr int D = NREG + 1;
  static constexpr int S = 1;  // unused placeholder (no recursion state)
  using R = double;
  using Y = double;
  static constexpr double kA0 = 2.0, kB0 = 1.0, kC0 = 100.0;

  struct Par {
    double b[NREG];
    double eta, iv;  // log s2, 1/s2
    const double *X;
  };

  __device__ static const Y *ydata(const DevModel &m) { return m.y; }

  // Functions of interest: the parameters themselves.
  static constexpr int kTests = D;
  __device__ static void test_fns(const double *th, const double (&st)[S], int64_t t, double *g) {
    (void)st;
    (void)t;
#pragma unroll
    for (int i = 0; i < D; ++i) g[i] = th[i];
  }

  __device__ static Par params(const double *th) {
    Par p;
#pragma unroll
    for (int i = 0; i < NREG; ++i) p.b[i] = th[i];
    p.eta = th[NREG];
    p.iv = exp(-th[NREG]);
    p.X = nullptr;
    return p;
  }

  __device__ static double logprior(const double *th) {
    const double eta = th[NREG];
    const double iv = exp(-eta);
    // log IG(s2; a0, b0) + eta  (Jacobian of s2 = exp(eta)); lgamma(2) = 0
    double lp = kA0 * log(kB0) - kA0 * eta - kB0 * iv;
#pragma unroll
    for (int i = 0; i < NREG; ++i)
      lp += -0.5 * (kLog2Pi + log(kC0)) - 0.5 * eta - th[i] * th[i] * iv / (2.0 * kC0);
    return lp;
  }

  __device__ static void prior_draw(uint64_t seed, uint64_t run, uint64_t p, double *th) {
    double z[NREG];
    normals<NREG>(seed, run, p, 0, 0, kPrior, z, NREG);
    // s2 = b0 / G, G ~ Gamma(2, 1) as a sum of two unit exponentials.
    const U64x4 w = draw4(seed, run, p, 0, 0, kPrior | ((uint64_t)((NREG + 3) / 4) << 8));
    const double g = -log(u01_oc(w.x0)) - log(u01_oc(w.x1));
    const double s2 = kB0 / g;
#pragma unroll
    for (int i = 0; i < NREG; ++i) th[i] = sqrt(kC0 * s2) * z[i];
    th[NREG] = log(s2);
  }

  __device__ static double advance_x(const Par &p, int64_t t0, int64_t t1, const double *__restrict__ y,
                                     const double *__restrict__ X) {
    double acc = 0.0;
    for (int64_t s = t0; s < t1; ++s) {
      double r = y[s];
#pragma unroll
      for (int i = 0; i < NREG; ++i) r = fma(-X[s * NREG + i], p.b[i], r);
      acc = fma(r, r, acc);
    }
    const double n = (double)(t1 - t0);
    return n * (-0.5 * kLog2Pi - 0.5 * p.eta) - 0.5 * p.iv * acc;
  }
};

// Uniform interface over the two families: the regression has no state and
// reads its regressors from the model description.
template <class M>
struct Eval {
  using R = typename M::R;
  using Y = typename M::Y;
  static constexpr int SR = M::S;
  __device__ __forceinline__ static double advance(const DevModel &dm, const typename M::Par &p,
                                                   R (&st)[SR], int64_t t0, int64_t t1) {
    return M::advance(p, st, t0, t1, M::ydata(dm));
  }
  // The same with the observations from a kernel argument declared
  // __restrict__: a kernel that also stores to global memory then still
  // reads them as uniform scalar loads.
  template <int U = kUnroll>
  __device__ __forceinline__ static double advance_y(const DevModel &dm, const Y *__restrict__ y,
                                                     const typename M::Par &p, R (&st)[SR],
                                                     int64_t t0, int64_t t1) {
    (void)dm;
    return M::template advance<U>(p, st, t0, t1, y);
  }
  template <class F, class G>
  __device__ __forceinline__ static void scan_y(const DevModel &dm, const Y *__restrict__ y,
                                                const typename M::Par &p, R (&st)[SR],
                                                int64_t t0, int64_t t1, F &&f, G &&g) {
    (void)dm;
    M::scan(p, st, t0, t1, y, f, g);
  }
  static const Y *host_y(const DevModel &dm) {
    if constexpr (sizeof(Y) == 4) return dm.y32;
    else return dm.y;
  }
  template <class F, class G>
  __device__ __forceinline__ static void scan(const DevModel &dm, const typename M::Par &p,
                                              R (&st)[SR], int64_t t0, int64_t t1, F &&f,
                                              G &&g) {
    M::scan(p, st, t0, t1, M::ydata(dm), f, g);
  }
};

template <int NREG>
struct Eval<Linreg<NREG>> {
  using R = double;
  using Y = double;
  static constexpr int SR = 1;
  __device__ __forceinline__ static double advance(const DevModel &dm,
                                                   const typename Linreg<NREG>::Par &p,
                                                   double (&st)[1], int64_t t0, int64_t t1) {
    (void)st;
    return Linreg<NREG>::advance_x(p, t0, t1, dm.y, dm.X);
  }
  template <int U = kUnroll>
  __device__ __forceinline__ static double advance_y(const DevModel &dm, const Y *__restrict__ y,
                                                     const typename Linreg<NREG>::Par &p,
                                                     double (&st)[1], int64_t t0, int64_t t1) {
    (void)st;
    return Linreg<NREG>::advance_x(p, t0, t1, y, dm.X);
  }
  template <class F, class G>
  __device__ __forceinline__ static void scan_y(const DevModel &dm, const Y *__restrict__ y,
                                                const typename Linreg<NREG>::Par &p,
                                                double (&st)[1], int64_t t0, int64_t t1, F &&f,
                                                G &&g) {
    (void)st;
    for (int64_t s = t0 + 1; s <= t1; ++s) {
      f(s, Linreg<NREG>::advance_x(p, s - 1, s, y, dm.X));
      if (((s - t0) & 15) == 0) g();
    }
  }
  static const Y *host_y(const DevModel &dm) { return dm.y; }
  template <class F, class G>
  __device__ __forceinline__ static void scan(const DevModel &dm,
                                              const typename Linreg<NREG>::Par &p,
                                              double (&st)[1], int64_t t0, int64_t t1, F &&f,
                                              G &&g) {
    (void)st;
    for (int64_t s = t0 + 1; s <= t1; ++s) {
      f(s, Linreg<NREG>::advance_x(p, s - 1, s, dm.y, dm.X));
      if (((s - t0) & 15) == 0) g();
    }
  }
};

// State width actually stored in memory (0 for the regression).
template <class M>
struct StoredS {
  static constexpr int value = M::S;
};
template <int NREG>
struct StoredS<Linreg<NREG>> {
  static constexpr int value = 0;
};

}  // namespace smc
