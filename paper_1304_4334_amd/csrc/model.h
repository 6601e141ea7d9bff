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

#include "common.h"
#include "rng.h"

namespace smc {

constexpr double kLog2Pi = 1.8378770664093453390819;
constexpr double kSqrt2OverPi = 0.79788456080286535588;
constexpr double kLn2 = 0.69314718055994530942;
constexpr int kUnroll = 8;

// exp(-v/2): FP64 by the device libm; FP32 by the hardware base-2 exponential.
__device__ __forceinline__ double exp_neg_half(double v) { return exp(-0.5 * v); }
__device__ __forceinline__ float exp_neg_half(float v) {
  return __builtin_amdgcn_exp2f(v * -0.721347520444481703680f);  // -log2(e)/2
}

// Student-t kernel term: FP64 log1p(q); FP32 log2(1 + q) (scaled by ln 2 at the end).
__device__ __forceinline__ double t_term(double e, double inu2) { return log1p(e * e * inu2); }
__device__ __forceinline__ float t_term(float e, float inu2) {
  return __builtin_amdgcn_logf(fmaf(e * inu2, e, 1.0f));
}
template <typename R>
__device__ __forceinline__ double t_scale();
template <>
__device__ __forceinline__ double t_scale<double>() { return 1.0; }
template <>
__device__ __forceinline__ double t_scale<float>() { return kLn2; }

__device__ __forceinline__ double normal_logpdf_std(double z) { return -0.5 * kLog2Pi - 0.5 * z * z; }

// ---------------------------------------------------------------- EGARCH --
// theta = (th1, th2, th3_1..K, th4_1..K, th5_1..K [, th9 = log(nu - 2)]),
// mu_Y = th1/1000, sigma_Y = exp(th2), alpha_k = tanh(th3k), beta_k = exp(th4k),
// gamma_k = th5k, nu = 2 + exp(th9) (Table 1; nu is an extension).
template <int K_, int SHOCK_, typename R_>
struct Egarch {
  static constexpr int K = K_;
  static constexpr bool kT = (SHOCK_ == SMC_SHOCK_STUDENT_T);
  static constexpr int D = 2 + 3 * K + (kT ? 1 : 0);
  static constexpr int S = K + 1;
  using R = R_;
  using Y = R_;

  struct Par {
    R al[K], be[K], ga[K], bc[K];  // alpha, beta, gamma, -beta sqrt(2/pi)
    R isig, mus;                   // 1/sigma_Y, mu_Y/sigma_Y
    R inu2;                        // 1/(nu - 2)
    double lsig;                   // log sigma_Y
    double cst;                    // per-observation log-density constant
    double hnu1;                   // (nu + 1)/2
  };

  __device__ static const Y *ydata(const DevModel &m) {
    if constexpr (sizeof(R) == 4) return m.y32;
    else return m.y;
  }

  __device__ static Par params(const double *th) {
    Par p;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double b = exp(th[2 + K + k]);
      p.al[k] = (R)tanh(th[2 + k]);
      p.be[k] = (R)b;
      p.ga[k] = (R)th[2 + 2 * K + k];
      p.bc[k] = (R)(-b * kSqrt2OverPi);
    }
    const double isig = exp(-th[1]);
    p.isig = (R)isig;
    p.mus = (R)(th[0] * 1e-3 * isig);
    p.lsig = th[1];
    if constexpr (kT) {
      const double nu = 2.0 + exp(th[2 + 3 * K]);
      p.inu2 = (R)exp(-th[2 + 3 * K]);
      p.hnu1 = 0.5 * (nu + 1.0);
      p.cst = lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(M_PI * (nu - 2.0));
    } else {
      p.inu2 = (R)0;
      p.hnu1 = 0.5;
      p.cst = -0.5 * kLog2Pi;
    }
    return p;
  }

  __device__ static void prior_moments(int i, double &mean, double &sd) {
    if (i == 0) { mean = 0.0; sd = 1.0; }
    else if (i == 1) { mean = log(0.01); sd = 1.0; }
    else if (i < 2 + K) { mean = atanh(0.95); sd = 1.0; }
    else if (i < 2 + 2 * K) { mean = log(0.10); sd = 1.0; }
    else if (i < 2 + 3 * K) { mean = 0.0; sd = 0.2; }
    else { mean = log(10.0); sd = 1.0; }
  }

  __device__ static double logprior(const double *th) {
    double lp = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double m, sd;
      prior_moments(i, m, sd);
      const double z = (th[i] - m) / sd;
      lp += normal_logpdf_std(z) - log(sd);
    }
    return lp;
  }

  __device__ static void prior_draw(uint64_t seed, uint64_t run, uint64_t p, double *th) {
    double z[D];
    normals<D>(seed, run, p, 0, 0, kPrior, z, D);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double m, sd;
      prior_moments(i, m, sd);
      th[i] = m + sd * z[i];
    }
  }

  // One observation at s >= 2: v_k <- alpha_k v_k + beta_k(|e| - c) + gamma_k e,
  // e <- (y - mu_Y) / (sigma_Y exp(sum v / 2)).  Accumulates sum v and the
  // shock term.
  __device__ __forceinline__ static void step(const Par &p, R y, R (&v)[K], R &e, R &av, R &ae) {
    const R a = fabs(e);
    R vs = (R)0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = fma(p.ga[k], e, fma(p.be[k], a, fma(p.al[k], v[k], p.bc[k])));
      vs += v[k];
    }
    const R ex = exp_neg_half(vs);
    const R z = fma(y, p.isig, -p.mus);
    e = z * ex;
    av += vs;
    if constexpr (kT) ae += t_term(e, p.inu2);
    else ae = fma(e, e, ae);
  }

  // Sum of log p(y_s | y_{1:s-1}, theta) over s = t0+1..t1 with the state at
  // t0 in st (advanced to t1).  The factors take no innovation at s = 1.
  __device__ static double advance(const Par &p, R (&st)[S], int64_t t0, int64_t t1,
                                   const Y *__restrict__ y) {
    R v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = st[k];
    R e = st[K];
    double sv = 0.0, se = 0.0;
    int64_t s = t0;
    if (s == 0 && t1 > 0) {
      e = fma(y[0], p.isig, -p.mus);
      if constexpr (kT) se += (double)t_term(e, p.inu2);
      else se += (double)(e * e);
      s = 1;
    }
    for (; s + kUnroll <= t1; s += kUnroll) {
      R yb[kUnroll];
#pragma unroll
      for (int i = 0; i < kUnroll; ++i) yb[i] = y[s + i];
      R av = (R)0, ae = (R)0;
#pragma unroll
      for (int i = 0; i < kUnroll; ++i) step(p, yb[i], v, e, av, ae);
      sv += (double)av;
      se += (double)ae;
    }
    for (; s < t1; ++s) {
      R av = (R)0, ae = (R)0;
      step(p, y[s], v, e, av, ae);
      sv += (double)av;
      se += (double)ae;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = v[k];
    st[K] = e;
    const double n = (double)(t1 - t0);
    // log h_s = log sigma_Y + sum_k v_ks / 2
    if constexpr (kT) return n * (p.cst - p.lsig) - 0.5 * sv - p.hnu1 * t_scale<R>() * se;
    else return n * (p.cst - p.lsig) - 0.5 * sv - 0.5 * se;
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
  static constexpr int SR = M::S;
  __device__ __forceinline__ static double advance(const DevModel &dm, const typename M::Par &p,
                                                   R (&st)[SR], int64_t t0, int64_t t1) {
    return M::advance(p, st, t0, t1, M::ydata(dm));
  }
};

template <int NREG>
struct Eval<Linreg<NREG>> {
  using R = double;
  static constexpr int SR = 1;
  __device__ __forceinline__ static double advance(const DevModel &dm,
                                                   const typename Linreg<NREG>::Par &p,
                                                   double (&st)[1], int64_t t0, int64_t t1) {
    (void)st;
    return Linreg<NREG>::advance_x(p, t0, t1, dm.y, dm.X);
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
