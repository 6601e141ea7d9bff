// Reverse-mode derivative of the log-likelihood recursion with respect to
// theta, and of the log prior.
//
// The forward sweep stores the exponents w_k of the observation that opens
// every segment of SEG observations (a checkpoint) in the workspace.  The
// reverse sweep visits the segments last to first: it recomputes the
// segment forward from its checkpoint, keeping each observation's exponents
// in a per-lane LDS buffer, then propagates the adjoints back through the
// segment.  Parameter adjoints are summed per segment in the recursion's
// precision and added to FP64 totals.
#pragma once

#include <hip/hip_runtime.h>

#include "model.h"

namespace smc {

// psi(x) by upward recurrence to x >= 8 and the asymptotic series in 1/x^2.
__device__ inline double digamma_dev(double x) {
  double acc = 0.0;
  while (x < 8.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double r = 1.0 / x, r2 = r * r;
  const double series =
      r2 * (1.0 / 12 - r2 * (1.0 / 120 - r2 * (1.0 / 252 - r2 * (1.0 / 240 - r2 * (1.0 / 132)))));
  return acc + log(x) - 0.5 * r - series;
}

// d log p(theta) / d theta.
template <class M>
__device__ inline void logprior_grad(const double *th, double *g);

// (Within the support of the truncated theta_8i the truncation only adds a
// constant, so every term is Gaussian.)
template <int K, int SH, typename R, int I>
struct PriorGrad {
  __device__ static void run(const double *th, double *g) {
    using E = Egarch<K, SH, R, I>;
#pragma unroll
    for (int i = 0; i < E::D; ++i) {
      double m, sd, lsd;
      E::prior_moments(i, m, sd, lsd);
      g[i] = -(th[i] - m) / (sd * sd);
    }
  }
};

// Segment lengths: checkpoints every 64 observations in FP32, every 32 in
// FP64 (the per-lane LDS buffer holds SEG x K values).
template <typename R>
struct SegLen {
  static constexpr int value = sizeof(R) == 4 ? 64 : 32;
};

template <class M>
struct Adjoint;

template <int K, int SH, typename R, int I>
struct Adjoint<Egarch<K, SH, R, I>> {
  using Md = Egarch<K, SH, R, I>;
  using Y = typename Md::Y;
  using Par = typename Md::Par;
  static constexpr int D = Md::D;
  static constexpr int SEG = SegLen<R>::value;
  static constexpr bool kT = Md::kT;
  static constexpr bool kMix = Md::kMix;
  static constexpr int kNM = Md::kNM;
  static constexpr int kLdsPerLane = SEG * K;  // values of type R

  __device__ static int64_t nseg(int64_t t) { return (t + SEG - 1) / SEG; }

  // Chain rule from the adjoints of the components' constants (lw_i =
  // log2(p_i / sigma_i), nb_i = -log2(e) / (2 sigma_i^2), mu_i) back through
  // eqs EGARCH_tran1/2 to theta_6i, theta_7i, theta_8i.
  __device__ static void mixture_chain(const double *th, const double *lwb, const double *nbb,
                                       const double *mub, double scale, double *g) {
    constexpr int b = 2 + 3 * K;
    double ps[kNM], pw[kNM], mss[kNM], ss[kNM], S = 0.0, mbar = 0.0, q = 0.0;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      ps[i] = tanh(th[b + i]) + 1.0;
      S += ps[i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      pw[i] = ps[i] / S;
      mbar += pw[i] * th[b + I + i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      mss[i] = th[b + I + i] - mbar;  // mu**
      ss[i] = exp(th[b + 2 * I + i]);  // sigma*
      q += pw[i] * (mss[i] * mss[i] + ss[i] * ss[i]);
    }
    const double c = 1.0 / sqrt(q);
    // adjoints of the normalised p_i, mu_i, sigma_i
    double pb[kNM], mb[kNM], sb[kNM], cb = 0.0;
#pragma unroll
    for (int i = 0; i < I; ++i) {
      const double si = c * ss[i];
      pb[i] = lwb[i] / (pw[i] * kLn2);
      sb[i] = -lwb[i] / (si * kLn2) + nbb[i] * kLog2e / (si * si * si);
      mb[i] = mub[i];
      cb += mb[i] * mss[i] + sb[i] * ss[i];
    }
    const double qb = cb * (-0.5 * c * c * c);
    double mbarb = 0.0, pdot = 0.0;
    double mssb[kNM], pbt[kNM];
#pragma unroll
    for (int i = 0; i < I; ++i) {
      mssb[i] = c * mb[i] + qb * 2.0 * pw[i] * mss[i];
      mbarb -= mssb[i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      pbt[i] = pb[i] + qb * (mss[i] * mss[i] + ss[i] * ss[i]) + mbarb * th[b + I + i];
      pdot += pbt[i] * pw[i];
    }
#pragma unroll
    for (int i = 0; i < I; ++i) {
      const double ssb = c * sb[i] + qb * 2.0 * pw[i] * ss[i];
      const double psb = (pbt[i] - pdot) / S;
      const double tn = tanh(th[b + i]);
      g[b + i] += scale * psb * (1.0 - tn * tn);
      g[b + I + i] += scale * (mssb[i] + mbarb * pw[i]);
      g[b + 2 * I + i] += scale * ssb * ss[i];
    }
  }

  // Log-likelihood over 1..t from s0 and its gradient g[D] (accumulated into
  // g, times `scale`).  ckpt: [nseg][K][P] of R; lds: this lane's column
  // base of a [SEG*K][64] buffer of R; st receives the state at t.
  __device__ static double value_and_grad(const Par &p, const double *th, int64_t t,
                                          const Y *__restrict__ y, R *ckpt, int64_t P, int64_t pidx,
                                          R *lds, double scale, double *g, R (&st)[Md::S]) {
    if (t <= 0) {
#pragma unroll
      for (int k = 0; k < Md::S; ++k) st[k] = (R)0;
      return 0.0;
    }
    typename Md::Run r;
#pragma unroll
    for (int k = 0; k < K; ++k) r.w[k] = (R)0;
    r.sw = (R)0;
    // ---- forward sweep with checkpoints
    double sv = 0.0, se = 0.0;
    const int64_t ns = nseg(t);
    R wl[K];
    R lastE = (R)1, lastz = (R)0;
    for (int64_t sg = 0; sg < ns; ++sg) {
#pragma unroll
      for (int k = 0; k < K; ++k) ckpt[(sg * K + k) * P + pidx] = r.w[k];
      // 32-bit counters and a segment pointer keep the loop's bookkeeping
      // off the scalar unit
      const int64_t s0 = sg * SEG;
      const int len = (int)(min(t, s0 + SEG) - s0);
      const Y *__restrict__ ys = y + s0;
      R av = (R)0, ae = (R)0, pm = (R)1;
      for (int j = 0; j < len; ++j) {
#pragma unroll
        for (int k = 0; k < K; ++k) wl[k] = r.w[k];
        av += Md::step(p, ys[j], r, ae, pm, lastE, lastz);
        if constexpr (kMix) {
          // the mixture sums' product, folded into log2 every 8 observations
          if ((j & 7) == 7) {
            se += (double)log2_fast(pm);
            pm = (R)1;
          }
        } else if constexpr (Md::kTProd) {
          // FP32 Student-t factors, multiplied in groups (Egarch::kTProd)
          if (j % Md::kTGroup == Md::kTGroup - 1) {
            ae += log2_fast(pm);
            pm = (R)1;
          }
        }
      }
      if constexpr (Md::kTProd) ae += log2_fast(pm);
      sv += (double)av;
      se += (double)ae;
      if constexpr (kMix) se += (double)log2_fast(pm);
    }
    const R kap = (R)Md::kKappa;
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = wl[k] / kap;
    st[K] = Md::shock(p, lastz, lastE);
    const double n = (double)t;
    double ll;
    if constexpr (kT) ll = n * (p.cst - p.lsig) + kLn2 * sv - p.hnu1 * t_scale<R>() * se;
    else if constexpr (kMix) ll = n * (p.cst - p.lsig) + kLn2 * (sv + se);
    else ll = n * (p.cst - p.lsig) + kLn2 * sv - 0.5 * se;

    // ---- reverse sweep
    R wb[K];  // adjoint of the exponents of the observation after the current one
#pragma unroll
    for (int k = 0; k < K; ++k) wb[k] = (R)0;
    double ab[K], c0b[K], kbb[K], kgb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ab[k] = c0b[k] = kbb[k] = kgb[k] = 0.0;
    double isigb = 0.0, musb = 0.0, inu2b = 0.0, hnu1b = 0.0;
    // mixture: adjoints of lw_i, nb_i and mu_i (the components' constants)
    double lwb[kNM], nbb[kNM], mub[kNM];
#pragma unroll
    for (int i = 0; i < kNM; ++i) lwb[i] = nbb[i] = mub[i] = 0.0;
    const R ln2 = (R)kLn2;
    for (int64_t sg = ns - 1; sg >= 0; --sg) {
      const int64_t s0 = sg * SEG;
      const int len = (int)(min(t, s0 + SEG) - s0);
      const Y *__restrict__ ys = y + s0;
      // recompute the segment, keeping each observation's exponents
#pragma unroll
      for (int k = 0; k < K; ++k) r.w[k] = ckpt[(sg * K + k) * P + pidx];
      R sw0 = r.w[0];
#pragma unroll
      for (int k = 1; k < K; ++k) sw0 += r.w[k];
      r.sw = sw0;
      for (int j = 0; j < len; ++j) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[(j * K + k) * 64] = r.w[k];
        R ae = (R)0, pm = (R)1, Ed, zd;
        (void)Md::step(p, ys[j], r, ae, pm, Ed, zd);
      }
      R a_ab[K], a_c0b[K], a_kbb[K], a_kgb[K];
#pragma unroll
      for (int k = 0; k < K; ++k) a_ab[k] = a_c0b[k] = a_kbb[k] = a_kgb[k] = (R)0;
      R a_isigb = (R)0, a_musb = (R)0, a_inu2b = (R)0, a_hnu1b = (R)0;
      R a_lwb[kNM], a_nbb[kNM], a_mub[kNM];
#pragma unroll
      for (int i = 0; i < kNM; ++i) a_lwb[i] = a_nbb[i] = a_mub[i] = (R)0;
      for (int j = len - 1; j >= 0; --j) {
        const R yv = ys[j];
        R w[K];
        R sw = (R)0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          w[k] = lds[(j * K + k) * 64];
          sw += w[k];
        }
        const R E = exp2_fast(sw);
        const R z = fma(yv, p.isig, -p.mus);
        const R az = fabs(z);
        const R sgn = z > (R)0 ? (R)1 : (z < (R)0 ? (R)-1 : (R)0);
        const R e = z * E;
        // w_k,s+1 = kz_k E + a_k w_k + c0_k
        R Eb = (R)0, zb = (R)0;
        R wn[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const R kz = fma(p.kb[k], az, p.kg[k] * z);
          Eb = fma(wb[k], kz, Eb);
          const R kzb = wb[k] * E;
          a_kbb[k] = fma(kzb, az, a_kbb[k]);
          a_kgb[k] = fma(kzb, z, a_kgb[k]);
          zb = fma(kzb, fma(p.kb[k], sgn, p.kg[k]), zb);
          a_ab[k] = fma(wb[k], w[k], a_ab[k]);
          a_c0b[k] += wb[k];
          wn[k] = wb[k] * p.a[k];
        }
        // the observation's log density: ln2 sw - e^2/2, or - hnu1 log(1 + e^2/(nu-2))
        R eb;
        if constexpr (kT) {
          const R q1 = fma(e * e, p.inu2, (R)1);
          const R h = (R)p.hnu1;
          eb = -h * (R)2 * e * p.inu2 / q1;
          a_inu2b = fma(-h, e * e / q1, a_inu2b);
          a_hnu1b -= t_term(e * e, p.inu2);
        } else if constexpr (kMix) {
          // log density ln2 log2 sum_i 2^x_i, x_i = lw_i + nb_i (e - mu_i)^2:
          // d/dx_i = ln2 pi_i with pi_i = 2^(x_i - m) / sum_j 2^(x_j - m)
          R dm[kNM], x[kNM];
#pragma unroll
          for (int i = 0; i < kNM; ++i) {
            dm[i] = e - p.mu[i];
            x[i] = fma(p.nb[i] * dm[i], dm[i], p.lw[i]);
          }
          R mx = x[0];
#pragma unroll
          for (int i = 1; i < kNM; ++i) mx = fmax(mx, x[i]);
          R ex[kNM], sm = (R)0;
#pragma unroll
          for (int i = 0; i < kNM; ++i) {
            ex[i] = exp2_lean(x[i] - mx);
            sm += ex[i];
          }
          const R inv = ln2 / sm;
          eb = (R)0;
#pragma unroll
          for (int i = 0; i < kNM; ++i) {
            const R pi = ex[i] * inv;  // ln2 pi_i
            a_lwb[i] += pi;
            a_nbb[i] = fma(pi * dm[i], dm[i], a_nbb[i]);
            const R g2 = (R)2 * pi * p.nb[i] * dm[i];
            a_mub[i] -= g2;
            eb += g2;
          }
        } else {
          eb = -e;
        }
        zb = fma(eb, E, zb);
        Eb = fma(eb, z, Eb);
        const R swb = fma(Eb * E, ln2, ln2);
#pragma unroll
        for (int k = 0; k < K; ++k) wb[k] = wn[k] + swb;
        a_isigb = fma(zb, yv, a_isigb);
        a_musb -= zb;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        ab[k] += (double)a_ab[k];
        c0b[k] += (double)a_c0b[k];
        kbb[k] += (double)a_kbb[k];
        kgb[k] += (double)a_kgb[k];
      }
      isigb += (double)a_isigb;
      musb += (double)a_musb;
      inu2b += (double)a_inu2b;
      hnu1b += (double)a_hnu1b;
#pragma unroll
      for (int i = 0; i < kNM; ++i) {
        lwb[i] += (double)a_lwb[i];
        nbb[i] += (double)a_nbb[i];
        mub[i] += (double)a_mub[i];
      }
    }
    // ---- chain rule to theta (Table 1 transforms)
    const double isig = exp(-th[1]);
    const double mus = th[0] * 1e-3 * isig;
    g[0] += scale * (musb * 1e-3 * isig);
    g[1] += scale * (-isigb * isig - musb * mus - n);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double a = tanh(th[2 + k]);
      const double b = exp(th[2 + K + k]);
      g[2 + k] += scale * ab[k] * (1.0 - a * a);
      g[2 + K + k] += scale * (c0b[k] * (-Md::kKappa * b * kSqrt2OverPi) + kbb[k] * Md::kKappa * b);
      g[2 + 2 * K + k] += scale * kgb[k] * Md::kKappa;
    }
    if constexpr (kT) {
      const double en = exp(th[2 + 3 * K]);
      const double nu = 2.0 + en;
      const double dcst = en * 0.5 * (digamma_dev(0.5 * (nu + 1.0)) - digamma_dev(0.5 * nu)) - 0.5;
      const double hb = hnu1b * t_scale<R>();
      g[2 + 3 * K] += scale * (inu2b * (-1.0 / en) + hb * 0.5 * en + n * dcst);
    }
    if constexpr (kMix) mixture_chain(th, lwb, nbb, mub, scale, g);
    return ll;
  }
};

// The regression needs no recursion: one pass gives the value and gradient.
template <int NREG>
struct Adjoint<Linreg<NREG>> {
  using Md = Linreg<NREG>;
  static constexpr int kLdsPerLane = 0;
  __device__ static int64_t nseg(int64_t) { return 0; }
  __device__ static double value_and_grad(const DevModel &dm, const double *th, int64_t t,
                                          double scale, double *g) {
    double acc = 0.0, gb[NREG];
#pragma unroll
    for (int i = 0; i < NREG; ++i) gb[i] = 0.0;
    for (int64_t s = 0; s < t; ++s) {
      double r = dm.y[s];
#pragma unroll
      for (int i = 0; i < NREG; ++i) r = fma(-dm.X[s * NREG + i], th[i], r);
      acc = fma(r, r, acc);
#pragma unroll
      for (int i = 0; i < NREG; ++i) gb[i] = fma(r, dm.X[s * NREG + i], gb[i]);
    }
    const double iv = exp(-th[NREG]), n = (double)t;
#pragma unroll
    for (int i = 0; i < NREG; ++i) g[i] += scale * gb[i] * iv;
    g[NREG] += scale * (-0.5 * n + 0.5 * iv * acc);
    return n * (-0.5 * kLog2Pi - 0.5 * th[NREG]) - 0.5 * iv * acc;
  }
};

template <int NREG>
struct PriorGradLin {
  __device__ static void run(const double *th, double *g) {
    const double eta = th[NREG], iv = exp(-eta);
    double sb = 0.0;
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
      g[i] = -th[i] * iv / Linreg<NREG>::kC0;
      sb += th[i] * th[i];
    }
    g[NREG] = -Linreg<NREG>::kA0 + Linreg<NREG>::kB0 * iv - 0.5 * NREG +
              0.5 * sb * iv / Linreg<NREG>::kC0;
  }
};

template <class M>
struct PriorGradOf;
template <int K, int SH, typename R, int I>
struct PriorGradOf<Egarch<K, SH, R, I>> {
  __device__ static void run(const double *th, double *g) { PriorGrad<K, SH, R, I>::run(th, g); }
};
template <int NREG>
struct PriorGradOf<Linreg<NREG>> {
  __device__ static void run(const double *th, double *g) { PriorGradLin<NREG>::run(th, g); }
};

}  // namespace smc
