/*
 * Plain FP64 CPU oracle of the adaptive sequential posterior simulator
 * (Durham & Geweke, "Adaptive sequential posterior simulators for massively
 * parallel computing environments").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the yardstick the HIP path is
 * checked against.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load it; the product library never links, calls or
 * reads it, and it shares no code with the HIP sources.
 *
 * Style: every step is written in the order the paper states it, one particle
 * and one observation at a time, with serial loops and the C library's
 * exp/log/lgamma.  No blocking, fusion or reordering beyond that.  The only
 * concession to speed is an OpenMP "parallel for" over independent
 * particles, which does not change any result.
 *
 * Layout: a population stores particle p's parameter vector contiguously,
 * theta[p*d + i], and its recursion state as state[p*S + k]; particle p
 * belongs to group j = p / N (Section 2.3: J groups of N particles).
 *
 * Pins (what checks this file against something other than itself) are in
 * tests/test_oracle_*.py; the functions without an external pin are listed
 * in the "parity unpinned" notes below.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DMAX 32 /* largest parameter dimension handled */

/* Threads the OpenMP particle loops use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
/* Sets the threads of the OpenMP particle loops (for timing the oracle on
 * one core or on all of them; results do not depend on it). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
#define ORC_SMAX 8  /* largest recursion state handled */

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror and     */
/* Shaw, SC'11).  Ten rounds of two 64x64->128 multiplies with a Weyl key   */
/* schedule.  Pinned against numpy.random.Philox.                           */
/* ------------------------------------------------------------------------ */
static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(prod >> 64);
  *lo = (uint64_t)prod;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mul_hi_lo(M0, x0, &hi0, &lo0);
    mul_hi_lo(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter coordinates: (index, cycle, iteration-or-block, purpose | sub<<8). */
enum { ORC_PRIOR = 1, ORC_RESAMPLE = 2, ORC_PROPOSAL = 3, ORC_ACCEPT = 4 };

static void draw4(uint64_t seed, uint64_t run, uint64_t c0, uint64_t c1, uint64_t c2,
                  uint64_t c3, uint64_t out[4]) {
  uint64_t ctr[4] = {c0, c1, c2, c3};
  uint64_t key[2] = {seed, run};
  orc_philox4x64_10(ctr, key, out);
}

/* u in [0,1): top 53 bits. */
static double u01_co(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
/* u in (0,1]: top 53 bits plus one. */
static double u01_oc(uint64_t x) { return ((double)(x >> 11) + 1.0) * 0x1.0p-53; }
/* u in (0,1): top 53 bits plus one half. */
static double u01_oo(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

/* n standard normals by Box-Muller: block b uses counter sub-index b; its
 * four 64-bit words (x0,x1,x2,x3) give the pairs (z_4b, z_4b+1) and
 * (z_4b+2, z_4b+3) as r cos(2 pi u2), r sin(2 pi u2), r = sqrt(-2 log u1),
 * u1 in (0,1] from the first word, u2 in [0,1) from the second. */
static void normals(uint64_t seed, uint64_t run, uint64_t c0, uint64_t c1, uint64_t c2,
                    uint64_t purpose, int n, double *z) {
  for (int b = 0; 4 * b < n; ++b) {
    uint64_t x[4];
    draw4(seed, run, c0, c1, c2, purpose | ((uint64_t)b << 8), x);
    for (int pair = 0; pair < 2; ++pair) {
      double u1 = u01_oc(x[2 * pair]);
      double u2 = u01_co(x[2 * pair + 1]);
      double r = sqrt(-2.0 * log(u1));
      double a = 2.0 * M_PI * u2;
      int i0 = 4 * b + 2 * pair;
      if (i0 < n) z[i0] = r * cos(a);
      if (i0 + 1 < n) z[i0 + 1] = r * sin(a);
    }
  }
}

void orc_normals(uint64_t seed, uint64_t run, uint64_t c0, uint64_t c1, uint64_t c2,
                 uint64_t purpose, int n, double *z) {
  normals(seed, run, c0, c1, c2, purpose, n, z);
}

/* ------------------------------------------------------------------------ */
/* Models (Section 5.1 and the conjugate regression workload).              */
/* ------------------------------------------------------------------------ */
enum { ORC_LINREG = 1, ORC_EGARCH = 2 };
enum { ORC_GAUSS = 0, ORC_STUDENT_T = 1, ORC_MIXTURE = 2 };

typedef struct {
  int32_t kind;    /* ORC_LINREG or ORC_EGARCH */
  int32_t K;       /* EGARCH volatility factors */
  int32_t shock;   /* ORC_GAUSS, ORC_STUDENT_T or ORC_MIXTURE */
  int32_t nreg;    /* regressors (LINREG) */
  int64_t T;       /* observations */
  const double *y; /* [T] */
  const double *X; /* [T][nreg] (LINREG) */
  int32_t I;       /* normal-mixture components (ORC_MIXTURE, I >= 2) */
  int32_t pad_;
} orc_model;

/* Lower truncation point of theta_8i (Table 1) and log P(Z >= -3) for the
 * normalising constant of the truncated prior. */
static const double MIX_TRUNC = -3.0;
static double mix_log_mass(void) { return log(0.5 * erfc(MIX_TRUNC / sqrt(2.0))); }

/* Conjugate prior of the regression: beta | s2 ~ N(0, c0 s2 I), s2 ~ IG(a0, b0). */
static const double LR_A0 = 2.0, LR_B0 = 1.0, LR_C0 = 100.0;

int orc_dim(const orc_model *m) {
  if (m->kind == ORC_LINREG) return m->nreg + 1;
  if (m->shock == ORC_MIXTURE) return 2 + 3 * m->K + 3 * m->I;
  return 2 + 3 * m->K + (m->shock == ORC_STUDENT_T ? 1 : 0);
}

int orc_state_dim(const orc_model *m) {
  if (m->kind == ORC_LINREG) return 0;
  return m->K + 1; /* v_1..v_K and the previous standardised shock */
}

/* Table 1 prior means and standard deviations on the transformed parameters,
 * in the order (th1, th2, th3_k.., th4_k.., th5_k.., then either
 * th9 = log(nu - 2) or th6_i.., th7_i.., th8_i..). */
static void egarch_prior_moments(const orc_model *m, double *mean, double *sd) {
  int K = m->K, i = 0;
  mean[i] = 0.0; sd[i] = 1.0; ++i;                        /* mu_Y = th1/1000 */
  mean[i] = log(0.01); sd[i] = 1.0; ++i;                  /* sigma_Y = exp(th2) */
  for (int k = 0; k < K; ++k, ++i) { mean[i] = atanh(0.95); sd[i] = 1.0; }  /* alpha */
  for (int k = 0; k < K; ++k, ++i) { mean[i] = log(0.10); sd[i] = 1.0; }   /* beta */
  for (int k = 0; k < K; ++k, ++i) { mean[i] = 0.0; sd[i] = 0.2; }         /* gamma */
  if (m->shock == ORC_STUDENT_T) { mean[i] = log(10.0); sd[i] = 1.0; ++i; } /* nu */
  if (m->shock == ORC_MIXTURE)  /* p*_i, mu*_i, sigma*_i: all N(0, 1) */
    for (int r = 0; r < 3 * m->I; ++r, ++i) { mean[i] = 0.0; sd[i] = 1.0; }
}

/* Index of the first theta_8i (mixture scales), or -1. */
static int mix_sigma_index(const orc_model *m) {
  return m->shock == ORC_MIXTURE ? 2 + 3 * m->K + 2 * m->I : -1;
}

double orc_logprior(const orc_model *m, const double *th) {
  int d = orc_dim(m);
  if (m->kind == ORC_LINREG) {
    int k = m->nreg;
    double eta = th[k]; /* log sigma^2 */
    /* log IG(s2; a0, b0) plus the log-Jacobian eta of s2 = exp(eta). */
    double lp = LR_A0 * log(LR_B0) - lgamma(LR_A0) - LR_A0 * eta - LR_B0 * exp(-eta);
    for (int i = 0; i < k; ++i)
      lp += -0.5 * log(2.0 * M_PI * LR_C0) - 0.5 * eta -
            th[i] * th[i] / (2.0 * LR_C0 * exp(eta));
    return lp;
  }
  double mean[ORC_DMAX], sd[ORC_DMAX];
  egarch_prior_moments(m, mean, sd);
  double lp = 0.0;
  for (int i = 0; i < d; ++i) {
    double z = (th[i] - mean[i]) / sd[i];
    lp += -0.5 * log(2.0 * M_PI) - log(sd[i]) - 0.5 * z * z;
  }
  /* theta_8i ~ N(0, 1) truncated to [-3, inf) */
  int i8 = mix_sigma_index(m);
  if (i8 >= 0)
    for (int i = 0; i < m->I; ++i) {
      if (th[i8 + i] < MIX_TRUNC) return -INFINITY;
      lp -= mix_log_mass();
    }
  return lp;
}

/* Draw particle p from the prior (Algorithm 1, step 1) using the counter
 * (p, 0, 0, PRIOR | block). */
void orc_prior_draw(const orc_model *m, uint64_t seed, uint64_t run, int64_t p, double *th) {
  int d = orc_dim(m);
  if (m->kind == ORC_LINREG) {
    int k = m->nreg;
    double z[ORC_DMAX];
    normals(seed, run, (uint64_t)p, 0, 0, ORC_PRIOR, k, z);
    /* s2 ~ IG(a0, b0) as b0 / Gamma(a0, 1); Gamma(2, 1) is a sum of two unit
     * exponentials, -log u_a - log u_b.  Uniforms come from the block after
     * the normals. */
    uint64_t x[4];
    draw4(seed, run, (uint64_t)p, 0, 0, ORC_PRIOR | ((uint64_t)((k + 3) / 4) << 8), x);
    double g = -log(u01_oc(x[0])) - log(u01_oc(x[1]));
    double s2 = LR_B0 / g;
    for (int i = 0; i < k; ++i) th[i] = sqrt(LR_C0 * s2) * z[i];
    th[k] = log(s2);
    return;
  }
  double mean[ORC_DMAX], sd[ORC_DMAX], z[ORC_DMAX];
  egarch_prior_moments(m, mean, sd);
  normals(seed, run, (uint64_t)p, 0, 0, ORC_PRIOR, d, z);
  for (int i = 0; i < d; ++i) th[i] = mean[i] + sd[i] * z[i];
  /* Truncated theta_8i by rejection: attempt a = 1, 2, ... redraws the whole
   * normal vector on counter (p, 0, a, PRIOR | block) and takes its entry
   * for that parameter.  After 32 failed attempts (probability 1e-92) the
   * truncation point itself is used. */
  int i8 = mix_sigma_index(m);
  if (i8 >= 0)
    for (int i = i8; i < i8 + m->I; ++i) {
      for (uint64_t a = 1; th[i] < MIX_TRUNC && a <= 32; ++a) {
        normals(seed, run, (uint64_t)p, 0, a, ORC_PRIOR, d, z);
        th[i] = mean[i] + sd[i] * z[i];
      }
      if (th[i] < MIX_TRUNC) th[i] = MIX_TRUNC;
    }
}

/* Mixture components from theta (eqs EGARCH_tran1 and EGARCH_tran2):
 * p*_i = tanh(th6i) + 1, mu*_i = th7i, sigma*_i = exp(th8i); p_i = p*_i /
 * sum p*; mu**_i = mu*_i - sum_j p_j mu*_j; c = [sum p_i (mu**_i^2 +
 * sigma*_i^2)]^(-1/2); mu_i = c mu**_i, sigma_i = c sigma*_i.  The result
 * has mean sum p_i mu_i = 0 and variance 1 (eq EGARCH_normalization). */
void orc_mixture_params(const orc_model *m, const double *th, double *pw, double *mu,
                        double *sg) {
  int I = m->I, b = 2 + 3 * m->K;
  double ps = 0.0, pm = 0.0, q = 0.0;
  for (int i = 0; i < I; ++i) { pw[i] = tanh(th[b + i]) + 1.0; ps += pw[i]; }
  for (int i = 0; i < I; ++i) { pw[i] /= ps; pm += pw[i] * th[b + I + i]; }
  for (int i = 0; i < I; ++i) {
    mu[i] = th[b + I + i] - pm;
    sg[i] = exp(th[b + 2 * I + i]);
    q += pw[i] * (mu[i] * mu[i] + sg[i] * sg[i]);
  }
  double c = 1.0 / sqrt(q);
  for (int i = 0; i < I; ++i) { mu[i] *= c; sg[i] *= c; }
}

void orc_state_init(const orc_model *m, double *state) {
  int S = orc_state_dim(m);
  for (int k = 0; k < S; ++k) state[k] = 0.0; /* v_k0 = 0 (Section 5.1, step 2) */
}

/* log p(y_s | y_{1:s-1}, theta) for s = 1..T (1-based), advancing the state.
 *
 * EGARCH, the four steps of Section 5.1:
 *   1. transform: mu_Y = th1/1000, sigma_Y = exp(th2), alpha_k = tanh(th3k),
 *      beta_k = exp(th4k), gamma_k = th5k (Table 1); nu = 2 + exp(th9);
 *   2. v_ks = alpha_k v_k,s-1 + beta_k (|eps_{s-1}| - sqrt(2/pi)) + gamma_k eps_{s-1}
 *      (eq EGARCH_mod1); the factors start at zero and take no innovation at
 *      s = 1, since no eps_0 exists;
 *   3. h_s = sigma_Y exp(sum_k v_ks / 2), eps_s = (y_s - mu_Y) / h_s;
 *   4. Gaussian shocks: log phi(eps_s) - log h_s.  Student-t shocks are
 *      rescaled to unit variance, so eps has density
 *      Gamma((nu+1)/2) / (Gamma(nu/2) sqrt(pi (nu-2))) (1 + eps^2/(nu-2))^(-(nu+1)/2).
 *      Normal-mixture shocks (eq normal_mixture): the density of eps is
 *      sum_i p_i phi(eps; mu_i, sigma_i^2), its logarithm taken as a
 *      log-sum-exp over the components (shifted by the largest term).
 * Regression: log N(y_s; x_s' beta, exp(eta)).
 */
static double obs_logdens(const orc_model *m, const double *th, int64_t s, double *state) {
  const double y = m->y[s - 1];
  if (m->kind == ORC_LINREG) {
    int k = m->nreg;
    double mean = 0.0;
    for (int i = 0; i < k; ++i) mean += m->X[(s - 1) * k + i] * th[i];
    double eta = th[k];
    double r = y - mean;
    return -0.5 * log(2.0 * M_PI) - 0.5 * eta - r * r / (2.0 * exp(eta));
  }
  int K = m->K;
  double mu = th[0] / 1000.0;
  double sig = exp(th[1]);
  double vsum = 0.0;
  for (int k = 0; k < K; ++k) {
    double alpha = tanh(th[2 + k]);
    double beta = exp(th[2 + K + k]);
    double gamma = th[2 + 2 * K + k];
    double eprev = state[K];
    if (s > 1)
      state[k] = alpha * state[k] + beta * (fabs(eprev) - sqrt(2.0 / M_PI)) + gamma * eprev;
    vsum += state[k];
  }
  double h = sig * exp(vsum / 2.0);
  double eps = (y - mu) / h;
  state[K] = eps;
  if (m->shock == ORC_GAUSS) return -0.5 * log(2.0 * M_PI) - log(h) - 0.5 * eps * eps;
  if (m->shock == ORC_MIXTURE) {
    double pw[ORC_DMAX], mc[ORC_DMAX], sg[ORC_DMAX], a[ORC_DMAX];
    orc_mixture_params(m, th, pw, mc, sg);
    double mx = -INFINITY, sum = 0.0;
    for (int i = 0; i < m->I; ++i) {
      double u = (eps - mc[i]) / sg[i];
      a[i] = log(pw[i]) - log(sg[i]) - 0.5 * u * u;
      if (a[i] > mx) mx = a[i];
    }
    for (int i = 0; i < m->I; ++i) sum += exp(a[i] - mx);
    return -0.5 * log(2.0 * M_PI) - log(h) + mx + log(sum);
  }
  double nu = 2.0 + exp(th[2 + 3 * K]);
  double c = lgamma((nu + 1.0) / 2.0) - lgamma(nu / 2.0) - 0.5 * log(M_PI * (nu - 2.0));
  return c - log(h) - (nu + 1.0) / 2.0 * log(1.0 + eps * eps / (nu - 2.0));
}

/* Sum of log p(y_s | y_{1:s-1}, theta) over s = t0+1..t1, with the state at
 * t0 in `state` (advanced to t1 on return). */
double orc_loglik_range(const orc_model *m, const double *th, int64_t t0, int64_t t1,
                        double *state) {
  double ll = 0.0;
  for (int64_t s = t0 + 1; s <= t1; ++s) ll += obs_logdens(m, th, s, state);
  return ll;
}

/* Full-data log-likelihood over 1..t for P particles ([P][d] layout); the
 * final state goes to state_out ([P][S]) when given. */
void orc_loglik_batch(const orc_model *m, int64_t P, const double *theta, int64_t t,
                      double *ll_out, double *state_out) {
  int d = orc_dim(m), S = orc_state_dim(m);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double st[ORC_SMAX];
    orc_state_init(m, st);
    ll_out[p] = orc_loglik_range(m, theta + p * d, 0, t, st);
    if (state_out)
      for (int k = 0; k < S; ++k) state_out[p * S + k] = st[k];
  }
}

/* ------------------------------------------------------------------------ */
/* Forward-mode derivatives (dual numbers) for the gradient of              */
/* log p(theta) + log p(y_{1:t} | theta), used by the Langevin M kernel and  */
/* to check the adjoint kernel.  Pinned by central finite differences.      */
/* ------------------------------------------------------------------------ */
typedef struct { double v; double g[ORC_DMAX]; } dual;

static dual dconst(double c) { dual r; r.v = c; memset(r.g, 0, sizeof r.g); return r; }
static dual dvar(double x, int i) { dual r = dconst(x); r.g[i] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = a.g[i] + b.g[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = a.g[i] - b.g[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i]; return r; }
static dual ddiv(dual a, dual b) { dual r; r.v = a.v / b.v; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = (a.g[i] * b.v - a.v * b.g[i]) / (b.v * b.v); return r; }
static dual dscale(dual a, double c) { dual r; r.v = a.v * c; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = a.g[i] * c; return r; }
static dual dchain(dual a, double f, double df) { dual r; r.v = f; for (int i = 0; i < ORC_DMAX; ++i) r.g[i] = a.g[i] * df; return r; }
static dual dexp(dual a) { double e = exp(a.v); return dchain(a, e, e); }
static dual dlog(dual a) { return dchain(a, log(a.v), 1.0 / a.v); }
static dual dtanh(dual a) { double t = tanh(a.v); return dchain(a, t, 1.0 - t * t); }
/* d|x|/dx taken as sign(x), with 0 at x = 0. */
static dual dabs(dual a) { double s = a.v > 0 ? 1.0 : (a.v < 0 ? -1.0 : 0.0); return dchain(a, fabs(a.v), s); }

/* Digamma by upward recurrence to x >= 8 and the asymptotic series. */
static double digamma(double x) {
  double acc = 0.0;
  while (x < 8.0) { acc -= 1.0 / x; x += 1.0; }
  double x2 = 1.0 / (x * x);
  return acc + log(x) - 0.5 / x -
         x2 * (1.0 / 12 - x2 * (1.0 / 120 - x2 * (1.0 / 252 - x2 * (1.0 / 240 - x2 * (1.0 / 132)))));
}
static dual dlgamma(dual a) { return dchain(a, lgamma(a.v), digamma(a.v)); }

static dual obs_logdens_dual(const orc_model *m, const dual *th, int64_t s, dual *state) {
  const double y = m->y[s - 1];
  if (m->kind == ORC_LINREG) {
    int k = m->nreg;
    dual mean = dconst(0.0);
    for (int i = 0; i < k; ++i) mean = dadd(mean, dscale(th[i], m->X[(s - 1) * k + i]));
    dual eta = th[k];
    dual r = dsub(dconst(y), mean);
    return dsub(dsub(dconst(-0.5 * log(2.0 * M_PI)), dscale(eta, 0.5)),
                ddiv(dmul(r, r), dscale(dexp(eta), 2.0)));
  }
  int K = m->K;
  dual mu = dscale(th[0], 1.0 / 1000.0);
  dual sig = dexp(th[1]);
  dual vsum = dconst(0.0);
  for (int k = 0; k < K; ++k) {
    dual alpha = dtanh(th[2 + k]);
    dual beta = dexp(th[2 + K + k]);
    dual gamma = th[2 + 2 * K + k];
    dual eprev = state[K];
    if (s > 1)
      state[k] = dadd(dadd(dmul(alpha, state[k]),
                           dmul(beta, dsub(dabs(eprev), dconst(sqrt(2.0 / M_PI))))),
                      dmul(gamma, eprev));
    vsum = dadd(vsum, state[k]);
  }
  dual h = dmul(sig, dexp(dscale(vsum, 0.5)));
  dual eps = ddiv(dsub(dconst(y), mu), h);
  state[K] = eps;
  if (m->shock == ORC_GAUSS)
    return dsub(dsub(dconst(-0.5 * log(2.0 * M_PI)), dlog(h)), dscale(dmul(eps, eps), 0.5));
  if (m->shock == ORC_MIXTURE) {
    /* the same transforms and log-sum-exp on dual numbers */
    int I = m->I, b = 2 + 3 * K;
    dual pw[ORC_DMAX], mc[ORC_DMAX], sg[ORC_DMAX], a[ORC_DMAX];
    dual ps = dconst(0.0), pm = dconst(0.0), q = dconst(0.0);
    for (int i = 0; i < I; ++i) { pw[i] = dadd(dtanh(th[b + i]), dconst(1.0)); ps = dadd(ps, pw[i]); }
    for (int i = 0; i < I; ++i) { pw[i] = ddiv(pw[i], ps); pm = dadd(pm, dmul(pw[i], th[b + I + i])); }
    for (int i = 0; i < I; ++i) {
      mc[i] = dsub(th[b + I + i], pm);
      sg[i] = dexp(th[b + 2 * I + i]);
      q = dadd(q, dmul(pw[i], dadd(dmul(mc[i], mc[i]), dmul(sg[i], sg[i]))));
    }
    dual c = ddiv(dconst(1.0), dchain(q, sqrt(q.v), 0.5 / sqrt(q.v)));
    double mx = -INFINITY;
    for (int i = 0; i < I; ++i) {
      mc[i] = dmul(mc[i], c);
      sg[i] = dmul(sg[i], c);
      dual u = ddiv(dsub(eps, mc[i]), sg[i]);
      a[i] = dsub(dsub(dlog(pw[i]), dlog(sg[i])), dscale(dmul(u, u), 0.5));
      if (a[i].v > mx) mx = a[i].v;
    }
    dual sum = dconst(0.0);
    for (int i = 0; i < I; ++i) sum = dadd(sum, dexp(dsub(a[i], dconst(mx))));
    return dadd(dsub(dconst(-0.5 * log(2.0 * M_PI) + mx), dlog(h)), dlog(sum));
  }
  dual nu = dadd(dconst(2.0), dexp(th[2 + 3 * K]));
  dual nu2 = dsub(nu, dconst(2.0));
  dual c = dsub(dsub(dlgamma(dscale(dadd(nu, dconst(1.0)), 0.5)), dlgamma(dscale(nu, 0.5))),
                dscale(dlog(dscale(nu2, M_PI)), 0.5));
  dual q = dlog(dadd(dconst(1.0), ddiv(dmul(eps, eps), nu2)));
  return dsub(dsub(c, dlog(h)), dmul(dscale(dadd(nu, dconst(1.0)), 0.5), q));
}

static dual logprior_dual(const orc_model *m, const dual *th) {
  int d = orc_dim(m);
  if (m->kind == ORC_LINREG) {
    int k = m->nreg;
    dual eta = th[k];
    dual lp = dsub(dsub(dconst(LR_A0 * log(LR_B0) - lgamma(LR_A0)), dscale(eta, LR_A0)),
                   dscale(dexp(dscale(eta, -1.0)), LR_B0));
    for (int i = 0; i < k; ++i)
      lp = dsub(dsub(dadd(lp, dconst(-0.5 * log(2.0 * M_PI * LR_C0))), dscale(eta, 0.5)),
                ddiv(dmul(th[i], th[i]), dscale(dexp(eta), 2.0 * LR_C0)));
    return lp;
  }
  double mean[ORC_DMAX], sd[ORC_DMAX];
  egarch_prior_moments(m, mean, sd);
  dual lp = dconst(0.0);
  for (int i = 0; i < d; ++i) {
    dual z = dscale(dsub(th[i], dconst(mean[i])), 1.0 / sd[i]);
    lp = dsub(dadd(lp, dconst(-0.5 * log(2.0 * M_PI) - log(sd[i]))), dscale(dmul(z, z), 0.5));
  }
  int i8 = mix_sigma_index(m);
  if (i8 >= 0)
    for (int i = 0; i < m->I; ++i) {
      if (th[i8 + i].v < MIX_TRUNC) return dconst(-INFINITY);
      lp = dsub(lp, dconst(mix_log_mass()));
    }
  return lp;
}

/* Gradient of log p(y_{1:t} | theta) (returned value is the log-likelihood). */
double orc_loglik_grad(const orc_model *m, const double *theta, int64_t t, double *grad) {
  int d = orc_dim(m), S = orc_state_dim(m);
  dual th[ORC_DMAX], st[ORC_SMAX];
  for (int i = 0; i < d; ++i) th[i] = dvar(theta[i], i);
  for (int k = 0; k < S; ++k) st[k] = dconst(0.0);
  dual ll = dconst(0.0);
  for (int64_t s = 1; s <= t; ++s) ll = dadd(ll, obs_logdens_dual(m, th, s, st));
  for (int i = 0; i < d; ++i) grad[i] = ll.g[i];
  return ll.v;
}

double orc_logprior_grad(const orc_model *m, const double *theta, double *grad) {
  int d = orc_dim(m);
  dual th[ORC_DMAX];
  for (int i = 0; i < d; ++i) th[i] = dvar(theta[i], i);
  dual lp = logprior_dual(m, th);
  for (int i = 0; i < d; ++i) grad[i] = lp.g[i];
  return lp.v;
}

/* ------------------------------------------------------------------------ */
/* Particle population and the C, S and M phases (Algorithm 1, Section 3.3) */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t J, N, d, S;
  double *theta;    /* [P][d] */
  double *logprior; /* [P] */
  double *loglik;   /* [P] log p(y_{1:t} | theta_p) at the current date t */
  double *state;    /* [P][S] recursion state at the current date */
  double *logw;     /* [P] log of the C-phase weight w_jn(s) */
} orc_pop;

/* Step 1 of Algorithm 1: theta_jn iid from the prior; weights one. */
void orc_init(const orc_model *m, orc_pop *pop, uint64_t seed, uint64_t run) {
  int64_t P = (int64_t)pop->J * pop->N;
  int d = pop->d, S = pop->S;
  for (int64_t p = 0; p < P; ++p) {
    orc_prior_draw(m, seed, run, p, pop->theta + p * d);
    pop->logprior[p] = orc_logprior(m, pop->theta + p * d);
    pop->loglik[p] = 0.0;
    pop->logw[p] = 0.0;
    orc_state_init(m, pop->state + p * S);
  }
}

/* RSS = ESS / (JN), ESS = (sum w)^2 / sum w^2 over all J*N particles
 * (Section 3.3, "C phase termination"), with w rescaled by exp(-max log w). */
double orc_rss(const double *logw, int64_t P) {
  double mx = -INFINITY;
  for (int64_t p = 0; p < P; ++p) if (logw[p] > mx) mx = logw[p];
  if (!(mx > -INFINITY)) return 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t p = 0; p < P; ++p) {
    double e = exp(logw[p] - mx);
    s1 += e;
    s2 += e * e;
  }
  return s1 * s1 / ((double)P * s2);
}

/* log of the group mean weight, log( N^-1 sum_n w_jn ) (Section 4.2). */
static double log_mean_exp(const double *a, int64_t n) {
  double mx = -INFINITY;
  for (int64_t i = 0; i < n; ++i) if (a[i] > mx) mx = a[i];
  if (!(mx > -INFINITY)) return -INFINITY;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += exp(a[i] - mx);
  return mx + log(s / (double)n);
}

/* C phase (Algorithm 1, step 2a): w_jn(t_from) = 1, then for s = t_from+1..
 * multiply in p(y_s | y_{1:s-1}, theta_jn) (eq C_phase_compute), the same term
 * also extending the particle's log-likelihood.  At each check date (every
 * `check_every`-th observation, and always at t_max) the RSS is computed and
 * the phase ends when RSS < rss_min (rss_min <= 0: run to t_max).  Returns
 * t_l; writes the final RSS and log wbar_j(l-1) for each group. */
int64_t orc_correct(const orc_model *m, orc_pop *pop, int64_t t_from, int64_t t_max,
                    int64_t check_every, double rss_min, double *rss_out, double *group_logwbar) {
  int64_t P = (int64_t)pop->J * pop->N;
  int d = pop->d, S = pop->S;
  for (int64_t p = 0; p < P; ++p) pop->logw[p] = 0.0;
  int64_t s = t_from;
  double rss = 1.0;
  while (s < t_max) {
    ++s;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
      double lp = obs_logdens(m, pop->theta + p * d, s, pop->state + p * S);
      if (isnan(lp)) lp = -INFINITY;
      pop->logw[p] += lp;
      pop->loglik[p] += lp;
    }
    if (s % check_every == 0 || s == t_max) {
      rss = orc_rss(pop->logw, P);
      if (rss < rss_min) break;
    }
  }
  for (int j = 0; j < pop->J; ++j)
    group_logwbar[j] = log_mean_exp(pop->logw + (int64_t)j * pop->N, pop->N);
  if (rss_out) *rss_out = rss;
  return s;
}

enum { ORC_RESIDUAL = 0, ORC_MULTINOMIAL = 1, ORC_STRATIFIED = 2, ORC_SYSTEMATIC = 3 };

/* S phase (Algorithm 1, step 2b) for every group independently.
 *
 * Residual resampling (Liu and Chen 1998), the default of Section 3.3: with
 * normalised weights W_n, particle n is first copied floor(N W_n) times; the
 * remaining R = N - sum_n floor(N W_n) draws are multinomial with
 * probabilities proportional to N W_n - floor(N W_n).  Multinomial
 * resampling makes all N draws that way from W_n.
 *
 * Draw k of group j in cycle l uses word k%4 of the Philox block with counter
 * (j, l, k/4, RESAMPLE) as u in [0,1); the draw is the first n whose running
 * residual sum exceeds u times the residual total.  Ancestors are written in
 * ascending order, each index repeated by its total count.
 *
 * `margin` (optional, [J]) receives, per group, the smallest distance of any
 * N W_n from a positive integer and of any draw target from a running-sum
 * boundary, relative to the scale of those sums: a tie-break indicator for
 * comparing implementations that round differently.
 * Returns the number of groups with no positive weight (their ancestors are
 * left as the identity). */
int orc_resample(const int32_t J, const int32_t N, const double *logw, int scheme, uint64_t seed,
                 uint64_t run, uint64_t cycle, int32_t *ancestor, double *margin) {
  int bad = 0;
  double *nw = (double *)malloc(sizeof(double) * N);
  double *cum = (double *)malloc(sizeof(double) * N);
  int64_t *count = (int64_t *)malloc(sizeof(int64_t) * N);
  for (int j = 0; j < J; ++j) {
    const double *lw = logw + (int64_t)j * N;
    int32_t *anc = ancestor + (int64_t)j * N;
    double mx = -INFINITY;
    for (int n = 0; n < N; ++n) if (lw[n] > mx) mx = lw[n];
    if (!(mx > -INFINITY)) {
      ++bad;
      for (int n = 0; n < N; ++n) anc[n] = j * N + n;
      if (margin) margin[j] = INFINITY;
      continue;
    }
    double sum = 0.0;
    for (int n = 0; n < N; ++n) sum += exp(lw[n] - mx);
    double mrg = INFINITY;
    int64_t copies = 0;
    for (int n = 0; n < N; ++n) {
      nw[n] = ((double)N * exp(lw[n] - mx)) / sum; /* N W_n */
      if (scheme == ORC_RESIDUAL) {
        count[n] = (int64_t)floor(nw[n]);
        double frac = nw[n] - floor(nw[n]);
        if (nw[n] >= 0.5) {
          double dist = frac < 0.5 ? frac : 1.0 - frac;
          if (dist < mrg) mrg = dist;
        }
      } else {
        count[n] = 0;
      }
      copies += count[n];
    }
    double run_sum = 0.0;
    for (int n = 0; n < N; ++n) {
      run_sum += nw[n] - (double)count[n];
      cum[n] = run_sum;
    }
    int64_t R = N - copies;
    uint64_t x0[4];
    draw4(seed, run, (uint64_t)j, cycle, 0, ORC_RESAMPLE, x0);
    for (int64_t k = 0; k < R; ++k) {
      uint64_t x[4];
      draw4(seed, run, (uint64_t)j, cycle, (uint64_t)(k / 4), ORC_RESAMPLE, x);
      double u = u01_co(x[k % 4]);
      if (scheme == ORC_STRATIFIED) u = ((double)k + u) / (double)N;
      if (scheme == ORC_SYSTEMATIC) u = ((double)k + u01_co(x0[0])) / (double)N;
      double target = u * cum[N - 1];
      int a = -1;
      for (int n = 0; n < N; ++n)
        if (cum[n] > target) { a = n; break; }
      if (a < 0) {
        /* u * total rounded up to the total: take the last index with a
         * positive residual */
        a = N - 1;
        while (a > 0 && !(cum[a] > cum[a - 1])) --a;
      }
      count[a] += 1;
      double lo = a > 0 ? cum[a - 1] : 0.0;
      double dist = fmin(fabs(target - lo), fabs(cum[a] - target));
      if (dist < mrg) mrg = dist;
    }
    int64_t pos = 0;
    for (int n = 0; n < N; ++n)
      for (int64_t c = 0; c < count[n]; ++c) anc[pos++] = j * N + n;
    if (margin) margin[j] = mrg;
  }
  free(nw);
  free(cum);
  free(count);
  return bad;
}

/* Replace every particle by its ancestor (theta, prior, likelihood, state). */
void orc_gather(orc_pop *pop, const int32_t *ancestor) {
  int64_t P = (int64_t)pop->J * pop->N;
  int d = pop->d, S = pop->S;
  double *th = (double *)malloc(sizeof(double) * P * d);
  double *lp = (double *)malloc(sizeof(double) * P);
  double *ll = (double *)malloc(sizeof(double) * P);
  double *st = (double *)malloc(sizeof(double) * (P * S + 1));
  for (int64_t p = 0; p < P; ++p) {
    int64_t a = ancestor[p];
    for (int i = 0; i < d; ++i) th[p * d + i] = pop->theta[a * d + i];
    for (int k = 0; k < S; ++k) st[p * S + k] = pop->state[a * S + k];
    lp[p] = pop->logprior[a];
    ll[p] = pop->loglik[a];
  }
  memcpy(pop->theta, th, sizeof(double) * P * d);
  memcpy(pop->logprior, lp, sizeof(double) * P);
  memcpy(pop->loglik, ll, sizeof(double) * P);
  if (S) memcpy(pop->state, st, sizeof(double) * P * S);
  free(th); free(lp); free(ll); free(st);
}

/* Sample mean and variance of the current population (divisor P - 1) and the
 * lower Cholesky factor of the variance; V_lr of Section 3.3.  Returns 0, or
 * -1 when the variance is not positive definite. */
int orc_moments(const orc_pop *pop, double *mean, double *cov, double *chol) {
  int64_t P = (int64_t)pop->J * pop->N;
  int d = pop->d;
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int64_t p = 0; p < P; ++p) s += pop->theta[p * d + i];
    mean[i] = s / (double)P;
  }
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      double s = 0.0;
      for (int64_t p = 0; p < P; ++p)
        s += (pop->theta[p * d + i] - mean[i]) * (pop->theta[p * d + k] - mean[k]);
      cov[i * d + k] = s / (double)(P - 1);
    }
  /* Cholesky-Banachiewicz: V = L L', L lower triangular, row by row. */
  for (int i = 0; i < d * d; ++i) chol[i] = 0.0;
  for (int i = 0; i < d; ++i) {
    for (int k = 0; k <= i; ++k) {
      double s = cov[i * d + k];
      for (int q = 0; q < k; ++q) s -= chol[i * d + q] * chol[k * d + q];
      if (i == k) {
        if (!(s > 0.0)) return -1;
        chol[i * d + i] = sqrt(s);
      } else {
        chol[i * d + k] = s / chol[k * d + k];
      }
    }
  }
  return 0;
}

enum { ORC_RW = 0, ORC_MALA = 1, ORC_INDEP = 2 };

/* One M-phase Metropolis iteration (Algorithm 1, step 2c with the Gaussian
 * random walk of Section 3.3) over every particle at date t:
 *   z ~ N(0, I) from counter (p, l, r, PROPOSAL | block),
 *   theta' = theta + (h L) z with Sigma_lr = h^2 V_lr = (hL)(hL)',
 *   accept when log u < log p(theta') + log p(y_{1:t}|theta') - (same at theta),
 *   u in (0,1) from counter (p, l, r, ACCEPT), first word.
 * The Langevin variant (kernel = ORC_MALA) adds the drift (1/2)(hL)(hL)' grad
 * log posterior to the proposal mean and the proposal-density ratio to the
 * acceptance test.  The independent Gaussian sampler of Section 3.3
 * (kernel = ORC_INDEP) proposes theta' = mean + L z from the particle mean
 * and variance, whatever the current particle, and adds
 * log q(theta) - log q(theta') to the acceptance test.  `hchol` is hL,
 * d x d row-major lower triangular, followed for ORC_INDEP by the mean [d].
 * Writes accept flags (optional) and returns the number accepted. */
/* The M step of one particle with global index p (its Philox counters use
 * p): theta (d), lp and ll are updated in place on acceptance, state (S)
 * too.  Returns 1 when the proposal is accepted. */
int orc_mutate_particle(const orc_model *m, int64_t p, double *th, double *lp, double *ll,
                        double *state, int64_t t, int kernel, const double *hchol, uint64_t seed,
                        uint64_t run, uint64_t cycle, uint64_t iter) {
  int d = orc_dim(m), S = orc_state_dim(m);
  double z[ORC_DMAX], prop[ORC_DMAX], st[ORC_SMAX];
  double g0[ORC_DMAX], g1[ORC_DMAX], gp[ORC_DMAX];
  normals(seed, run, (uint64_t)p, cycle, iter, ORC_PROPOSAL, d, z);
  double drift[ORC_DMAX];
  for (int i = 0; i < d; ++i) drift[i] = 0.0;
  if (kernel == ORC_MALA) {
    /* gradient of the log posterior kernel at the current particle */
    orc_loglik_grad(m, th, t, g0);
    orc_logprior_grad(m, th, gp);
    for (int i = 0; i < d; ++i) g0[i] += gp[i];
    /* (1/2) (hL)(hL)' g0 */
    double w[ORC_DMAX];
    for (int k = 0; k < d; ++k) {
      w[k] = 0.0;
      for (int i = k; i < d; ++i) w[k] += hchol[i * d + k] * g0[i];
    }
    for (int i = 0; i < d; ++i) {
      drift[i] = 0.0;
      for (int k = 0; k <= i; ++k) drift[i] += 0.5 * hchol[i * d + k] * w[k];
    }
  }
  /* the independent sampler centres its proposal on the particle mean, which
   * follows the d x d factor in hchol */
  const double *centre = (kernel == ORC_INDEP) ? hchol + d * d : th;
  for (int i = 0; i < d; ++i) {
    double step = 0.0;
    for (int k = 0; k <= i; ++k) step += hchol[i * d + k] * z[k];
    prop[i] = centre[i] + drift[i] + step;
  }
  double lp_new = orc_logprior(m, prop);
  int acc = 0;
  double ll_new = -INFINITY;
  if (lp_new > -INFINITY) {
    double logq_ratio = 0.0;
    if (kernel == ORC_MALA) {
      ll_new = orc_loglik_grad(m, prop, t, g1);
      orc_logprior_grad(m, prop, gp);
      for (int i = 0; i < d; ++i) g1[i] += gp[i];
      /* reverse move: solve (hL) w = theta - theta' - (1/2)(hL)(hL)' g1 */
      double v[ORC_DMAX], a[ORC_DMAX], wv[ORC_DMAX];
      for (int k = 0; k < d; ++k) {
        v[k] = 0.0;
        for (int i = k; i < d; ++i) v[k] += hchol[i * d + k] * g1[i];
      }
      for (int i = 0; i < d; ++i) {
        double dr = 0.0;
        for (int k = 0; k <= i; ++k) dr += 0.5 * hchol[i * d + k] * v[k];
        a[i] = th[i] - prop[i] - dr;
      }
      for (int i = 0; i < d; ++i) {
        double s = a[i];
        for (int k = 0; k < i; ++k) s -= hchol[i * d + k] * wv[k];
        wv[i] = s / hchol[i * d + i];
      }
      double zz = 0.0, ww = 0.0;
      for (int i = 0; i < d; ++i) { zz += z[i] * z[i]; ww += wv[i] * wv[i]; }
      logq_ratio = -0.5 * ww + 0.5 * zz;
      /* the state at t is needed on acceptance */
      orc_state_init(m, st);
      orc_loglik_range(m, prop, 0, t, st);
    } else {
      orc_state_init(m, st);
      ll_new = orc_loglik_range(m, prop, 0, t, st);
      if (kernel == ORC_INDEP) {
        /* q(theta) / q(theta') with q = N(mean, L L'): w = L^-1 (theta - mean),
         * and L^-1 (theta' - mean) = z */
        double wv[ORC_DMAX], zz = 0.0, ww = 0.0;
        for (int i = 0; i < d; ++i) {
          double s = th[i] - centre[i];
          for (int k = 0; k < i; ++k) s -= hchol[i * d + k] * wv[k];
          wv[i] = s / hchol[i * d + i];
          ww += wv[i] * wv[i];
          zz += z[i] * z[i];
        }
        logq_ratio = -0.5 * ww + 0.5 * zz;
      }
    }
    double delta = (lp_new + ll_new) - (*lp + *ll) + logq_ratio;
    uint64_t x[4];
    draw4(seed, run, (uint64_t)p, cycle, iter, ORC_ACCEPT, x);
    double logu = log(u01_oo(x[0]));
    acc = (logu < delta) ? 1 : 0; /* false for NaN */
  }
  if (acc) {
    for (int i = 0; i < d; ++i) th[i] = prop[i];
    for (int k = 0; k < S; ++k) state[k] = st[k];
    *lp = lp_new;
    *ll = ll_new;
  }
  return acc;
}

/* One M-phase Metropolis iteration (Algorithm 1, step 2c with the Gaussian
 * random walk of Section 3.3) over every particle at date t:
 *   z ~ N(0, I) from counter (p, l, r, PROPOSAL | block),
 *   theta' = theta + (h L) z with Sigma_lr = h^2 V_lr = (hL)(hL)',
 *   accept when log u < log p(theta') + log p(y_{1:t}|theta') - (same at theta),
 *   u in (0,1) from counter (p, l, r, ACCEPT), first word.
 * The Langevin variant (kernel = ORC_MALA) adds the drift (1/2)(hL)(hL)' grad
 * log posterior to the proposal mean and the proposal-density ratio to the
 * acceptance test.  The independent Gaussian sampler of Section 3.3
 * (kernel = ORC_INDEP) proposes theta' = mean + L z from the particle mean
 * and variance, whatever the current particle, and adds
 * log q(theta) - log q(theta') to the acceptance test.  `hchol` is hL,
 * d x d row-major lower triangular, followed for ORC_INDEP by the mean [d].
 * Writes accept flags (optional) and returns the number accepted. */
int64_t orc_mutate(const orc_model *m, orc_pop *pop, int64_t t, int kernel, const double *hchol,
                   uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter, uint8_t *accepted) {
  int64_t P = (int64_t)pop->J * pop->N;
  int d = pop->d, S = pop->S;
  int64_t n_acc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_acc)
  for (int64_t p = 0; p < P; ++p) {
    double stp[ORC_SMAX];
    for (int k = 0; k < S; ++k) stp[k] = pop->state[p * S + k];
    int acc = orc_mutate_particle(m, p, pop->theta + p * d, pop->logprior + p, pop->loglik + p,
                                  stp, t, kernel, hchol, seed, run, cycle, iter);
    if (acc) {
      for (int k = 0; k < S; ++k) pop->state[p * S + k] = stp[k];
      n_acc += 1;
    }
    if (accepted) accepted[p] = (uint8_t)acc;
  }
  return n_acc;
}

/* Mean over the parameters theta_i (the test functions g_i(theta) = theta_i)
 * of RNE = var-hat / v-hat (Section 2.3): var-hat the pooled variance with
 * divisor NJ - 1, v-hat = N/(J-1) sum_j (gbar_j - gbar)^2. */
double orc_rne_mean(const orc_pop *pop) {
  int J = pop->J, N = pop->N, d = pop->d;
  int64_t P = (int64_t)J * N;
  double acc = 0.0;
  for (int i = 0; i < d; ++i) {
    double gbar = 0.0;
    double gj[4096];
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += pop->theta[((int64_t)j * N + n) * d + i];
      gj[j] = s / N;
      gbar += gj[j];
    }
    gbar /= J;
    double vhat = 0.0;
    for (int j = 0; j < J; ++j) vhat += (gj[j] - gbar) * (gj[j] - gbar);
    vhat *= (double)N / (double)(J - 1);
    double var = 0.0;
    for (int64_t p = 0; p < P; ++p) {
      double e = pop->theta[p * d + i] - gbar;
      var += e * e;
    }
    var /= (double)(P - 1);
    acc += var / vhat;
  }
  return acc / d;
}

/* ------------------------------------------------------------------------ */
/* Functions of interest and their posterior moments (Sections 2.3, 5.2)   */
/* ------------------------------------------------------------------------ */
enum { ORC_TEST_PARAMS = 0, ORC_TEST_MODEL = 1 };

/* Number of test functions: the parameters (d), or the model's functions of
 * interest.  For EGARCH those are Section 5.2's g1 (log volatility), g2 (the
 * shock's third moment, mixtures only: it is zero for the symmetric shocks)
 * and g3 (the 3% loss probability).  The regression uses its parameters. */
int orc_num_test_fns(const orc_model *m, int which) {
  if (which == ORC_TEST_PARAMS || m->kind == ORC_LINREG) return orc_dim(m);
  return m->shock == ORC_MIXTURE ? 3 : 2;
}

static double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Regularised incomplete beta function I_x(a, b), 0 <= x <= 1: the
 * continued fraction of DLMF 8.17.22,
 *   I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) / (1 + d1 / (1 + d2 / (1 + ...))),
 *   d_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1)),
 *   d_{2m}   = m (b - m) x / ((a + 2m - 1)(a + 2m)),
 * summed by the modified Lentz method where it converges quickly
 * (x < (a + 1) / (a + b + 2)), else through I_x(a, b) = 1 - I_{1-x}(b, a).
 * lx and l1x are log x and log(1 - x), passed separately so that neither
 * loses digits to cancellation. */
static double inc_beta(double a, double b, double x, double lx, double l1x) {
  if (x > (a + 1.0) / (a + b + 2.0)) return 1.0 - inc_beta(b, a, 1.0 - x, l1x, lx);
  const double tiny = 1e-300;
  double f = 1.0, C = 1.0, D = 0.0;
  for (int j = 1; j <= 100000; ++j) {
    int m = j / 2;
    double dj = (j & 1) ? -(a + m) * (a + b + m) * x / ((a + 2 * m) * (a + 2 * m + 1))
                        : m * (b - m) * x / ((a + 2 * m - 1) * (a + 2 * m));
    D = 1.0 + dj * D;
    if (fabs(D) < tiny) D = tiny;
    C = 1.0 + dj / C;
    if (fabs(C) < tiny) C = tiny;
    D = 1.0 / D;
    f *= C * D;
    if (fabs(C * D - 1.0) < 1e-16) break;
  }
  double lpre = a * lx + b * l1x + lgamma(a + b) - lgamma(a) - lgamma(b);
  return exp(lpre) / (a * f);
}

/* Distribution function of the unit-variance Student-t shock (the density
 * of step 4 of the likelihood) at x, nu2 = nu - 2: eps = z sqrt(nu2 / nu)
 * with z ~ t_nu, and P(t_nu < z) = I_w(nu/2, 1/2) / 2 for z < 0 with
 * w = nu / (nu + z^2) (DLMF 8.17.22's relation for the t distribution), which
 * in terms of x is w = nu2 / (nu2 + x^2); symmetry gives z >= 0. */
static double student_t_unit_cdf(double x, double nu2) {
  if (isinf(x)) return x < 0.0 ? 0.0 : 1.0; /* the limits at -inf and +inf */
  double r = nu2 + x * x;
  double tail = 0.5 * inc_beta(0.5 * (nu2 + 2.0), 0.5, nu2 / r, log(nu2) - log(r),
                               2.0 * log(fabs(x)) - log(r));
  return x < 0.0 ? tail : 1.0 - tail;
}

/* The test functions at parameter theta and state (v_1..v_K, eps_t) at date t:
 *   g1 = log sigma_Y + sum_k v_kt / 2 = log h_t;
 *   g2 = E(eps^3) = sum_i p_i (mu_i^3 + 3 mu_i sigma_i^2);
 *   g3 = P(Y_{t+1} < -0.03 | theta, y_{1:t}) = F((-0.03 - mu_Y) / h_{t+1}),
 * F the shock distribution (Phi, the unit-variance t, or
 * sum_i p_i Phi((x - mu_i) / sigma_i)),
 * h_{t+1} from eq EGARCH_mod1 one step ahead (no innovation when t = 0). */
void orc_test_fns(const orc_model *m, int which, const double *th, const double *state, int64_t t,
                  double *g) {
  int d = orc_dim(m);
  if (which == ORC_TEST_PARAMS || m->kind == ORC_LINREG) {
    for (int i = 0; i < d; ++i) g[i] = th[i];
    return;
  }
  int K = m->K, q = 0;
  double vs = 0.0, vn = 0.0;
  double eprev = state[K];
  for (int k = 0; k < K; ++k) {
    vs += state[k];
    double alpha = tanh(th[2 + k]), beta = exp(th[2 + K + k]), gamma = th[2 + 2 * K + k];
    vn += (t >= 1) ? alpha * state[k] + beta * (fabs(eprev) - sqrt(2.0 / M_PI)) + gamma * eprev : 0.0;
  }
  g[q++] = th[1] + vs / 2.0;
  double pw[ORC_DMAX], mc[ORC_DMAX], sg[ORC_DMAX];
  if (m->shock == ORC_MIXTURE) {
    orc_mixture_params(m, th, pw, mc, sg);
    double m3 = 0.0;
    for (int i = 0; i < m->I; ++i) m3 += pw[i] * (mc[i] * mc[i] * mc[i] + 3.0 * mc[i] * sg[i] * sg[i]);
    g[q++] = m3;
  }
  double h1 = exp(th[1]) * exp(vn / 2.0);
  double x = (-0.03 - th[0] / 1000.0) / h1;
  if (m->shock == ORC_GAUSS) {
    g[q++] = std_normal_cdf(x);
  } else if (m->shock == ORC_STUDENT_T) {
    g[q++] = student_t_unit_cdf(x, exp(th[2 + 3 * K]));
  } else {
    double F = 0.0;
    for (int i = 0; i < m->I; ++i) F += pw[i] * std_normal_cdf((x - mc[i]) / sg[i]);
    g[q++] = F;
  }
}

/* Posterior moment report of G functions from their values g[P][G] over J
 * groups of N (Section 2.3): grand mean, standard deviation
 * (var-hat with divisor NJ - 1), NSE (eq NSE_def) and RNE = var-hat / v-hat
 * (eq vhat); out[G][4]. */
void orc_report(int32_t J, int32_t N, int G, const double *g, double *out) {
  int64_t P = (int64_t)J * N;
  double *gj = (double *)malloc(sizeof(double) * J);
  for (int i = 0; i < G; ++i) {
    double gbar = 0.0;
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += g[((int64_t)j * N + n) * G + i];
      gj[j] = s / N;
      gbar += gj[j];
    }
    gbar /= J;
    double b = 0.0;
    for (int j = 0; j < J; ++j) b += (gj[j] - gbar) * (gj[j] - gbar);
    double var = 0.0;
    for (int64_t p = 0; p < P; ++p) {
      double e = g[p * G + i] - gbar;
      var += e * e;
    }
    var /= (double)(P - 1);
    double vhat = (double)N / (double)(J - 1) * b;
    out[i * 4 + 0] = gbar;
    out[i * 4 + 1] = sqrt(var);
    out[i * 4 + 2] = sqrt(b / ((double)J * (J - 1)));
    out[i * 4 + 3] = var / vhat;
  }
  free(gj);
}

/* The report of the population's test functions at date t (out[G][4]);
 * returns G. */
int orc_test_report(const orc_model *m, const orc_pop *pop, int which, int64_t t, double *out) {
  int G = orc_num_test_fns(m, which);
  int64_t P = (int64_t)pop->J * pop->N;
  double *g = (double *)malloc(sizeof(double) * P * G);
  double zero[ORC_SMAX] = {0};
  for (int64_t p = 0; p < P; ++p)
    orc_test_fns(m, which, pop->theta + p * pop->d, pop->S ? pop->state + p * pop->S : zero, t,
                 g + p * G);
  orc_report(pop->J, pop->N, G, g, out);
  free(g);
  return G;
}

/* Marginal likelihood from the per-cycle group mean weights (Section 4.2):
 *   log wbar_j = sum_l log wbar_j(l-1),  wbar = J^-1 sum_j wbar_j,
 *   wtilde = prod_l J^-1 sum_j wbar_j(l-1),
 *   NSE of log wbar by the delta method of eq ML_se:
 *   sqrt( [J(J-1)]^-1 sum_j (wbar_j - wbar)^2 ) / wbar.
 * out = {log wbar, NSE, log wtilde}. */
void orc_log_ml(int32_t L, int32_t J, const double *group_logwbar, double *out) {
  double lw[4096];
  for (int j = 0; j < J; ++j) {
    lw[j] = 0.0;
    for (int l = 0; l < L; ++l) lw[j] += group_logwbar[(int64_t)l * J + j];
  }
  double mx = -INFINITY;
  for (int j = 0; j < J; ++j) if (lw[j] > mx) mx = lw[j];
  double rbar = 0.0;
  for (int j = 0; j < J; ++j) rbar += exp(lw[j] - mx);
  rbar /= J;
  double ss = 0.0;
  for (int j = 0; j < J; ++j) {
    double e = exp(lw[j] - mx) - rbar;
    ss += e * e;
  }
  out[0] = mx + log(rbar);
  out[1] = sqrt(ss / ((double)J * (J - 1))) / rbar;
  double lt = 0.0;
  for (int l = 0; l < L; ++l) lt += log_mean_exp(group_logwbar + (int64_t)l * J, J);
  out[2] = lt;
}

/* ------------------------------------------------------------------------ */
/* Whole simulator: Algorithm 2 with the rules of Section 3.3 (adaptive), or */
/* Algorithm 1 driven by a recorded design {t_l, Sigma_lr, R_l} (replay,     */
/* step 2 of Algorithm 3).                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t J, N;
  uint64_t seed, run;
  int32_t check_every;  /* C-phase RSS checks: every k-th observation */
  int32_t force_every;  /* dates of interest every k-th observation (0: none) */
  double D1, D2;        /* C-phase end and long-M thresholds */
  int32_t Rbar, kappa;  /* deterministic M-phase rule */
  int32_t stop_rule;    /* 0 deterministic, 1 RNE-based */
  double E1;            /* RNE threshold */
  int32_t Rmax;         /* cap on M iterations */
  int32_t scheme;       /* ORC_RESIDUAL, ORC_MULTINOMIAL, ORC_STRATIFIED, ORC_SYSTEMATIC */
  int32_t kernel;       /* ORC_RW, ORC_MALA or ORC_INDEP */
  int32_t replay;       /* 0 adaptive, 1 replay the record */
  int32_t Lmax;         /* capacity of the record, cycles */
  int32_t RmaxRec;      /* capacity of the record, iterations per cycle */
  int32_t test_fn;      /* RNE rule and moment report: ORC_TEST_PARAMS or ORC_TEST_MODEL */
  int32_t pad_;
  double E2;            /* RNE threshold after a C phase ending at a date of interest */
  int64_t burn_in;      /* log-score burn-in date b (a date of interest; 0: none) */
} orc_cfg;

typedef struct {
  int32_t L;
  int64_t *t_end;        /* [Lmax] */
  int32_t *R;            /* [Lmax] */
  double *hchol;         /* [Lmax][RmaxRec][d*d] */
  double *rss;           /* [Lmax] RSS at the end of each C phase */
  int64_t *n_acc;        /* [Lmax][RmaxRec] */
  double *group_logwbar; /* [Lmax][J] */
  double log_ml, nse, log_ml_tilde;
  int64_t evals;         /* particle x observation log-density evaluations */
  double *moments;       /* [Lmax][G][4] report at each cycle end, or NULL */
  double *mean;          /* [Lmax][RmaxRec][d] particle means (independent sampler), or NULL */
  double log_score, log_score_nse, log_score_tilde; /* over (burn_in, T] */
  int32_t *mh;           /* [Lmax][RmaxRec] step size in tenths used by each iteration, or NULL */
  double *chol;          /* [Lmax][RmaxRec][d*d] unscaled Cholesky factor of V_lr, or NULL */
} orc_record;

/* Returns 0, or a negative code: -1 record too small, -2 non-PD variance,
 * -3 a group lost all weight. */
int orc_run(const orc_model *m, const orc_cfg *cfg, orc_pop *pop, orc_record *rec) {
  int d = pop->d;
  int64_t P = (int64_t)cfg->J * cfg->N;
  int64_t T = m->T;
  double mean[ORC_DMAX], cov[ORC_DMAX * ORC_DMAX], chol[ORC_DMAX * ORC_DMAX];
  double rep[ORC_DMAX * 4];
  int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * P);
  int status = 0;
  int64_t evals = 0;
  orc_init(m, pop, cfg->seed, cfg->run);
  int64_t t = 0;
  int l = 0;
  while (t < T) {
    if (l >= cfg->Lmax) { status = -1; break; }
    double rss;
    /* A C phase ends at RSS < D1, at T, or at the next date of interest
     * (Section 3.3: S and M phases are executed at such dates). */
    int64_t t_stop = T;
    if (cfg->force_every > 0) {
      int64_t next = (t / cfg->force_every + 1) * cfg->force_every;
      if (next < t_stop) t_stop = next;
    }
    if (cfg->burn_in > t && cfg->burn_in < t_stop) t_stop = cfg->burn_in;
    if (cfg->replay) t_stop = rec->t_end[l];
    double rss_min = cfg->replay ? 0.0 : cfg->D1;
    int64_t t_new = orc_correct(m, pop, t, t_stop, cfg->check_every, rss_min, &rss,
                                rec->group_logwbar + (int64_t)l * cfg->J);
    evals += P * (t_new - t);
    rec->t_end[l] = t_new;
    rec->rss[l] = rss;
    if (orc_resample(cfg->J, cfg->N, pop->logw, cfg->scheme, cfg->seed, cfg->run,
                     (uint64_t)(l + 1), anc, NULL)) { status = -3; break; }
    orc_gather(pop, anc);
    int32_t R;
    if (cfg->replay) R = rec->R[l];
    else R = (rss < cfg->D2) ? cfg->kappa * cfg->Rbar : cfg->Rbar;
    int mh = 5; /* h = mh / 10, Section 3.3: start at 0.5, steps of 0.1 in [0.1, 1] */
    int r = 0;
    for (;;) {
      ++r;
      if (r > cfg->RmaxRec) { status = -1; break; }
      double *hl = rec->hchol + ((int64_t)l * cfg->RmaxRec + (r - 1)) * d * d;
      double *mrec = rec->mean ? rec->mean + ((int64_t)l * cfg->RmaxRec + (r - 1)) * d : NULL;
      if (!cfg->replay) {
        if (orc_moments(pop, mean, cov, chol)) { status = -2; break; }
        /* the independent sampler uses the particle variance unscaled */
        double h = (cfg->kernel == ORC_INDEP) ? 1.0 : mh / 10.0;
        for (int i = 0; i < d * d; ++i) hl[i] = h * chol[i];
        if (rec->mh) rec->mh[(int64_t)l * cfg->RmaxRec + (r - 1)] = (cfg->kernel == ORC_INDEP) ? 10 : mh;
        if (rec->chol)
          for (int i = 0; i < d * d; ++i)
            rec->chol[((int64_t)l * cfg->RmaxRec + (r - 1)) * d * d + i] = chol[i];
        if (mrec)
          for (int i = 0; i < d; ++i) mrec[i] = mean[i];
      }
      const double *kern_arg = hl;
      double lm[ORC_DMAX * ORC_DMAX + ORC_DMAX];
      if (cfg->kernel == ORC_INDEP) {
        if (!mrec) { status = -1; break; }
        for (int i = 0; i < d * d; ++i) lm[i] = hl[i];
        for (int i = 0; i < d; ++i) lm[d * d + i] = mrec[i];
        kern_arg = lm;
      }
      int64_t acc = orc_mutate(m, pop, t_new, cfg->kernel, kern_arg, cfg->seed, cfg->run,
                               (uint64_t)(l + 1), (uint64_t)r, NULL);
      evals += P * t_new;
      rec->n_acc[(int64_t)l * cfg->RmaxRec + (r - 1)] = acc;
      int up = (cfg->kernel == ORC_MALA) ? (1000 * acc > 574 * P) : (4 * acc > P);
      mh += up ? 1 : -1;
      if (mh < 1) mh = 1;
      if (mh > 10) mh = 10;
      if (cfg->replay || cfg->stop_rule == 0) {
        if (r >= R) break;
      } else {
        /* Section 3.3: the higher threshold E2 at dates of interest */
        int at_date = t_new == T || t_new == cfg->burn_in ||
                      (cfg->force_every > 0 && t_new % cfg->force_every == 0);
        double rne_bar = 0.0;
        int G = orc_test_report(m, pop, cfg->test_fn, t_new, rep);
        for (int i = 0; i < G; ++i) rne_bar += rep[i * 4 + 3];
        rne_bar /= G;
        if (rne_bar > (at_date ? cfg->E2 : cfg->E1) || r >= cfg->Rmax) break;
      }
    }
    if (status) break;
    if (rec->moments) {
      int G = orc_num_test_fns(m, cfg->test_fn);
      orc_test_report(m, pop, cfg->test_fn, t_new, rec->moments + (int64_t)l * G * 4);
    }
    rec->R[l] = r;
    t = t_new;
    ++l;
  }
  rec->L = l;
  rec->evals = evals;
  if (!status) {
    double out[3];
    orc_log_ml(l, cfg->J, rec->group_logwbar, out);
    rec->log_ml = out[0];
    rec->nse = out[1];
    rec->log_ml_tilde = out[2];
    /* log score over (b, T]: the cycles starting at or after b */
    rec->log_score = rec->log_score_nse = rec->log_score_tilde = NAN;
    if (cfg->burn_in > 0 && cfg->burn_in < T) {
      int l0 = 0;
      while (l0 < l && (l0 == 0 ? 0 : rec->t_end[l0 - 1]) < cfg->burn_in) ++l0;
      if (l0 > 0 && l0 < l && rec->t_end[l0 - 1] == cfg->burn_in) {
        orc_log_ml(l - l0, cfg->J, rec->group_logwbar + (int64_t)l0 * cfg->J, out);
        rec->log_score = out[0];
        rec->log_score_nse = out[1];
        rec->log_score_tilde = out[2];
      }
    }
  }
  free(anc);
  return status;
}
