/*
 * smc.h - C ABI of the MI355X (gfx950) sequential posterior simulator.
 *
 * The library implements the data-parallel path of the adaptive sequential
 * posterior simulator of Durham & Geweke (Sections 3.1-3.3, 4.2 and 5.1):
 * J groups of N particles cycled through Correction (reweight by the
 * incremental likelihood, RSS test), Selection (within-group resampling) and
 * Mutation (random-walk Metropolis with the particle covariance), where each
 * Metropolis step evaluates the full-data log-likelihood recursion of every
 * particle.
 *
 * Conventions for every call:
 *  - Return value: SMC_OK (0) or a negative smc_status.  Argument errors are
 *    detected before anything is enqueued.  A HIP launch failure returns
 *    SMC_E_DEVICE; smc_last_error() gives a thread-local message.
 *  - Memory: every array argument is caller-owned DEVICE memory unless the
 *    comment says host.  The library never allocates device memory; scratch
 *    comes from the caller's workspace (smc_workspace_bytes).
 *  - Layout: particle p = j*N + n (group j, member n), P = J*N.  Parameter
 *    arrays are parameter-major, theta[i*P + p] for i < d; states likewise
 *    state[k*P + p] for k < S.  All such arrays hold FP64, except the state of
 *    a model created with SMC_FP32, which holds float.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  All
 *    device work is enqueued on it.  Only the calls documented as
 *    synchronising wait for it.
 *  - Random numbers: Philox4x64-10 (Salmon et al. 2011) keyed by
 *    (rng.seed, rng.run) with counters (index, cycle, iteration, purpose),
 *    so results do not depend on launch geometry.
 *  - A non-finite per-particle density is not an error: its weight becomes
 *    zero (log weight -inf) or the proposal is rejected.
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smc_status;
#define SMC_OK 0
#define SMC_E_INVALID_ARG (-1) /* bad pointer, size, enum or shape */
#define SMC_E_UNSUPPORTED (-2) /* valid request the library does not provide */
#define SMC_E_DEVICE (-3)      /* a HIP call failed */
#define SMC_E_NUMERIC (-4)     /* a group lost all weight, or V is not PD */
#define SMC_E_WORKSPACE (-5)   /* workspace smaller than smc_workspace_bytes */

/* Model family (Section 5.1; the regression is the conjugate test model). */
#define SMC_MODEL_LINREG 1 /* y_t = x_t' beta + e_t, e_t ~ N(0, s2) */
#define SMC_MODEL_EGARCH 2 /* eqs EGARCH_mod1/2 with K factors */
#define SMC_SHOCK_GAUSS 0
#define SMC_SHOCK_STUDENT_T 1 /* unit-variance Student-t(nu) shocks */
#define SMC_SHOCK_MIXTURE 2   /* I-component normal mixture, eq normal_mixture */
/* Arithmetic of the likelihood recursion.  Log weights, log-likelihood sums,
 * logsumexp, covariance, Cholesky, the marginal likelihood and its NSE are
 * FP64 in both cases. */
#define SMC_FP64 0
#define SMC_FP32 1

#define SMC_RESAMPLE_RESIDUAL 0    /* Section 3.3 default */
#define SMC_RESAMPLE_MULTINOMIAL 1
#define SMC_RESAMPLE_STRATIFIED 2  /* Section 3.3, experimental (Kitagawa 1996) */
#define SMC_RESAMPLE_SYSTEMATIC 3  /* Section 3.3, experimental (Carpenter et al. 1999) */

#define SMC_KERNEL_RW 0   /* Gaussian random walk, Section 3.3 (default) */
#define SMC_KERNEL_MALA 1 /* preconditioned Langevin proposal (extension) */
#define SMC_KERNEL_INDEPENDENT 2 /* independent Gaussian sampler, Section 3.3 (experimental) */

#define SMC_FLAG_DEAD_GROUP 1 /* a group had no positive weight (S phase) */
#define SMC_FLAG_NOT_PD 2     /* particle variance not positive definite */

/* Model description.  The parameter vector theta (dimension d) is:
 *   LINREG: (beta_1..beta_k, log s2), d = k + 1, prior beta | s2 ~
 *           N(0, 100 s2 I), s2 ~ InvGamma(2, 1) (conjugate);
 *   EGARCH: (theta_1, theta_2, theta_3k.., theta_4k.., theta_5k..) with
 *           Table 1's transforms and Gaussian priors, followed by log(nu - 2)
 *           ~ N(log 10, 1) for Student-t shocks, or by theta_6i.., theta_7i..,
 *           theta_8i.. (i = 1..I) for normal-mixture shocks, transformed by
 *           eqs EGARCH_tran1/2 and with theta_8i ~ N(0, 1) truncated below
 *           at -3 (Table 1; egarch_KI of Section 5.1).  d = 2 + 3K, +1 for
 *           Student-t, +3I for mixtures; state S = K + 1 (the K factors and
 *           the previous standardised shock).  Gaussian and Student-t
 *           shocks: K in {1, 2}; mixtures: K in 1..4, I in 2..4 (FP64 or
 *           FP32). */
typedef struct {
  int32_t kind;      /* SMC_MODEL_* */
  int32_t K;         /* EGARCH factors (see above) */
  int32_t shock;     /* SMC_SHOCK_* (EGARCH) */
  int32_t nreg;      /* regressors k, 1..8 (LINREG) */
  int32_t precision; /* SMC_FP64 or SMC_FP32 (FP32: EGARCH only) */
  int32_t ncomp;     /* mixture components I (SMC_SHOCK_MIXTURE), else 0 */
  int64_t T;         /* observations, >= 1 */
  const double *y;   /* device [T] */
  const float *y32;  /* device [T], y as float; required for SMC_FP32 */
  const double *X;   /* device [T][nreg] row-major (LINREG), else NULL */
} smc_model_desc;

/* Opaque, immutable after creation; may be used from several streams.  The
 * device arrays it points to must outlive it. */
typedef struct smc_model smc_model;

/* A particle population; every pointer is caller-owned device memory. */
typedef struct {
  int32_t J, N;       /* groups and particles per group, J >= 2, N >= 2 */
  double *theta;      /* [d][P] */
  double *logprior;   /* [P] log p(theta_p) */
  double *loglik;     /* [P] log p(y_{1:t} | theta_p) at the current date */
  void *state;        /* [S][P] recursion state at the current date (NULL if S = 0) */
  double *logw;       /* [P] log C-phase weight */
  double *grad;       /* [d][P] gradient of log prior + log likelihood, MALA only, else NULL */
  int32_t *ancestor;  /* [P] last S-phase ancestors */
  void *ws;           /* workspace, >= smc_workspace_bytes(...) bytes, 256-byte aligned */
  size_t ws_bytes;
} smc_particles;

typedef struct {
  uint64_t seed; /* Philox key word 0 */
  uint64_t run;  /* Philox key word 1 (independent runs) */
} smc_rng;

/* --- models and sizing -------------------------------------------------- */

/* Validates the description and creates a handle (host allocation only). */
smc_status smc_model_create(const smc_model_desc *desc, smc_model **out);
smc_status smc_model_destroy(smc_model *m);
/* Launch shape of the model's random-walk step (smc_mutate, smc_run) and of
 * its runs' share of a batch: particles per block, 64, 128 or 256 (one
 * thread each; smc_run's 256-particle step blocks have one more wave, which
 * forms the proposal scale), and observations per load batch of the
 * likelihood loop, 4, 8 or 16 (0 = the defaults 64 and 8).  A shape changes only the speed: every shape gives
 * the same results to the bit.  Shapes other than the default exist for
 * EGARCH(1) with Gaussian shocks and EGARCH(2) with Student-t shocks
 * (SMC_E_UNSUPPORTED otherwise).  The handle is changed: call it before the
 * model is in use on any stream.  tune.py chooses shapes by timing them. */
smc_status smc_model_set_launch(smc_model *m, int32_t block, int32_t unroll);
int32_t smc_model_dim(const smc_model *m);       /* d, or -1 for NULL */
int32_t smc_model_state_dim(const smc_model *m); /* S, or -1 for NULL */

/* Workspace bytes needed by a population of J x N particles whose C phases
 * are evaluated in chunks of at most `max_chunk` observations (0 = default
 * 256).  The same workspace serves every call below. */
size_t smc_workspace_bytes(const smc_model *m, int32_t J, int32_t N, int64_t max_chunk);

/* --- the seven calls of the simulator --------------------------------- */

/* Algorithm 1 step 1: theta_p ~ p(theta) (counter (p, 0, 0, PRIOR)),
 * logprior, loglik = 0, logw = 0, state = the initial state s0. */
smc_status smc_init_from_prior(const smc_model *m, smc_particles *pop, smc_rng rng,
                               void *stream);

/* C phase of cycle `cycle` (Algorithm 1 step 2a, eq C_phase_compute): sets
 * logw = 0 and, for s = t_from+1, ..., adds log p(y_s | y_{1:s-1}, theta_p)
 * to logw_p and loglik_p while advancing the state.  At every check date (s a
 * multiple of `check_every`, and s = t_max) the pooled RSS = (sum w)^2 /
 * (P sum w^2) is formed (Section 3.3); the phase stops at the first check
 * date with RSS < rss_min, or at t_max.  Writes group_logwbar[j] = log(N^-1
 * sum_n w_jn) (device [J], Section 4.2), *t_to (host) = the end date and,
 * when rss is not NULL, *rss (host) = the RSS there.
 * With rss_min <= 0 the phase runs to t_max; if in addition rss is NULL the
 * call does not synchronise (capturable).  Otherwise it waits once per
 * evaluated chunk of observations for that chunk's stopping decision, which
 * a kernel takes on the device and stores in a page-locked slot of the
 * calling host thread; the commit to the decided date is queued before the
 * wait and may still be running when the call returns. */
smc_status smc_correct(const smc_model *m, smc_particles *pop, int64_t t_from, int64_t t_max,
                       int64_t check_every, double rss_min, double *group_logwbar,
                       int64_t *t_to, double *rss, void *stream);

/* The same C phase (Algorithm 1 step 2a, with Section 3.3's stopping rule)
 * with its outputs in device memory and no host synchronisation: *t_to
 * (device int64 [1]) = the end date and, when rss is not NULL, *rss (device
 * double [1]) = the RSS there; group_logwbar as for smc_correct.  The results
 * are those of smc_correct, to the bit.  Argument errors are those of
 * smc_correct; a numerical problem shows in smc_flags afterwards.  Every stopping decision is taken and applied
 * on the device (the state lives in the workspace): smc_correct's sequence of
 * chunks (16 observations, doubling up to the workspace's capacity) is
 * enqueued up front, enough to reach t_max, and the chunks after the phase's
 * end return at once, so the call can be captured in a graph.  Calls that
 * overlap on one population race. */
smc_status smc_correct_async(const smc_model *m, smc_particles *pop, int64_t t_from,
                             int64_t t_max, int64_t check_every, double rss_min,
                             double *group_logwbar, int64_t *t_to, double *rss, void *stream);

/* S phase (Algorithm 1 step 2b) in every group independently: residual
 * (Section 3.3 default) or multinomial resampling on logw.  Residual: copy n
 * floor(N W_n) times, then draw the remaining R = N - sum floor(N W_n) from
 * the residuals N W_n - floor(N W_n); draw k of group j uses word k%4 of
 * Philox(j, cycle, k/4, RESAMPLE) as u in [0,1) and selects the first n whose
 * running residual sum exceeds u times the total.  Ancestors are written in
 * ascending order to pop->ancestor; theta, logprior, loglik, state and grad
 * (if not NULL) are replaced by the ancestors'.  A group without positive
 * weight keeps its particles and raises SMC_FLAG_DEAD_GROUP (smc_flags).
 * Stratified and systematic schemes take the k-th of N draws at (k + U_k)/N,
 * respectively (k + U)/N, of the running sum of W_n (U: draw 0's uniform). */
smc_status smc_resample(const smc_model *m, smc_particles *pop, int32_t scheme, smc_rng rng,
                        int32_t cycle, void *stream);

/* One Metropolis iteration (Algorithm 1 step 2c, Section 3.3) at date t for
 * every particle: z ~ N(0, I_d) from Philox(p, cycle, iter, PROPOSAL | b<<8)
 * by Box-Muller, theta' = theta + hL z (hchol: device [d][d] row-major lower
 * triangular, hL with Sigma = hL hL' = h^2 V); accept iff
 * log u < log p(theta') + log p(y_{1:t}|theta') - (same at theta), u in (0,1)
 * from Philox(p, cycle, iter, ACCEPT).  The likelihood is the full recursion
 * over 1..t from s0.  Accepted particles take theta', logprior, loglik and the
 * state at t.  With kernel = SMC_KERNEL_MALA the proposal mean adds
 * (1/2) hL hL' grad and the acceptance includes the proposal-density ratio;
 * pop->grad must hold the gradient at the current particles and is updated.
 * With kernel = SMC_KERNEL_INDEPENDENT, hchol holds L (d x d, V = L L') followed
 * by the particle mean m [d]: theta' = m + L z whatever the current particle,
 * and the acceptance includes log q(theta) - log q(theta') for q = N(m, V).
 * The number accepted is ADDED to *n_accept (device int64); accepted
 * (device [P] bytes, may be NULL) receives the 0/1 decisions. */
smc_status smc_mutate(const smc_model *m, smc_particles *pop, int64_t t, int32_t kernel,
                      const double *hchol, smc_rng rng, int32_t cycle, int32_t iter,
                      int64_t *n_accept, uint8_t *accepted, void *stream);

/* log p(y_{1:t} | theta_p) for P parameter vectors (theta device [d][P]) by
 * the model's recursion from s0 (eq p(y|theta) as a product of
 * p(y_s | y_{1:s-1}, theta)).  loglik: device [P]; state_out: device [S][P]
 * (precision of the model) or NULL. */
smc_status smc_loglik(const smc_model *m, int64_t P, const double *theta, int64_t t,
                      double *loglik, void *state_out, void *stream);

/* Adjoint of smc_loglik: dtheta[i][p] = dloglik[p] * d log p(y_{1:t}|theta_p)
 * / d theta_ip.  The forward recursion is checkpointed every 64 observations
 * (FP32 models; 32 for FP64) into ws (>= smc_backward_ws_bytes bytes, device)
 * and replayed segment by segment in reverse through a per-lane LDS buffer.
 * d|x|/dx is taken as 0 at x = 0. */
smc_status smc_loglik_backward(const smc_model *m, int64_t P, const double *theta, int64_t t,
                               const double *dloglik, double *dtheta, void *ws,
                               size_t ws_bytes, void *stream);
size_t smc_backward_ws_bytes(const smc_model *m, int64_t P, int64_t t);

/* grad[i][p] = d/dtheta_i [log p(theta_p) + log p(y_{1:t} | theta_p)] for every
 * particle (pop->grad must be set; uses the workspace tail for checkpoints,
 * see smc_mala_workspace_bytes).  The Langevin kernel needs it at each new
 * date before its first iteration. */
smc_status smc_posterior_grad(const smc_model *m, smc_particles *pop, int64_t t, void *stream);

/* Workspace bytes for a population that also runs the Langevin kernel or
 * smc_posterior_grad at any date up to T (the checkpoints share the tail of
 * the workspace with the C-phase chunks). */
size_t smc_mala_workspace_bytes(const smc_model *m, int32_t J, int32_t N, int64_t max_chunk);

/* Marginal likelihood from the per-cycle group mean weights (Section 4.2):
 * group_logwbar: device [L][J] (log wbar_j(l-1)); out: device [3] =
 * { log wbar, NSE of log wbar by the delta method of eq ML_se, log wtilde }. */
smc_status smc_log_ml(int32_t L, int32_t J, const double *group_logwbar, double *out,
                      void *stream);

/* Log score over a burn-in (Section 3.3's software outputs; Section 4.2):
 * log p(y_{b+1:T} | y_{1:b}) from the cycles that start at or after the
 * burn-in date b, which must be a cycle end (t_end: host [L], the dates of
 * the L cycles).  out: device [3] as for smc_log_ml.  SMC_E_INVALID_ARG if no
 * cycle ends at b. */
smc_status smc_log_score(int32_t L, int32_t J, const double *group_logwbar, const int64_t *t_end,
                         int64_t burn_in, double *out, void *stream);

/* --- functions of interest (Sections 2.3 and 5.2) ------------------------ */

#define SMC_TEST_PARAMS 0 /* g_i(theta) = theta_i */
#define SMC_TEST_MODEL 1  /* the model's functions of interest, see below */

/* Number of test functions: d for SMC_TEST_PARAMS; for SMC_TEST_MODEL, EGARCH
 * has Section 5.2's g1 = log sigma_Y + sum_k v_kt / 2 (log volatility at the
 * current date), g2 = E(eps^3) (mixture shocks only; zero for symmetric
 * shocks) and g3 = P(Y_{t+1} < -0.03 | theta, y_{1:t}) (with the shock's
 * distribution function: normal, unit-variance Student-t or the mixture), in
 * that order; the regression uses its parameters.  -1 for a NULL model or a
 * bad `which`. */
int32_t smc_num_test_functions(const smc_model *m, int32_t which);

/* Posterior moments of the test functions over the (equally weighted)
 * population at date t: out device [G][4] = (mean, standard deviation with
 * divisor NJ - 1, NSE of eq NSE_def, RNE = var-hat / v-hat of eq vhat), from
 * the J group means (Section 2.3).  The state must be the one at date t.
 * Uses the workspace. */
smc_status smc_test_moments(const smc_model *m, smc_particles *pop, int64_t t, int32_t which,
                            double *out, void *stream);

/* --- helpers of the M phase -------------------------------------------- */

/* Pooled particle mean (device [d]), variance V with divisor P - 1 (device
 * [d][d]) and hchol = h L with V = L L' and h = (*mh) / 10 (mh: device int32
 * holding h in tenths, Section 3.3).  mean and cov may be NULL.  A variance
 * that is not positive definite raises SMC_FLAG_NOT_PD and leaves hchol
 * zero (a zero step: every proposal equals the current particle). */
smc_status smc_particle_moments(const smc_model *m, const smc_particles *pop, const int32_t *mh,
                                double *mean, double *cov, double *hchol, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): smc_particle_moments
 * with the same arguments, results and error behaviour, except that pop->ws is
 * not used (it may be NULL).  The scratch of its kernels (up to 129 moment
 * matrices of 32 x 32 doubles, then a flags word: SMC_MOMENTS_SCRATCH_BYTES in
 * all) lives in a static device array that each GPU the library runs on holds
 * until the process ends; the call allocates nothing.  Every call on a GPU
 * shares that GPU's array and clears its flags word first, so calls that
 * overlap on one GPU race.  A variance that is not positive definite leaves
 * hchol zero (hchol[0] == 0; the flag is not reported).  SMC_E_WORKSPACE if a
 * population's partials would exceed the array (never for d < 32). */
#define SMC_MOMENTS_SCRATCH_BYTES 1057024
smc_status smc_particle_moments_noalloc(const smc_model *m, const smc_particles *pop,
                                        const int32_t *mh, double *mean, double *cov,
                                        double *hchol, void *stream);

/* Step-size rule of Section 3.3 on device: with a = *n_accept / P,
 * *mh += 1 if a > target_permille / 1000 else *mh -= 1, clamped to [1, 10].
 * The comparison is exact in integers. */
smc_status smc_adapt_scale(const int64_t *n_accept, int64_t P, int32_t target_permille,
                           int32_t *mh, void *stream);

/* Mean over the parameters of RNE = var-hat / v-hat with g_i(theta) = theta_i
 * (Section 2.3): device double [1]. */
smc_status smc_rne(const smc_model *m, const smc_particles *pop, double *rne, void *stream);

/* Reads and clears the SMC_FLAG_* bits raised in the workspace (host int32;
 * synchronises the stream). */
smc_status smc_flags(const smc_particles *pop, int32_t *flags, void *stream);

/* --- the whole simulator ------------------------------------------------ */

/* Algorithm 2 with the rules of Section 3.3 (adaptive), or Algorithm 1 on a
 * recorded design {t_l, Sigma_lr, R_l} (replay = step 2 of Algorithm 3). */
typedef struct {
  int32_t J, N;
  smc_rng rng;
  int32_t check_every;  /* RSS check dates: every k-th observation (1) */
  int32_t force_every;  /* dates of interest: cycle ends every k-th obs (0 = none) */
  double D1, D2;        /* 0.5, 0.2 */
  int32_t Rbar, kappa;  /* 7, 3 */
  int32_t stop_rule;    /* 0 deterministic R_l, 1 RNE-based */
  double E1;            /* 0.35 */
  int32_t Rmax;         /* 100 */
  int32_t scheme;       /* SMC_RESAMPLE_* */
  int32_t kernel;       /* SMC_KERNEL_* */
  int32_t replay;       /* 0 adaptive, 1 replay the record's design */
  int32_t Lmax;         /* record capacity in cycles */
  int32_t RmaxRec;      /* record capacity in iterations per cycle */
  int64_t max_chunk;    /* C-phase chunk bound, as given to smc_workspace_bytes */
  int32_t test_fn;      /* SMC_TEST_*: the RNE rule's functions and the moment reports */
  int32_t graph;        /* 0: host-driven cycles; 1: device-driven (see smc_run) */
  double E2;            /* 0.90: RNE threshold after a C phase that ends at a date of
                           interest (a multiple of force_every, burn_in or T) */
  int64_t burn_in;      /* log-score burn-in date b, a date of interest (0 = none) */
} smc_run_config;

typedef struct {
  int32_t L;             /* out: cycles run */
  int32_t time_every;    /* with mutate_ms: time every k-th Metropolis iteration of
                            the run, counted from the first (0 or 1: every one) */
  int64_t *t_end;        /* host [Lmax]: out (adaptive) / in (replay) */
  int32_t *R;            /* host [Lmax]: out / in */
  double *rss;           /* host [Lmax]: out, RSS at the end of each C phase */
  int64_t *n_accept;     /* device [Lmax][RmaxRec]: out, accepted per iteration */
  double *hchol;         /* device [Lmax][RmaxRec][d][d]: out / in */
  double *group_logwbar; /* device [Lmax][J]: out */
  double *log_ml;        /* device [3]: out, as smc_log_ml */
  int64_t evals;         /* out: particle x observation density evaluations */
  int64_t mh_steps;      /* out: Metropolis iterations */
  float *mutate_ms;      /* host [Lmax][RmaxRec] or NULL: when given, each timed
                            mutation launch (time_every) carries HIP start and
                            stop events on its own dispatch (a Langevin step,
                            several kernels, is bracketed by two event records)
                            and its duration in ms is stored here; the entries
                            of untimed launches are -1 */
  double *moments;       /* device [Lmax][G][4] or NULL: smc_test_moments of
                            cfg->test_fn at the end of every cycle */
  double *log_score;     /* device [3] or NULL: smc_log_score over cfg->burn_in */
  double *mean;          /* device [Lmax][RmaxRec][d]: the particle means of the
                            independent sampler (out / in); NULL otherwise */
} smc_run_record;

/* Runs the simulator on `pop` (which must hold a workspace for
 * cfg->max_chunk): Algorithm 2 with the Section 3.3 rules, or Algorithm 1
 * on the recorded design when cfg->replay is set.  The host waits once per
 * C-phase chunk for the chunk's stopping decision (taken on the device; the
 * commit and, should the phase end there, the S phase are queued before the
 * wait), once per M iteration under the RNE rule, and once after the last
 * cycle (for its numerical flags); the log-ML is queued after that.  In an adaptive random-walk run each Metropolis step also
 * computes its proposal scale (the step-size rule, V and h L, recorded in
 * rec->hchol) from the moment partials itself.
 *
 * With cfg->graph = 1 the adaptive random-walk run with deterministic R_l
 * (stop_rule 0, no moment reports or timings, kappa * Rbar <= RmaxRec,
 * Lmax <= 4096) is driven on the device: every stopping decision, the choice
 * of R_l, the cycle's record and the next chunk are taken by kernels, and the
 * host launches one captured step (a C-phase chunk, the S phase, Rbar M
 * iterations, the step's end) until the run has ended, keeping up to three
 * steps queued and never waiting for a decision.  The results are the
 * host-driven run's, bit for bit.  The step graph is captured on the first
 * such call for a given model, population, record and rule set, and launched
 * again by later calls with the same ones (whatever their Philox key); the
 * graph reads the key, dates, counters and record slots from the workspace,
 * so calls that overlap on one population race.  SMC_E_UNSUPPORTED for the other configurations. */
smc_status smc_run(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                   smc_run_record *rec, void *stream);

/* Algorithm 3 (hybrid): step 1 runs the adaptive simulator with cfg (cfg->replay
 * must be 0) into rec1 and retains its design {t_l, Sigma_lr, R_l}; step 2
 * replays that design into rec2 with the new Philox key (seed2, cfg->rng.run)
 * for every draw, so step 2 is a run of Algorithm 1 (Proposition 3).  The two
 * records need the same capacities; rec2's design arrays are overwritten.
 * seconds (host double [2], may be NULL) receives each step's wall time,
 * stream synchronised.  pop ends with step 2's particles. */
smc_status smc_run_hybrid(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                          uint64_t seed2, smc_run_record *rec1, smc_run_record *rec2,
                          double *seconds, void *stream);

/* The agreement of Algorithm 3's two steps (Section 3.4's comparison of
 * independent estimates): out (host double [2]) receives
 * |a - b| / sqrt(NSE_a^2 + NSE_b^2) for the log-ML of rec1 and rec2
 * (log_ml[0..1] of each) and, when both records carry a log score, for the
 * log score (else NaN).  Reads the device estimates on `stream` and
 * synchronises it. */
smc_status smc_hybrid_report(const smc_run_record *rec1, const smc_run_record *rec2,
                             double *out, void *stream);

/* --- many runs at once (extension: batching) -------------------------- */

/* Device workspace bytes of a batch of n_runs runs (1..32). */
size_t smc_batch_ws_bytes(int32_t n_runs);

/* Optional timing of a batch's persistent M-step launches: each launch
 * carries HIP start and stop events on its own dispatch.  Host arrays. */
typedef struct {
  int32_t capacity; /* in: entries of ms (and pairs of evals) */
  int32_t launches; /* out: launches recorded (at most capacity; later ones untimed) */
  float *ms;        /* [capacity]: duration of each launch in ms */
  int64_t *evals;   /* [capacity][2]: the launch's particle x observation evaluations,
                       by EGARCH(1) Gaussian runs and by EGARCH(2) Student-t runs */
} smc_batch_timing;

/* Runs n independent simulators (each with its own model, population and
 * workspace, configuration and record, as for smc_run) together.  The runs
 * must share one recursion precision and one Metropolis kernel (the random
 * walk, or the Langevin step: then every population needs pop->grad and a
 * workspace of smc_mala_workspace_bytes), use EGARCH(1) Gaussian or EGARCH(2)
 * Student-t models and the deterministic R_l rule, and either all adapt or
 * all replay.  At every step of the batch, the M
 * iterations of all runs then in their M phase go to one persistent kernel
 * launch in which each block takes (run, block of particles) items, longest
 * date first, from a device counter until they are exhausted; their moments
 * go to one pair of launches; C-phase chunks of different runs share one
 * host synchronisation.  `waves` is the number of persistent waves (0 =
 * 2048).  FP32 random-walk batches take the launch shape set on their first
 * model (smc_model_set_launch: particles per block and item, observations
 * per load batch); other batches use 64 and 8.  bws: device, >= smc_batch_ws_bytes(n), 256-byte aligned.  A replay
 * batch never synchronises the stream (capturable in a graph); an adaptive
 * one synchronises once per batch step that evaluates C-phase chunks, and
 * stops with SMC_E_NUMERIC at the first such readback after a run raised a
 * numerical flag.  timing may be NULL (when given, the call synchronises at
 * its end to read the events).  Each run's results equal those of smc_run
 * with the same arguments. */
smc_status smc_run_batch(int32_t n, const smc_model *const *models, smc_particles *const *pops,
                         const smc_run_config *cfgs, smc_run_record *recs, void *bws,
                         size_t bws_bytes, int32_t waves, smc_batch_timing *timing,
                         void *stream);

/* --- diagnostics ------------------------------------------------------- */
const char *smc_status_string(smc_status s);
const char *smc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H */
