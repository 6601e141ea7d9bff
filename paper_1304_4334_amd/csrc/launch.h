// Host-side launchers of the device kernels (kernels.hip) used by the C ABI
// (abi.hip).  Each enqueues on the given stream and returns SMC_OK or
// SMC_E_DEVICE.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace smc {

template <class T>
struct Tag {
  using type = T;
};

// Records a thread-local message and returns `status`.
smc_status set_error(smc_status status, const char *fmt, ...);

smc_status fill_f64(double *a, int64_t n, double v, hipStream_t s);
smc_status fill_i64(int64_t *a, int64_t n, int64_t v, hipStream_t s);
smc_status fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t s);

// Optional timing of one launch: the two events take the start and end
// stamps of the kernel's own dispatch (no packets of their own on the
// stream).  Both created by the caller with timing enabled; NULL = untimed.
struct KernelTimer {
  hipEvent_t start, stop;
};

// The proposal scale folded into the random-walk step (d < 32): each block
// sums the moment partials, applies the step-size rule and factors the
// particle variance itself, with the arithmetic of the separate moments
// kernels (so the results agree to the bit); block 0 writes the step size and
// h L for the record.
struct MomFuse {
  const double *part;        // [nb][W * W] partial sums, W = 16 (d < 16) or 32; NULL: unfused
  int32_t nb;
  int32_t mh_reset;          // > 0: the step size is set to this value
  const int32_t *mh_in;      // the previous iteration's step size (tenths)
  int32_t *mh_out;           // this iteration's, written by block 0
  const int64_t *prev_nacc;  // the previous iteration's accepts, or NULL
  int32_t target_permille;   // step-size rule target
  int32_t pad;
  double *hchol_out;         // h L (d x d row-major) for the record, by block 0
  int32_t *flags;            // SMC_FLAG_NOT_PD when the variance is not positive definite
};

// Launchers of the kernels templated on the model, one table per model type
// (model_kernels.h); the family tables below return NULL for a description
// they do not cover.
struct ModelOps {
  smc_status (*init)(const DevModel &, int64_t, uint64_t, uint64_t, double *, double *, double *,
                     void *, double *, hipStream_t);
  smc_status (*cscan)(const DevModel &, int64_t, const double *, const void *, const double *,
                      int64_t, int64_t, int64_t, int64_t, bool, double *, hipStream_t);
  smc_status (*ccommit)(const DevModel &, int64_t, const double *, void *, double *, double *,
                        int64_t, int64_t, bool, const int64_t *, hipStream_t);
  smc_status (*mutate_rw)(const DevModel &, int64_t, int64_t, double *, double *, double *,
                          void *, const double *, uint64_t, uint64_t, uint64_t, uint64_t,
                          int64_t *, uint8_t *, const KernelTimer *, const MomFuse *,
                          hipStream_t);
  smc_status (*loglik)(const DevModel &, int64_t, const double *, int64_t, double *, void *,
                       hipStream_t);
  size_t (*ckpt_bytes)(const DevModel &, int64_t, int64_t);
  smc_status (*loglik_backward)(const DevModel &, int64_t, const double *, int64_t,
                                const double *, double *, void *, hipStream_t);
  smc_status (*grad_post)(const DevModel &, int64_t, const double *, int64_t, double *, void *,
                          hipStream_t);
  smc_status (*mutate_mala)(const DevModel &, int64_t, int64_t, double *, double *, double *,
                            void *, double *, const double *, uint64_t, uint64_t, uint64_t,
                            uint64_t, int64_t *, uint8_t *, void *, hipStream_t);
  int32_t (*num_tests)(int32_t which);
  smc_status (*test_fns)(const DevModel &, int64_t, const double *, const void *, int64_t,
                         int32_t, double *, hipStream_t);
  smc_status (*mutate_indep)(const DevModel &, int64_t, int64_t, double *, double *, double *,
                             void *, const double *, const double *, uint64_t, uint64_t,
                             uint64_t, uint64_t, int64_t *, uint8_t *, const KernelTimer *,
                             hipStream_t);
};
const ModelOps *ops_linreg(const DevModel &m);     // ops_linreg.hip
const ModelOps *ops_egarch(const DevModel &m);     // ops_egarch.hip: Gaussian, Student-t
const ModelOps *ops_mixture64(const DevModel &m);  // ops_mixture64.hip
const ModelOps *ops_mixture32(const DevModel &m);  // ops_mixture32.hip
// The table for a model description, or NULL (error recorded) if none.
const ModelOps *ops_for(const DevModel &m);

smc_status launch_init(const DevModel &m, int64_t P, uint64_t seed, uint64_t run, double *theta,
                       double *logprior, double *loglik, void *state, double *logw,
                       hipStream_t s);
// zero_first: treat the log weights as zero on entry (the first call of a C
// phase), which saves a separate fill.
smc_status launch_cscan(const DevModel &m, int64_t P, const double *theta, const void *state,
                        const double *logw, int64_t t0, int64_t t1, int64_t check_every,
                        int64_t t_max, bool zero_first, double *W, hipStream_t s);
// t1_dev (may be NULL): the commit's end date read on the device (at most t1).
smc_status launch_ccommit(const DevModel &m, int64_t P, const double *theta, void *state,
                          double *logw, double *loglik, int64_t t0, int64_t t1, bool zero_first,
                          hipStream_t s, const int64_t *t1_dev = nullptr);
// RSS of ncols columns; with ncols_dev (a device-driven chunk) of the first
// *ncols_dev <= ncols columns.  rss is the workspace's RSS region:
// [kMaxChunk] values, then rss_slice_doubles(P) doubles of partial sums of
// columns longer than one slice.
smc_status launch_rss_cols(const double *W, int64_t P, int64_t ncols, double *rss,
                           hipStream_t s, const int32_t *ncols_dev = nullptr);
int64_t rss_slice_doubles(int64_t P);
// RSS of the C-phase scan's recorded dates from its per-wave sums (trip, as
// k_cscan writes them: [ncols][ceil(P/64)][3] doubles); with ncols_dev (a
// device-driven chunk) of the first *ncols_dev <= ncols dates.
smc_status launch_rss_scan(const double *trip, int64_t P, int64_t ncols, double *rss,
                           hipStream_t s, const int32_t *ncols_dev = nullptr);
smc_status launch_group_logwbar(const double *logw, int32_t J, int32_t N, double *out,
                                hipStream_t s);
// The stopping decision over the nc RSS values of the chunk (t, t1] into *out,
// and with *flags into page-locked host memory host_slot (tagged with seq)
// when that is not NULL; with cyc, the chunk and decision of a device-driven
// cycle (the by-value chunk arguments are then unused).
smc_status launch_find_stop(const double *rss, int64_t nc, int64_t t, int64_t t1,
                            int64_t check_every, int64_t t_max, double rss_min, StopInfo *out,
                            hipStream_t s, DecisionSlot *host_slot = nullptr, uint32_t seq = 0,
                            const int32_t *flags = nullptr, CycleDyn *cyc = nullptr);
// Resampling and the replacement of every particle by its ancestor, one block
// per group; with `go` (device flag, may be NULL) the kernel does nothing
// while *go is 0; with group_logwbar (may be NULL) it also writes each
// group's log mean weight, as launch_group_logwbar does.  With cyc, the S
// phase of a device-driven cycle: it runs when the step's C phase ended, with
// counter l + 1 and group weights in record row l.
smc_status launch_resample(const double *logw, int32_t J, int32_t N, int32_t scheme,
                           uint64_t seed, uint64_t run, uint64_t cycle, int32_t *anc,
                           double *cum_ws, int32_t *flags, int32_t d, int32_t S, int32_t st_bytes,
                           double *theta, double *logprior, double *loglik, void *state,
                           double *grad, double *tmp, hipStream_t s,
                           const int32_t *go = nullptr, double *group_logwbar = nullptr,
                           const CycleDyn *cyc = nullptr);
// Device-driven cycles (CycleDyn): the state's start, and the end of a step
// (record, counters, the next chunk; progress word in mapped host memory).
smc_status launch_cycle_init(CycleDyn *c, const CycleDyn &init, hipStream_t s);
smc_status launch_cycle_end(CycleDyn *c, int64_t *t_end, int32_t *r_rec, double *rss_rec,
                            const int32_t *flags, uint32_t *host, const AccSink &acc,
                            hipStream_t s);
// Adds the pending accept counts of a P-particle Metropolis step to their
// counter (AccSink); nothing pending: nothing to do.
smc_status launch_acc_flush(const AccSink &acc, int64_t P, hipStream_t s);
// A C phase driven on the device (smc_correct_async): open the first chunk,
// advance after each chunk, copy the end date and RSS to the caller (with
// c NULL: t_fixed and *rss_src).
smc_status launch_phase_init(CycleDyn *c, const CycleDyn &init, hipStream_t s);
smc_status launch_phase_step(CycleDyn *c, hipStream_t s);
smc_status launch_phase_out(const CycleDyn *c, const double *rss_src, int64_t t_fixed,
                            int64_t *t_to, double *rss, hipStream_t s);
struct MomArgs {
  const double *theta;
  int64_t P;
  int32_t d;
  int32_t target_permille;  // step-size rule target when prev_nacc is given
  double *part;             // [kMomBlocks][W*W] partial sums, W = 16 or 32 (workspace)
  int32_t *mh;              // step size in tenths (device)
  const int64_t *prev_nacc; // accepts of the previous iteration, or NULL
  int32_t mh_reset;         // > 0: set mh to this value first
  int32_t slot;             // with cyc: the M slot of a device-driven step (partials only)
  double *mean_out, *cov_out, *hchol;
  int32_t *flags;
  const CycleDyn *cyc;      // device-driven cycle, else NULL
  AccSink acc;              // with acc.pending: the partials' launch also adds the
                            // previous step's pending accept counts (acc_flush)
};
smc_status launch_moments(const MomArgs &a, hipStream_t s);
// Only the partial sums of launch_moments, for a step that folds the rest in
// (MomFuse): *part and nb receive the partials to add (for d >= 16 they are
// first summed into one).
smc_status launch_moment_partials(const MomArgs &a, const double **part, int64_t &nb,
                                  hipStream_t s);
// Particles per wave (chunk) and blocks (nb <= kMomBlocks) of the moment
// partials of P particles of dimension d.
void moment_partition(int64_t P, int32_t d, int64_t &chunk, int64_t &nb);
smc_status launch_mutate_rw(const DevModel &m, int64_t P, int64_t t, double *theta,
                            double *logprior, double *loglik, void *state, const double *hchol,
                            uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter,
                            int64_t *n_accept, uint8_t *accepted, hipStream_t s,
                            const KernelTimer *timer = nullptr, const MomFuse *fuse = nullptr);
// The random-walk step in the model's tuned launch shape (m.block threads
// per block, m.unroll observations per load batch), for the models that have
// tuned shapes (ops_shapes32.hip, ops_shapes64.hip, and for egarch_23
// ops_shapes_mix32.hip, ops_shapes_mix64.hip); SMC_E_UNSUPPORTED otherwise.
smc_status launch_mutate_rw_shaped32(const DevModel &m, int64_t P, int64_t t, double *theta,
                                     double *logprior, double *loglik, void *state,
                                     const double *hchol, uint64_t seed, uint64_t run,
                                     uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                     uint8_t *accepted, const KernelTimer *timer,
                                     const MomFuse *fuse, hipStream_t s);
smc_status launch_mutate_rw_shaped64(const DevModel &m, int64_t P, int64_t t, double *theta,
                                     double *logprior, double *loglik, void *state,
                                     const double *hchol, uint64_t seed, uint64_t run,
                                     uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                     uint8_t *accepted, const KernelTimer *timer,
                                     const MomFuse *fuse, hipStream_t s);
smc_status launch_mutate_rw_shaped_mix32(const DevModel &m, int64_t P, int64_t t, double *theta,
                                        double *logprior, double *loglik, void *state,
                                        const double *hchol, uint64_t seed, uint64_t run,
                                        uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                        uint8_t *accepted, const KernelTimer *timer,
                                        const MomFuse *fuse, hipStream_t s);
smc_status launch_mutate_rw_shaped_mix64(const DevModel &m, int64_t P, int64_t t, double *theta,
                                        double *logprior, double *loglik, void *state,
                                        const double *hchol, uint64_t seed, uint64_t run,
                                        uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                        uint8_t *accepted, const KernelTimer *timer,
                                        const MomFuse *fuse, hipStream_t s);
// Whether a model has tuned launch shapes.
bool has_launch_shapes(const DevModel &m);
smc_status launch_loglik(const DevModel &m, int64_t P, const double *theta, int64_t t,
                         double *out, void *state_out, hipStream_t s);
// The independent Gaussian sampler: chol = L (d x d), mean [d].
smc_status launch_mutate_indep(const DevModel &m, int64_t P, int64_t t, double *theta,
                               double *logprior, double *loglik, void *state, const double *chol,
                               const double *mean, uint64_t seed, uint64_t run, uint64_t cycle,
                               uint64_t iter, int64_t *n_accept, uint8_t *accepted,
                               hipStream_t s, const KernelTimer *timer = nullptr);
smc_status launch_adapt(const int64_t *n_accept, int64_t P, int32_t target_permille,
                        int32_t *mh, hipStream_t s);
smc_status launch_rne(const double *theta, int32_t J, int32_t N, int32_t d, double *part,
                      double *rne, hipStream_t s);
smc_status launch_log_ml(int32_t L, int32_t J, const double *g, double *out, hipStream_t s);
// Posterior moment report of G rows g[G][P] (J groups of N): out[G][4] =
// (mean, sd, NSE, RNE); rne_mean (device scalar, may be NULL) = mean RNE.
smc_status launch_report(const double *g, int32_t J, int32_t N, int32_t G, double *part,
                         double *out, double *rne_mean, hipStream_t s);
int32_t num_test_fns(const DevModel &m, int32_t which);  // -1 if unsupported
smc_status launch_test_fns(const DevModel &m, int64_t P, const double *theta, const void *state,
                           int64_t t, int32_t which, double *out, hipStream_t s);

// Bytes of the adjoint checkpoints of P particles over t observations.
size_t adjoint_ckpt_bytes(const DevModel &m, int64_t P, int64_t t);
smc_status launch_loglik_backward(const DevModel &m, int64_t P, const double *theta, int64_t t,
                                  const double *dloglik, double *dtheta, void *ckpt,
                                  hipStream_t s);
smc_status launch_grad_post(const DevModel &m, int64_t P, const double *theta, int64_t t,
                            double *grad, void *ckpt, hipStream_t s);
smc_status launch_mutate_mala(const DevModel &m, int64_t P, int64_t t, double *theta,
                              double *logprior, double *loglik, void *state, double *grad,
                              const double *hchol, uint64_t seed, uint64_t run, uint64_t cycle,
                              uint64_t iter, int64_t *n_accept, uint8_t *accepted, void *ckpt,
                              hipStream_t s);

}  // namespace smc
