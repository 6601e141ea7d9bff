// Device-side descriptors and launchers of the batched driver (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"
#include "launch.h"

namespace smc {

constexpr int kMaxBatch = 32;   // runs per batch call (kernel-argument descriptors)
constexpr int32_t kFamilyFp32 = 1, kFamilyFp64 = 0;

// Per-run data fixed for the whole batch call (device table).
struct BatchStatic {
  double *theta, *logprior, *loglik;
  void *state;
  double *part;     // moment partials (the run's workspace)
  int32_t *mh;      // step size in tenths (the run's workspace)
  int32_t *flags;   // numerical flags (the run's workspace)
  const void *y;    // observations in the recursion's precision
  double *grad;     // [d][P] posterior gradient (Langevin batches), else NULL
  void *ckpt;       // the adjoint's checkpoint area (Langevin batches), else NULL
  uint64_t seed, run;
  int64_t P;
  int32_t tag;      // 0: EGARCH(1) Gaussian, 1: EGARCH(2) Student-t
  int32_t d;
};

// Per-run values of one batch step (kernel argument).
struct BatchDyn {
  double *hchol;                 // this iteration's h L (record slot)
  unsigned long long *n_accept;  // this iteration's accept counter (record slot)
  const int64_t *prev_nacc;      // the previous iteration's, or NULL
  int64_t t;                     // date of the likelihood
  int32_t idx;                   // row of the static table
  int32_t cycle, iter, mh_reset;
  int32_t mut_begin, mom_begin, mom_nb, mom_chunk;
};

struct BatchArgs {
  const BatchStatic *runs;
  unsigned int *queue;  // work counter of the persistent kernel
  int32_t n_active, n_mut_items, n_mom_items, target_permille;
  int32_t kernel;       // SMC_KERNEL_RW or SMC_KERNEL_MALA
  int32_t pad;
  BatchDyn dyn[kMaxBatch];  // active runs, decreasing t
};

struct BatchStaticArgs {
  BatchStatic *dst;
  int32_t n;
  int32_t pad;
  BatchStatic src[kMaxBatch];
};

// timer (may be NULL): start and stop events carried by the persistent
// launch's own dispatch.
// block, unroll: launch shape of the FP32 random-walk batches (threads per
// block and observations per load batch; 0 = 64 and 8); other batches use
// the default.
smc_status launch_batch_m(const BatchArgs &a, bool moments, int32_t family, int32_t waves,
                          hipStream_t s, const KernelTimer *timer = nullptr, int32_t block = 0,
                          int32_t unroll = 0);
smc_status launch_batch_static(const BatchStaticArgs &a, hipStream_t s);

}  // namespace smc
