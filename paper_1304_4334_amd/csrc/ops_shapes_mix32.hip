// Every tuned launch shape of the random-walk step for the FP32 recursion of
// egarch_23 (two factors, three-component normal-mixture shocks).
#include "model_kernels.h"

namespace smc {

smc_status launch_mutate_rw_shaped_mix32(const DevModel &m, int64_t P, int64_t t, double *theta,
                                        double *logprior, double *loglik, void *state,
                                        const double *hchol, uint64_t seed, uint64_t run,
                                        uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                        uint8_t *accepted, const KernelTimer *timer,
                                        const MomFuse *fuse, hipStream_t s) {
  const int32_t B = m.block ? m.block : 64, U = m.unroll ? m.unroll : kUnroll;
  if (m.kind == SMC_MODEL_EGARCH && m.K == 2 && m.shock == SMC_SHOCK_MIXTURE && m.ncomp == 3)
    return launch_rw_any_shape<Egarch<2, SMC_SHOCK_MIXTURE, float, 3>>(
        B, U, m, P, t, theta, logprior, loglik, state, hchol, seed, run, cycle, iter, n_accept,
        accepted, timer, fuse, s);
  return set_error(SMC_E_UNSUPPORTED, "no tuned launch shapes for this model");
}

}  // namespace smc
