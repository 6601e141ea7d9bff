// Launcher tables of EGARCH with K = 1 or 2 factors and Gaussian or
// Student-t shocks, FP64 or FP32 recursion.
#include "model_kernels.h"

namespace smc {

const ModelOps *ops_egarch(const DevModel &m) {
  const bool t = m.shock == SMC_SHOCK_STUDENT_T;
  if (m.shock != SMC_SHOCK_GAUSS && !t) return nullptr;
  if (m.prec == SMC_FP64) {
    if (m.K == 1) return t ? ops_table<Egarch<1, 1, double>>() : ops_table<Egarch<1, 0, double>>();
    if (m.K == 2) return t ? ops_table<Egarch<2, 1, double>>() : ops_table<Egarch<2, 0, double>>();
  } else {
    if (m.K == 1) return t ? ops_table<Egarch<1, 1, float>>() : ops_table<Egarch<1, 0, float>>();
    if (m.K == 2) return t ? ops_table<Egarch<2, 1, float>>() : ops_table<Egarch<2, 0, float>>();
  }
  return nullptr;
}

}  // namespace smc
