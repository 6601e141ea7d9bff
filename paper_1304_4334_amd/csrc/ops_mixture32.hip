// Launcher tables of the egarch_KI family with normal-mixture shocks
// (Section 5.1): K = 1..4 factors, I = 2..4 components, FP32 recursion.
#include "model_kernels.h"

namespace smc {

namespace {
template <int K>
const ModelOps *by_components(int I) {
  constexpr int SH = SMC_SHOCK_MIXTURE;
  switch (I) {
    case 2: return ops_table<Egarch<K, SH, float, 2>>();
    case 3: return ops_table<Egarch<K, SH, float, 3>>();
    case 4: return ops_table<Egarch<K, SH, float, 4>>();
    default: return nullptr;
  }
}
}  // namespace

const ModelOps *ops_mixture32(const DevModel &m) {
  switch (m.K) {
    case 1: return by_components<1>(m.ncomp);
    case 2: return by_components<2>(m.ncomp);
    case 3: return by_components<3>(m.ncomp);
    case 4: return by_components<4>(m.ncomp);
    default: return nullptr;
  }
}

}  // namespace smc
