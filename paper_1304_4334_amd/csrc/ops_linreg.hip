// Launcher table of the conjugate regression with 1..4 regressors.
#include "model_kernels.h"

namespace smc {

const ModelOps *ops_linreg(const DevModel &m) {
  switch (m.nreg) {
    case 1: return ops_table<Linreg<1>>();
    case 2: return ops_table<Linreg<2>>();
    case 3: return ops_table<Linreg<3>>();
    case 4: return ops_table<Linreg<4>>();
    default: return nullptr;
  }
}

}  // namespace smc
