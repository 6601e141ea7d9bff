// Cholesky factor of the particle variance for the M-phase proposal.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace smc {

// V = L L' by one wave (call from lanes 0..63 of a wave, d < W): lane r keeps
// row r of V (Ms, W x W row-major in LDS) and of L in registers, and row `col`
// of L reaches the other lanes through shuffles, so the factorisation needs
// no block barrier; the operations and their order are those of a
// column-by-column factorisation.  Writes h L (d x d row-major) to hchol; a V
// that is not positive definite gives hchol = 0 and raises SMC_FLAG_NOT_PD.
template <int W>
__device__ __forceinline__ void wave_cholesky(const double *Ms, int d, double h, double *hchol,
                                              int32_t *flags) {
  const int r = threadIdx.x & 63;
  double vr[W], lr[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    vr[c] = (r < d && c < d) ? Ms[r * W + c] : 0.0;
    lr[c] = 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int col = 0; col < W; ++col) {
    if (col < d) {
      double q = vr[col];  // lane col: V[col][col] - sum_t L[col][t]^2
#pragma unroll
      for (int t = 0; t < col; ++t) q -= lr[t] * lr[t];
      const double qc = __shfl(q, col, 64);
      ok = ok && qc > 0.0;
      const double dg = ok ? sqrt(qc) : 1.0;
      double b = vr[col];  // lane r: V[r][col] - sum_t L[r][t] L[col][t]
#pragma unroll
      for (int t = 0; t < col; ++t) b -= lr[t] * __shfl(lr[t], col, 64);
      if (r == col) lr[col] = dg;
      else if (r > col && r < d) lr[col] = b / dg;
    }
  }
  if (r < d)
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c < d) hchol[r * d + c] = (ok && c <= r) ? h * lr[c] : 0.0;
  if (r == 0 && !ok) atomicOr(flags, SMC_FLAG_NOT_PD);
}

}  // namespace smc
