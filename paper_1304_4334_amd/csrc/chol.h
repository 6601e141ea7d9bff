// Cholesky factor of the particle variance for the M-phase proposal.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace smc {

// Row stride of the LDS factor Ls: one more than W, so that the rows the
// lanes read at the same time fall in different LDS banks.
template <int W>
constexpr int chol_ld() { return W + 1; }

// V = L L' by one wave (call from lanes 0..63 of a wave, d < W).  V is Ms
// (W x W row-major, LDS); L is built in Ls (W rows of stride chol_ld<W>(),
// LDS): lane r writes row r only, and row `col` is read by every lane as a
// broadcast once lane col has written it in earlier columns.  LDS operations
// of one wave complete in order, so the factorisation needs no block
// barrier; the operations and their order are those of a column-by-column
// factorisation.  Writes h L
// (d x d row-major) to hchol (if not NULL); a V that is not positive definite
// gives hchol = 0 and raises SMC_FLAG_NOT_PD in flags (if not NULL).  Returns
// whether V was positive definite (the same in every lane).
template <int W>
__device__ __forceinline__ bool wave_cholesky(const double *Ms, double *Ls, int d, double h,
                                              double *hchol, int32_t *flags) {
  constexpr int LD = chol_ld<W>();
  const int r = threadIdx.x & 63;
  bool ok = true;
  constexpr int kU = 8;  // LDS loads issued together (terms past col add 0 exactly)
  for (int col = 0; col < d; ++col) {
    // the diagonal, computed identically by every lane from row col, and
    // lane r's entry below it
    double q = Ms[col * W + col];
    double b = Ms[(r < d ? r : 0) * W + col];
    for (int t0 = 0; t0 < col; t0 += kU) {
      double lc[kU], lr[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const bool in = t0 + u < col;
        lc[u] = in ? Ls[col * LD + t0 + u] : 0.0;
        lr[u] = (in && r > col && r < d) ? Ls[r * LD + t0 + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        q -= lc[u] * lc[u];
        b -= lr[u] * lc[u];
      }
    }
    ok = ok && q > 0.0;
    const double dg = ok ? sqrt(q) : 1.0;
    if (r > col && r < d) Ls[r * LD + col] = b / dg;
    else if (r == col) Ls[col * LD + col] = dg;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  if (hchol && r < d)
    for (int c = 0; c < d; ++c) hchol[r * d + c] = (ok && c <= r) ? h * Ls[r * LD + c] : 0.0;
  if (flags && r == 0 && !ok) atomicOr(flags, SMC_FLAG_NOT_PD);
  return ok;
}

// The same factorisation for a dimension D fixed at compile time, with the
// loops unrolled: lane r keeps its own row of L in registers, so only the
// broadcast row `col` is read from LDS (Ls is still written in full).  The
// operations and their order are those of wave_cholesky, so both give the
// same bits.
template <int W, int D>
__device__ __forceinline__ bool wave_cholesky_fixed(const double *Ms, double *Ls, double h,
                                                    double *hchol, int32_t *flags) {
  static_assert(D < W, "D must be below the padded width");
  constexpr int LD = chol_ld<W>();
  const int r = threadIdx.x & 63;
  bool ok = true;
  double lrow[D];
#pragma unroll
  for (int c = 0; c < D; ++c) lrow[c] = 0.0;
#pragma unroll
  for (int col = 0; col < D; ++col) {
    double q = Ms[col * W + col];
    double b = Ms[(r < D ? r : 0) * W + col];
    double lc[D];
#pragma unroll
    for (int t = 0; t < col; ++t) lc[t] = Ls[col * LD + t];
#pragma unroll
    for (int t = 0; t < col; ++t) {
      const double lr = (r > col && r < D) ? lrow[t] : 0.0;
      q -= lc[t] * lc[t];
      b -= lr * lc[t];
    }
    ok = ok && q > 0.0;
    const double dg = ok ? sqrt(q) : 1.0;
    if (r > col && r < D) {
      lrow[col] = b / dg;
      Ls[r * LD + col] = lrow[col];
    } else if (r == col) {
      lrow[col] = dg;
      Ls[col * LD + col] = dg;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  if (hchol && r < D) {
#pragma unroll
    for (int c = 0; c < D; ++c) hchol[r * D + c] = (ok && c <= r) ? h * lrow[c] : 0.0;
  }
  if (flags && r == 0 && !ok) atomicOr(flags, SMC_FLAG_NOT_PD);
  return ok;
}

}  // namespace smc
