// Shared host/device definitions of the HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "decision.h"
#include "smc.h"

namespace smc {

constexpr int kDMax = 32;      // parameter dimension bound: d + 1 <= 32 (padded MFMA tiles)
constexpr int kSMax = 5;       // largest recursion state (K <= 4 factors and the shock)
constexpr int kBlock = 256;    // threads per block of the bandwidth-shaped kernels

// Philox purposes (counter word 3, low byte).
enum Purpose : uint64_t { kPrior = 1, kResample = 2, kProposal = 3, kAccept = 4 };

// Everything a kernel needs to know about a model, passed by value.
struct DevModel {
  int32_t kind;
  int32_t K;
  int32_t shock;
  int32_t nreg;
  int32_t prec;
  int32_t d;
  int32_t S;
  int32_t ncomp;  // normal-mixture components I (mixture shocks), else 0
  int32_t block;  // launch shape of the random-walk step: threads per block (0: 64)
  int32_t unroll; // and observations per load batch (0: 8); smc_model_set_launch
  int64_t T;
  const double *y;
  const float *y32;
  const double *X;
};

// Workspace carve-up (offsets in bytes, each 256-aligned).  The speculative
// C-phase columns come last, so their capacity follows from the workspace size.
struct WsLayout {
  size_t small;    // flags, mh, counters, small vectors (kSmallBytes)
  size_t rsscols;  // [kMaxChunk] doubles
  size_t gather;   // [2d + S + 2][P] doubles
  size_t cum;      // [P] doubles (resample running sums)
  size_t mpart;    // [kMomBlocks + 1][W^2] doubles (moment partials and their sum)
  size_t rpart;    // [J][2 * kDMax] doubles (RNE)
  size_t wcols;    // [chunk][P] doubles: speculative C-phase log weights
  size_t fixed;    // bytes before wcols
};

constexpr int64_t kMaxChunk = 4096;
constexpr int64_t kDefaultChunk = 256;
constexpr int kMomBlocks = 128;  // moment partial blocks (moment_partition keeps nb <= 128)

// Offsets inside the `small` region.
constexpr size_t kSmallFlags = 0;    // int32
constexpr size_t kSmallMh = 16;      // int32[2]
constexpr size_t kSmallNacc = 32;    // int64
constexpr size_t kSmallRss = 64;     // double
constexpr size_t kSmallRne = 72;     // double
constexpr size_t kSmallMean = 256;    // double[32]
constexpr size_t kSmallCov = 512;     // double[32 * 32]
constexpr size_t kSmallHchol = 8704;  // double[32 * 32]
constexpr size_t kSmallStop = 16896;  // StopInfo
constexpr size_t kSmallBytes = 17152;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout ws_layout(const DevModel &m, int32_t J, int32_t N);

}  // namespace smc

// Opaque model handle.
struct smc_model {
  smc::DevModel dev;
};
