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

struct CycleDyn;

// Accepted-proposal counts without same-address atomics (a launch's
// per-wave atomic adds on one counter serialise in memory at its end, about
// 10 us for 1,024 waves): each wave of a Metropolis step that holds particles
// stores its count at its own index, and block 0 stores the address of the
// counter the counts belong to in *pending.  A later kernel on the stream
// (acc_flush: the next iteration's moment partials, a device-driven step's
// end, or a launch of its own) adds them to that counter and clears
// *pending.  part == NULL: the step adds to its counter atomically.
struct AccSink {
  int32_t *part;                // [ceil(P / 64)] per-wave counts
  unsigned long long *pending;  // address of the counter they belong to, or 0
};

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
  int32_t block;  // launch shape of the random-walk step: particles per block (0: 64)
  int32_t unroll; // and observations per load batch (0: 8); smc_model_set_launch
  int64_t T;
  const double *y;
  const float *y32;
  const double *X;
  const CycleDyn *cyc;  // device-driven cycle (graph steps), else NULL
  AccSink acc;          // where the Metropolis steps leave their accept counts
};

// State of an adaptive run whose C/S/M cycles are driven on the device
// (smc_run with cfg->graph): one captured step (a C-phase chunk, the S phase,
// up to m_slots M iterations, then k_cycle_end) is replayed until the run
// ends.  The step's kernels read their dates, counters and record slots here
// instead of taking them by value, and return at once when their gate is 0.
struct CycleDyn {
  // fixed for the run
  uint64_t seed, run;  // the Philox key
  int64_t T, P, check_every, force_every, burn_in, cap;
  double D2;
  int32_t Rbar, kR, Lmax, rec_stride, m_slots, J;
  // the chunk of this step
  int64_t t;        // committed date (the chunk starts here)
  int64_t t1;       // end of the chunk
  int64_t t_stop;   // last date of this cycle's C phase
  int64_t t_phase;  // date this cycle's C phase began
  int64_t chunk;    // length bound of this chunk
  int64_t t_new;    // the decided date (the chunk's commit date; the M phase's date)
  int64_t last_len; // length of the previous C phase
  int64_t evals;    // particle x observation evaluations so far
  int64_t steps;    // Metropolis iterations so far
  double rss;       // RSS at the decided date
  int32_t nc;       // checked dates in (t, t1]
  int32_t l;        // cycle index (its Philox counter is l + 1)
  int32_t zero_first;
  // gates: the C-phase kernels (go_c), the scan (go_scan = go_c and nc > 0),
  // the S phase (go_s) and the M slots (go_m); slot k runs iteration r0 + k
  // while r0 + k <= R
  int32_t go_c, go_scan, go_s, go_m;
  int32_t r0, R;
  int32_t done;     // 1: the run reached T
  int32_t err;      // 1: the record is full, 2: a numerical flag was raised
  int32_t flags;    // the flags word when err = 2
  uint32_t progress;  // steps that did work
};

__device__ __forceinline__ bool m_slot_off(const CycleDyn *c, int32_t k) {
  return c && (!c->go_m || c->r0 + k > c->R);
}

// The end of a Metropolis step's wave (wave: its index in the launch): its
// accept count goes to acc, or without a sink atomically to *n_accept.
__device__ __forceinline__ void acc_store(const AccSink &acc, unsigned long long mask,
                                          int64_t wave, int64_t P,
                                          unsigned long long *n_accept) {
  if (acc.part) {
    if ((threadIdx.x & 63) == 0 && wave * 64 < P) acc.part[wave] = (int32_t)__popcll(mask);
    if (blockIdx.x == 0 && threadIdx.x == 0)
      *acc.pending = reinterpret_cast<unsigned long long>(n_accept);
  } else if ((threadIdx.x & 63) == 0 && mask) {
    atomicAdd(n_accept, (unsigned long long)__popcll(mask));
  }
}

// Adds the pending per-wave counts of a P-particle step to their counter and
// clears the mark (nothing pending: nothing to do).  Called by a whole wave;
// the counts are loaded together with the mark, and the total goes to the
// counter by one atomic add, so the chain is a single round trip.
__device__ __forceinline__ void acc_flush(const AccSink &acc, int64_t P) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (P + 63) / 64;
  constexpr int kB = 16;  // loads per lane in flight together (1,024 waves in one round)
  long long s = 0;
  unsigned long long dst = 0;
  for (int64_t base = 0; base < nw; base += 64 * kB) {
    int32_t x[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int64_t i = base + u * 64 + lane;
      x[u] = i < nw ? acc.part[i] : 0;
    }
    if (base == 0) dst = *acc.pending;
#pragma unroll
    for (int u = 0; u < kB; ++u) s += x[u];
  }
  if (!dst) return;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    atomicAdd(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)s);
    *acc.pending = 0;
  }
}

// Cycles a graph-replayed run records on the device.
constexpr int32_t kGraphMaxCycles = 4096;

// Workspace carve-up (offsets in bytes, each 256-aligned).  The C-phase scan's
// per-date sums come last, so the chunk capacity follows from the workspace size.
struct WsLayout {
  size_t small;    // flags, mh, counters, small vectors (kSmallBytes)
  size_t rsscols;  // [kMaxChunk] doubles, then the RSS slices' partial sums
  size_t gather;   // [2d + S + 2][P] doubles
  size_t cum;      // [P] doubles (resample running sums)
  size_t mpart;    // [kMomBlocks + 1][W^2] doubles (moment partials and their sum)
  size_t rpart;    // [J][2 * kDMax] doubles (RNE)
  size_t cyc;      // CycleDyn, then t_end [kGraphMaxCycles] int64, R [..] int32, rss [..]
  size_t acc;      // AccSink: the pending counter's address, then at +256 the
                   // per-wave accept counts [ceil(P/64)] int32
  size_t wcols;    // tail of [chunk][P] doubles: the C-phase scan's per-wave RSS sums
                   // ([chunk][ceil(P/64)][3]) or the adjoint's checkpoints
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
