// Kernels templated on the model type, and the table of their launchers.
//
// Each ops_*.hip translation unit instantiates the table (ModelOps) for a set
// of models, so the model families compile in parallel; kernels.hip routes a
// model description to its table.  Geometry: one particle per lane, 64-thread
// blocks (one wave each), so a population spreads over as many compute units
// as it has waves; observations are wave-uniform (every lane of a wave loads
// the same ones, eight at a time).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "adjoint.h"
#include "chol.h"
#include "common.h"
#include "launch.h"
#include "model.h"
#include "reduce.h"
#include "rng.h"

namespace smc {

namespace {

inline dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

inline smc_status launch_status(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SMC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return SMC_OK;
}

template <typename T>
__device__ __forceinline__ T *typed(void *p) { return reinterpret_cast<T *>(p); }
template <typename T>
__device__ __forceinline__ const T *typed(const void *p) { return reinterpret_cast<const T *>(p); }

}  // namespace

// --------------------------------------------------------- prior (a1) ------
template <class M>
__global__ void __launch_bounds__(64) k_init(DevModel dm, int64_t P, uint64_t seed, uint64_t run,
                                             double *theta, double *logprior, double *loglik,
                                             void *state, double *logw) {
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  double th[M::D];
  M::prior_draw(seed, run, (uint64_t)p, th);
#pragma unroll
  for (int i = 0; i < M::D; ++i) theta[i * P + p] = th[i];
  logprior[p] = M::logprior(th);
  loglik[p] = 0.0;
  logw[p] = 0.0;
  using R = typename M::R;
#pragma unroll
  for (int k = 0; k < StoredS<M>::value; ++k) typed<R>(state)[k * P + p] = (R)0;
}

// ------------------------------------------------------------ C phase (a2) --
// Speculative pass: from the committed state at t0, evaluate observations
// t0+1..t1 and, at every check date, the RSS sums of the running log weights
// over the block's wave of 64 particles, without committing anything.  The
// weights of up to 32 recorded dates wait in a ring in LDS; after every 16
// observations (and at the end) each group of 16 dates is reduced: four
// lanes per date take the maximum m of 16 weights each, then
// s1 = sum exp(w - m) and s2 = sum exp(2 (w - m)), combined over the four
// lanes (quad exchanges), and the wave's triple (m, s1, s2) for date c goes
// to trip[(c * nwaves + wave) * 3] (k_rss_scan merges the waves).  Lanes
// beyond P follow the recursion of particle P - 1 and record weight -inf.
// Dates are counted relative to t0 in 32 bits (a chunk holds at most
// kMaxChunk dates).  kEvery1: every date is checked (check_every = 1).
constexpr int kScanRing = 32;  // recorded dates held in LDS (a power of two)

template <class M, bool kEvery1>
__global__ void __launch_bounds__(64) k_cscan(DevModel dm, int64_t P, const double *theta,
                                              const void *state, const double *logw, int64_t t0,
                                              int64_t t1, int64_t check_every, int64_t t_max,
                                              int32_t zero_first, double *trip,
                                              const typename M::Y *__restrict__ ydata) {
  __shared__ double ring[kScanRing * 64];
  const int lane = threadIdx.x;
  const int64_t p0 = blockIdx.x * 64ll + lane;
  const bool live = p0 < P;
  const int64_t p = live ? p0 : P - 1;
  if (const CycleDyn *c = dm.cyc) {  // a device-driven chunk
    if (!c->go_scan) return;
    t0 = c->t;
    t1 = c->t1;
    t_max = c->t_stop;
    zero_first = c->zero_first;
  }
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  double th[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) th[i] = theta[i * P + p];
  const auto par = M::params(th);
  R st[SR];
#pragma unroll
  for (int k = 0; k < SR; ++k) st[k] = (k < StoredS<M>::value) ? typed<R>(state)[k * P + p] : (R)0;
  double lw = !live ? -INFINITY : (zero_first ? 0.0 : logw[p]);
  const int64_t nw = gridDim.x;
  int32_t nrec = 0, ndone = 0;  // dates recorded, dates reduced
  auto record = [&]() {
    ring[(nrec & (kScanRing - 1)) * 64 + lane] = lw;
    ++nrec;
  };
  // dates ndone .. ndone + n - 1 (n <= 16, all lanes)
  auto reduce = [&](int32_t n) {
    __syncthreads();  // the block is this wave: orders the ring's writes and reads
    const int c = lane >> 2, q = lane & 3;
    const bool mine = c < n;
    double v[16];
    double m = -INFINITY;
    if (mine) {
      const double *src = ring + ((ndone + c) & (kScanRing - 1)) * 64 + q * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = src[j];
#pragma unroll
      for (int j = 0; j < 16; ++j) m = fmax(m, v[j]);
    }
    m = fmax(m, dpp_f64<0xB1>(m));
    m = fmax(m, dpp_f64<0x4E>(m));
    double s1 = 0.0, s2 = 0.0;
    if (mine && m > -INFINITY) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        // FP32 recursions: the hardware base-2 exponential (its 1e-7 relative
        // error is far below that of weights summed from FP32 log densities;
        // terms below 2^-126 of the maximum are dropped); FP64: exp_nonpos
        double e;
        if constexpr (std::is_same_v<R, float>)
          e = (double)__builtin_amdgcn_exp2f((float)((v[j] - m) * kLog2e));
        else
          e = exp_nonpos(v[j] - m);
        s1 += e;
        s2 = fma(e, e, s2);
      }
    }
    s1 += dpp_f64<0xB1>(s1);
    s2 += dpp_f64<0xB1>(s2);
    s1 += dpp_f64<0x4E>(s1);
    s2 += dpp_f64<0x4E>(s2);
    if (mine && q == 0) {
      double *o = trip + ((int64_t)(ndone + c) * nw + blockIdx.x) * 3;
      o[0] = m;
      o[1] = s1;
      o[2] = s2;
    }
    ndone += n;
  };
  auto group = [&]() {
    if (nrec - ndone >= 16) reduce(16);
  };
  if constexpr (kEvery1) {
    Eval<M>::scan_y(
        dm, ydata, par, st, t0, t1,
        [&](int64_t, double lp) {
          if (isnan(lp)) lp = -INFINITY;
          lw += lp;
          record();
        },
        group);
  } else {
    // dates relative to t0: the next multiple of check_every, and t_max
    // (both capped beyond the chunk, where they are never reached)
    const int64_t span = t1 - t0 + 1;
    const int64_t first = (t0 / check_every + 1) * check_every - t0;
    int32_t next_rel = (int32_t)(first < span ? first : span);
    const int32_t max_rel = (int32_t)(t_max - t0 < span ? t_max - t0 : span);
    const int32_t every = (int32_t)(check_every < span ? check_every : span);
    int32_t rel = 0;
    Eval<M>::scan_y(
        dm, ydata, par, st, t0, t1,
        [&](int64_t, double lp) {
          if (isnan(lp)) lp = -INFINITY;
          lw += lp;
          ++rel;
          const bool at_check = rel == next_rel;
          if (at_check || rel == max_rel) record();
          if (at_check) next_rel += every;
        },
        group);
  }
  // at most 16 dates between two calls of group(), so the ring never holds
  // more than 31 unreduced ones
  while (nrec > ndone) reduce(min(16, nrec - ndone));
}

// Commit: advance from t0 to t1 (or to *t1_dev when given), adding the log
// densities to logw and loglik.  A device-driven chunk takes t0, t1 and
// zero_first from dm.cyc.
template <class M>
__global__ void __launch_bounds__(64) k_ccommit(DevModel dm, int64_t P, const double *theta,
                                                void *state, double *logw, double *loglik,
                                                int64_t t0, int64_t t1, int32_t zero_first,
                                                const int64_t *t1_dev,
                                                const typename M::Y *__restrict__ ydata) {
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  if (const CycleDyn *c = dm.cyc) {
    if (!c->go_c) return;
    t0 = c->t;
    t1 = c->t1;
    zero_first = c->zero_first;
  }
  if (t1_dev) t1 = min(t1, *t1_dev);
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  constexpr int SS = StoredS<M>::value;
  double th[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) th[i] = theta[i * P + p];
  const auto par = M::params(th);
  R st[SR];
#pragma unroll
  for (int k = 0; k < SR; ++k) st[k] = (k < SS) ? typed<R>(state)[k * P + p] : (R)0;
  double lp = Eval<M>::advance_y(dm, ydata, par, st, t0, t1);
  if (isnan(lp)) lp = -INFINITY;
  logw[p] = (zero_first ? 0.0 : logw[p]) + lp;
  loglik[p] += lp;
#pragma unroll
  for (int k = 0; k < SS; ++k) typed<R>(state)[k * P + p] = st[k];
}

// ------------------------------------------------------------ M phase (a5) --
// The proposal scale of a random-walk step computed by one wave of the
// step's own block, its scaling wave or its first particle wave (MomFuse):
// the moment partials summed entry by entry in block order, the step-size
// rule, V and its Cholesky factor in LDS, exactly as the separate moments
// kernels do (k_mom_final).  Returns whether V was positive definite; h
// receives the step size.  The wave orders its LDS accesses by wavefront
// fences (LDS operations of one wave complete in order); the block
// synchronises afterwards.
// The first partial matrix's entries (lane entries idx = lane + 64 q), the
// step size and the previous accept count, all loaded together.
template <int D>
struct ScalePre {
  static constexpr int E = (D + 1) * (D + 1);  // entries used: rows and columns 0..D
  static constexpr int Q = (E + 63) / 64;
  double x0[Q];
  int32_t m;
  int64_t nacc;
};

template <int D, int W>
__device__ __forceinline__ void fused_scale_issue(const MomFuse &fm, ScalePre<D> &pre) {
  const int lane = threadIdx.x & 63;
  pre.m = 0;
  pre.nacc = 0;
  if (lane == 0) {
    pre.m = *fm.mh_in;
    if (fm.mh_reset <= 0 && fm.prev_nacc) pre.nacc = *fm.prev_nacc;
  }
#pragma unroll
  for (int q = 0; q < ScalePre<D>::Q; ++q) {
    const int idx = lane + 64 * q;
    const int e = (idx / (D + 1)) * W + idx % (D + 1);
    pre.x0[q] = (idx < ScalePre<D>::E && fm.nb > 0) ? fm.part[e] : 0.0;
  }
}

template <int D, int W>
__device__ __forceinline__ bool fused_scale(const MomFuse &fm, int64_t P, double *Ms, double *Ls,
                                            double *sh_h, double &h, const ScalePre<D> &pre) {
  const auto sync = [] { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); };
  constexpr int E = ScalePre<D>::E;
  const int lane = threadIdx.x & 63;
  int32_t m = pre.m;
  const int64_t nacc = pre.nacc;
  // Lane entries idx = lane + 64 q, added in block order; the first partial
  // came with pre, the rest (none when the partials come pre-summed into one
  // matrix) in batches whose loads are all issued before any is added.
  constexpr int Q = ScalePre<D>::Q;
  constexpr int kB = Q >= 32 ? 1 : 32 / Q;  // partials per entry in flight
  double sum[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) sum[q] = 0.0 + pre.x0[q];
  for (int b0 = 1; b0 < fm.nb; b0 += kB) {
    double x[Q][kB];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int idx = lane + 64 * q;
      const int e = (idx / (D + 1)) * W + idx % (D + 1);
#pragma unroll
      for (int u = 0; u < kB; ++u)
        x[q][u] = (idx < E && b0 + u < fm.nb) ? fm.part[(int64_t)(b0 + u) * W * W + e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int u = 0; u < kB; ++u)
        if (b0 + u < fm.nb) sum[q] += x[q][u];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = lane + 64 * q;
    if (idx < E) Ms[(idx / (D + 1)) * W + idx % (D + 1)] = sum[q];
  }
  if (lane == 0) {
    if (fm.mh_reset > 0) {
      m = fm.mh_reset;
    } else if (fm.prev_nacc) {
      m += (nacc * 1000 > (int64_t)fm.target_permille * P) ? 1 : -1;
      m = m < 1 ? 1 : (m > 10 ? 10 : m);
    }
    if (blockIdx.x == 0) *fm.mh_out = m;
    *sh_h = (double)m / 10.0;
  }
  sync();
  // V in place: entry (r, c) with r, c < D reads only itself and column D,
  // which is not written here
  const double invP = 1.0 / (double)P;
#pragma unroll
  for (int q = 0; q < (D * D + 63) / 64; ++q) {
    const int idx = lane + 64 * q;
    if (idx < D * D) {
      const int r = idx / D, c = idx % D;
      Ms[r * W + c] = (Ms[r * W + c] - Ms[r * W + D] * Ms[c * W + D] * invP) / (double)(P - 1);
    }
  }
  sync();
  h = *sh_h;
  return wave_cholesky_fixed<W, D>(Ms, Ls, h, blockIdx.x == 0 ? fm.hchol_out : nullptr,
                                   blockIdx.x == 0 ? fm.flags : nullptr);
}

// B particles (B/64 waves) per block, observations loaded U at a time; the
// launch shape does not change any result.  With the proposal scale folded
// in (fm.part) and B = 256, the launch has one wave more per block, threads
// B..B+63: it loads the summed moments and factors V while the particle
// waves load their particles and draw their proposals, and hands h L over in
// LDS.  Smaller blocks, several to a compute unit, would then stack two
// particle waves on some SIMDs while others hold only scaling waves, so
// there the first particle wave does that work after its own draws.  In
// a device-driven cycle (dm.cyc) the launch is M slot `iter` of its step: it
// runs iteration r = r0 + iter of the cycle while r <= R, at the cycle's date
// and key, with the record slots, step-size slots and rule of that iteration.
template <int B>
constexpr bool scale_wave() { return B >= 256; }

template <class M, int B = 64, int U = kUnroll>
__global__ void __launch_bounds__(scale_wave<B>() ? B + 64 : B) k_mutate_rw(DevModel dm, int64_t P,
                                                                            int64_t t,
                                                      double *theta,
                                                 double *logprior, double *loglik, void *state,
                                                 const double *__restrict__ hchol, uint64_t seed,
                                                 uint64_t run, uint64_t cycle, uint64_t iter,
                                                 unsigned long long *n_accept, uint8_t *accepted,
                                                 MomFuse fm,
                                                 const typename M::Y *__restrict__ ydata) {
  constexpr int D = M::D;
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  constexpr int SS = StoredS<M>::value;
  constexpr int W = D < 16 ? 16 : 32;  // padded width of the moment matrices
  constexpr bool kCanFuse = D < 32;
  __shared__ double Ms[kCanFuse ? W * W : 1], Ls[kCanFuse ? W * chol_ld<W>() : 1], sh_h;
  __shared__ int sh_ok;
  if (const CycleDyn *c = dm.cyc) {
    if (m_slot_off(c, (int32_t)iter)) return;
    const int32_t r = c->r0 + (int32_t)iter;
    iter = (uint64_t)r;
    t = c->t_new;
    seed = c->seed;
    run = c->run;
    cycle = (uint64_t)(c->l + 1);
    const int64_t slot = (int64_t)c->l * c->rec_stride + (r - 1);
    n_accept += slot;
    fm.hchol_out += slot * D * D;
    fm.prev_nacc = r == 1 ? nullptr : reinterpret_cast<const int64_t *>(n_accept) - 1;
    fm.mh_reset = r == 1 ? 5 : 0;
    int32_t *mh = fm.mh_out;  // the two step-size slots, alternating with r
    fm.mh_in = (r & 1) ? mh + 1 : mh;
    fm.mh_out = (r & 1) ? mh : mh + 1;
  }
  constexpr bool kScaleWave = scale_wave<B>();
  if constexpr (kCanFuse && kScaleWave) {
    if (threadIdx.x >= B) {  // the scaling wave (launched with fm.part only)
      ScalePre<D> pre;
      fused_scale_issue<D, W>(fm, pre);
      double hs = 0.0;
      const bool ok = fused_scale<D, W>(fm, P, Ms, Ls, &sh_h, hs, pre);
      if (threadIdx.x == B) sh_ok = ok;
      __syncthreads();
      return;
    }
  }
  const int64_t p = blockIdx.x * (int64_t)B + threadIdx.x;
  const int64_t pc = p < P ? p : P - 1;
  // without a scaling wave, the first particle wave's scale loads go first,
  // so that their latency overlaps its draws
  ScalePre<D> pre;
  if constexpr (kCanFuse && !kScaleWave)
    if (fm.part && threadIdx.x < 64) fused_scale_issue<D, W>(fm, pre);
  double th[D], z[D];
#pragma unroll
  for (int i = 0; i < D; ++i) th[i] = theta[i * P + pc];
  normals<D>(seed, run, (uint64_t)pc, cycle, iter, kProposal, z, D);
  bool fused = false, chol_ok = true;
  double h = 0.0;
  if constexpr (kCanFuse) {
    if (fm.part) {
      fused = true;
      if constexpr (!kScaleWave) {
        if (threadIdx.x < 64) {
          double hs = 0.0;
          const bool ok = fused_scale<D, W>(fm, P, Ms, Ls, &sh_h, hs, pre);
          if (threadIdx.x == 0) sh_ok = ok;
        }
      }
      __syncthreads();  // h L from the scaling wave (or the first particle wave)
      chol_ok = sh_ok != 0;
      h = sh_h;
    }
  }
  int acc = 0;
  if (p < P) {
    double pr[D];
    if (fused) {
      // h L rounded as the moments kernels round it: h * L_ik (0 without a factor)
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k)
          s = fma(chol_ok ? h * Ls[kCanFuse ? i * chol_ld<W>() + k : 0] : 0.0, z[k], s);
        pr[i] = th[i] + s;
      }
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k) s = fma(hchol[i * D + k], z[k], s);
        pr[i] = th[i] + s;
      }
    }
    const double lp1 = M::logprior(pr);
    R st[SR];
#pragma unroll
    for (int k = 0; k < SR; ++k) st[k] = (R)0;
    double ll1 = -INFINITY;
    if (lp1 > -INFINITY) {
      const auto par = M::params(pr);
      ll1 = Eval<M>::template advance_y<U>(dm, ydata, par, st, 0, t);
      const double delta = (lp1 + ll1) - (logprior[p] + loglik[p]);
      const U64x4 w = draw4(seed, run, (uint64_t)p, cycle, iter, kAccept);
      acc = (log(u01_oo(w.x0)) < delta) ? 1 : 0;
    }
    if (acc) {
#pragma unroll
      for (int i = 0; i < D; ++i) theta[i * P + p] = pr[i];
      logprior[p] = lp1;
      loglik[p] = ll1;
#pragma unroll
      for (int k = 0; k < SS; ++k) typed<R>(state)[k * P + p] = st[k];
    }
    if (accepted) accepted[p] = (uint8_t)acc;
  }
  acc_store(dm.acc, __ballot(acc), (blockIdx.x * (int64_t)B + threadIdx.x) >> 6, P, n_accept);
}

// Launch of the random-walk step in shape (B, U).
template <class M, int B, int U>
smc_status launch_rw_shape(const DevModel &m, int64_t P, int64_t t, double *theta,
                           double *logprior, double *loglik, void *state, const double *hchol,
                           uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter,
                           int64_t *n_accept, uint8_t *accepted, const KernelTimer *timer,
                           const MomFuse *fuse, hipStream_t s) {
  auto *acc = reinterpret_cast<unsigned long long *>(n_accept);
  MomFuse fm{};
  if (fuse) {
    if (M::D >= 32) return set_error(SMC_E_UNSUPPORTED, "folded proposal scale needs d < 32");
    fm = *fuse;
  }
  const typename M::Y *yd = Eval<M>::host_y(m);
  const dim3 threads(fm.part && scale_wave<B>() ? B + 64 : B);  // a folded scale's scaling wave
  if (timer)
    hipExtLaunchKernelGGL((k_mutate_rw<M, B, U>), grid_for(P, B), threads, 0, s, timer->start,
                          timer->stop, 0, m, P, t, theta, logprior, loglik, state, hchol, seed,
                          run, cycle, iter, acc, accepted, fm, yd);
  else
    hipLaunchKernelGGL((k_mutate_rw<M, B, U>), grid_for(P, B), threads, 0, s, m, P, t, theta,
                       logprior, loglik, state, hchol, seed, run, cycle, iter, acc, accepted, fm,
                       yd);
  return launch_status("mutate");
}

// Every tuned launch shape (threads per block 64, 128 or 256; observations
// per load batch 4, 8 or 16) of a model's random-walk step.
template <class M>
smc_status launch_rw_any_shape(int32_t B, int32_t U, const DevModel &m, int64_t P, int64_t t,
                               double *theta, double *logprior, double *loglik, void *state,
                               const double *hchol, uint64_t seed, uint64_t run, uint64_t cycle,
                               uint64_t iter, int64_t *n_accept, uint8_t *accepted,
                               const KernelTimer *timer, const MomFuse *fuse, hipStream_t s) {
#define SMC_RW_SHAPE(b, u)                                                                   \
  if (B == b && U == u)                                                                     \
    return launch_rw_shape<M, b, u>(m, P, t, theta, logprior, loglik, state, hchol, seed, run, \
                                    cycle, iter, n_accept, accepted, timer, fuse, s);
  SMC_RW_SHAPE(64, 4) SMC_RW_SHAPE(64, 8) SMC_RW_SHAPE(64, 16)
  SMC_RW_SHAPE(128, 4) SMC_RW_SHAPE(128, 8) SMC_RW_SHAPE(128, 16)
  SMC_RW_SHAPE(256, 4) SMC_RW_SHAPE(256, 8) SMC_RW_SHAPE(256, 16)
#undef SMC_RW_SHAPE
  return set_error(SMC_E_UNSUPPORTED, "launch shape %d x %d", B, U);
}

// The independent Gaussian Metropolis sampler (Section 3.3's alternative):
// theta' = mean + L z whatever the current particle, accepted with the
// proposal-density ratio q(theta) / q(theta') = exp(|z|^2/2 - |w|^2/2),
// L w = theta - mean.
template <class M>
__global__ void __launch_bounds__(64) k_mutate_indep(DevModel dm, int64_t P, int64_t t,
                                                     double *theta, double *logprior,
                                                     double *loglik, void *state,
                                                     const double *__restrict__ chol,
                                                     const double *__restrict__ mean,
                                                     uint64_t seed, uint64_t run, uint64_t cycle,
                                                     uint64_t iter, unsigned long long *n_accept,
                                                     uint8_t *accepted,
                                                     const typename M::Y *__restrict__ ydata) {
  constexpr int D = M::D;
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  constexpr int SS = StoredS<M>::value;
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  int acc = 0;
  if (p < P) {
    double th[D], z[D], pr[D];
#pragma unroll
    for (int i = 0; i < D; ++i) th[i] = theta[i * P + p];
    normals<D>(seed, run, (uint64_t)p, cycle, iter, kProposal, z, D);
    double ww = 0.0, zz = 0.0, w[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0.0, a = th[i] - mean[i];
#pragma unroll
      for (int k = 0; k < i; ++k) {
        s = fma(chol[i * D + k], z[k], s);
        a = fma(-chol[i * D + k], w[k], a);
      }
      s = fma(chol[i * D + i], z[i], s);
      pr[i] = mean[i] + s;
      w[i] = a / chol[i * D + i];
      ww = fma(w[i], w[i], ww);
      zz = fma(z[i], z[i], zz);
    }
    const double lp1 = M::logprior(pr);
    R st[SR];
#pragma unroll
    for (int k = 0; k < SR; ++k) st[k] = (R)0;
    double ll1 = -INFINITY;
    if (lp1 > -INFINITY) {
      const auto par = M::params(pr);
      ll1 = Eval<M>::advance_y(dm, ydata, par, st, 0, t);
      const double delta =
          (lp1 + ll1) - (logprior[p] + loglik[p]) + (-0.5 * ww + 0.5 * zz);
      const U64x4 u = draw4(seed, run, (uint64_t)p, cycle, iter, kAccept);
      acc = (log(u01_oo(u.x0)) < delta) ? 1 : 0;
    }
    if (acc) {
#pragma unroll
      for (int i = 0; i < D; ++i) theta[i * P + p] = pr[i];
      logprior[p] = lp1;
      loglik[p] = ll1;
#pragma unroll
      for (int k = 0; k < SS; ++k) typed<R>(state)[k * P + p] = st[k];
    }
    if (accepted) accepted[p] = (uint8_t)acc;
  }
  acc_store(dm.acc, __ballot(acc), blockIdx.x, P, n_accept);
}

// ------------------------------------------------- standalone likelihood --
template <class M>
__global__ void __launch_bounds__(64) k_loglik(DevModel dm, int64_t P, const double *theta,
                                               int64_t t, double *out, void *state_out) {
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  double th[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) th[i] = theta[i * P + p];
  const auto par = M::params(th);
  R st[SR];
#pragma unroll
  for (int k = 0; k < SR; ++k) st[k] = (R)0;
  out[p] = Eval<M>::advance(dm, par, st, 0, t);
  if (state_out)
#pragma unroll
    for (int k = 0; k < StoredS<M>::value; ++k) typed<R>(state_out)[k * P + p] = st[k];
}

// ------------------------------------- gradients and the Langevin step (a8) --
template <class M>
struct IsLinreg : std::false_type {};
template <int NREG>
struct IsLinreg<Linreg<NREG>> : std::true_type {};

// Value of log p(y_{1:t} | theta) with its gradient added (times scale) to
// g, and the state at t.  ckpt: this call's checkpoint area; lds: this lane's
// column of the block's LDS buffer.
template <class M>
__device__ __forceinline__ double ll_and_grad(const DevModel &dm, const double *th, int64_t t,
                                              void *ckpt, int64_t P, int64_t p, void *lds,
                                              double scale, double *g,
                                              typename M::R (&st)[Eval<M>::SR]) {
  if constexpr (IsLinreg<M>::value) {
    st[0] = 0.0;
    return Adjoint<M>::value_and_grad(dm, th, t, scale, g);
  } else {
    using R = typename M::R;
    const auto par = M::params(th);
    return Adjoint<M>::value_and_grad(par, th, t, M::ydata(dm), typed<R>(ckpt), P, p,
                                      typed<R>(lds) + threadIdx.x, scale, g, st);
  }
}

template <class M>
constexpr size_t lds_bytes_of() {
  if constexpr (IsLinreg<M>::value) return 0;
  else return (size_t)Adjoint<M>::kLdsPerLane * 64 * sizeof(typename M::R);
}

template <class M>
__global__ void __launch_bounds__(64) k_loglik_backward(DevModel dm, int64_t P, const double *theta,
                                                        int64_t t, const double *dloglik,
                                                        double *dtheta, void *ckpt) {
  extern __shared__ double lds_dyn[];
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  double th[M::D], g[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) {
    th[i] = theta[i * P + p];
    g[i] = 0.0;
  }
  typename M::R st[Eval<M>::SR];
  (void)ll_and_grad<M>(dm, th, t, ckpt, P, p, lds_dyn, dloglik[p], g, st);
#pragma unroll
  for (int i = 0; i < M::D; ++i) dtheta[i * P + p] = g[i];
}

// grad = d/dtheta [log p(theta) + log p(y_{1:t} | theta)] for every particle.
template <class M>
__global__ void __launch_bounds__(64) k_grad_post(DevModel dm, int64_t P, const double *theta,
                                                  int64_t t, double *grad, void *ckpt) {
  extern __shared__ double lds_dyn[];
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  double th[M::D], g[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) th[i] = theta[i * P + p];
  PriorGradOf<M>::run(th, g);
  typename M::R st[Eval<M>::SR];
  (void)ll_and_grad<M>(dm, th, t, ckpt, P, p, lds_dyn, 1.0, g, st);
#pragma unroll
  for (int i = 0; i < M::D; ++i) grad[i * P + p] = g[i];
}

// One preconditioned Langevin (MALA) Metropolis iteration of particle p:
// proposal mean theta + (1/2)(hL)(hL)' grad, noise hL z; the acceptance test
// adds log q(theta | theta') - log q(theta' | theta) = -|w|^2/2 + |z|^2/2
// with (hL) w = theta - theta' - (1/2)(hL)(hL)' grad'.  ckpt: the adjoint's
// checkpoint area of the population; lds: the block's LDS buffer.  Returns
// whether the proposal was accepted (the particle's arrays are updated).
template <class M>
__device__ __forceinline__ int mala_one(const DevModel &dm, int64_t P, int64_t p, int64_t t,
                                        double *theta, double *logprior, double *loglik,
                                        void *state, double *grad,
                                        const double *__restrict__ hchol, uint64_t seed,
                                        uint64_t run, uint64_t cycle, uint64_t iter, void *ckpt,
                                        void *lds) {
  constexpr int D = M::D;
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  constexpr int SS = StoredS<M>::value;
  int acc = 0;
  double th[D], z[D], pr[D], g0[D], g1[D], u[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    th[i] = theta[i * P + p];
    g0[i] = grad[i * P + p];
  }
  normals<D>(seed, run, (uint64_t)p, cycle, iter, kProposal, z, D);
  // u = (hL)' g0
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = k; i < D; ++i) s = fma(hchol[i * D + k], g0[i], s);
    u[k] = s;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double dr = 0.0, st = 0.0;
#pragma unroll
    for (int k = 0; k <= i; ++k) {
      dr = fma(hchol[i * D + k], u[k], dr);
      st = fma(hchol[i * D + k], z[k], st);
    }
    pr[i] = th[i] + 0.5 * dr + st;
  }
  const double lp1 = M::logprior(pr);
  R stv[SR];
#pragma unroll
  for (int k = 0; k < SR; ++k) stv[k] = (R)0;
  double ll1 = -INFINITY;
  if (lp1 > -INFINITY) {
    PriorGradOf<M>::run(pr, g1);
    ll1 = ll_and_grad<M>(dm, pr, t, ckpt, P, p, lds, 1.0, g1, stv);
    // reverse move
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = k; i < D; ++i) s = fma(hchol[i * D + k], g1[i], s);
      u[k] = s;
    }
    double ww = 0.0, zz = 0.0, w[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double dr = 0.0;
#pragma unroll
      for (int k = 0; k <= i; ++k) dr = fma(hchol[i * D + k], u[k], dr);
      double a = th[i] - pr[i] - 0.5 * dr;
#pragma unroll
      for (int k = 0; k < i; ++k) a = fma(-hchol[i * D + k], w[k], a);
      w[i] = a / hchol[i * D + i];
      ww = fma(w[i], w[i], ww);
      zz = fma(z[i], z[i], zz);
    }
    const double delta = (lp1 + ll1) - (logprior[p] + loglik[p]) + (-0.5 * ww + 0.5 * zz);
    const U64x4 wr = draw4(seed, run, (uint64_t)p, cycle, iter, kAccept);
    acc = (log(u01_oo(wr.x0)) < delta) ? 1 : 0;
  }
  if (acc) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      theta[i * P + p] = pr[i];
      grad[i * P + p] = g1[i];
    }
    logprior[p] = lp1;
    loglik[p] = ll1;
#pragma unroll
    for (int k = 0; k < SS; ++k) typed<R>(state)[k * P + p] = stv[k];
  }
  return acc;
}

template <class M>
__global__ void __launch_bounds__(64) k_mutate_mala(DevModel dm, int64_t P, int64_t t, double *theta,
                                                    double *logprior, double *loglik, void *state,
                                                    double *grad, const double *__restrict__ hchol,
                                                    uint64_t seed, uint64_t run, uint64_t cycle,
                                                    uint64_t iter, unsigned long long *n_accept,
                                                    uint8_t *accepted, void *ckpt) {
  extern __shared__ double lds_dyn[];
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  int acc = 0;
  if (p < P) {
    acc = mala_one<M>(dm, P, p, t, theta, logprior, loglik, state, grad, hchol, seed, run, cycle,
                      iter, ckpt, lds_dyn);
    if (accepted) accepted[p] = (uint8_t)acc;
  }
  acc_store(dm.acc, __ballot(acc), blockIdx.x, P, n_accept);
}

// ---------------------------------------------- functions of interest (f) --
// out[i][p]: the parameters (which = 0) or the model's functions of interest
// (which = 1) of every particle at date t.
template <class M>
__global__ void __launch_bounds__(64) k_test_fns(DevModel dm, int64_t P, const double *theta,
                                                 const void *state, int64_t t, int32_t which,
                                                 double *out) {
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
  double th[M::D];
#pragma unroll
  for (int i = 0; i < M::D; ++i) th[i] = theta[i * P + p];
  if (which == 0) {
#pragma unroll
    for (int i = 0; i < M::D; ++i) out[i * P + p] = th[i];
    return;
  }
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  R st[SR];
#pragma unroll
  for (int k = 0; k < SR; ++k) st[k] = (k < StoredS<M>::value) ? typed<R>(state)[k * P + p] : (R)0;
  double g[M::kTests];
  M::test_fns(th, st, t, g);
#pragma unroll
  for (int q = 0; q < M::kTests; ++q) out[q * P + p] = g[q];
}

// Every model has a hand-written adjoint.
template <class M>
struct HasAdjoint : std::true_type {};

// ============================================================ launchers ====
template <class M>
struct OpsOf {
  static smc_status init(const DevModel &m, int64_t P, uint64_t seed, uint64_t run, double *theta,
                         double *logprior, double *loglik, void *state, double *logw,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_init<M>, grid_for(P, 64), dim3(64), 0, s, m, P, seed, run, theta,
                       logprior, loglik, state, logw);
    return launch_status("init_from_prior");
  }

  static smc_status cscan(const DevModel &m, int64_t P, const double *theta, const void *state,
                          const double *logw, int64_t t0, int64_t t1, int64_t check_every,
                          int64_t t_max, bool zero_first, double *W, hipStream_t s) {
    const typename M::Y *yd = Eval<M>::host_y(m);
    if (check_every == 1)
      hipLaunchKernelGGL((k_cscan<M, true>), grid_for(P, 64), dim3(64), 0, s, m, P, theta, state,
                         logw, t0, t1, check_every, t_max, (int32_t)zero_first, W, yd);
    else
      hipLaunchKernelGGL((k_cscan<M, false>), grid_for(P, 64), dim3(64), 0, s, m, P, theta, state,
                         logw, t0, t1, check_every, t_max, (int32_t)zero_first, W, yd);
    return launch_status("correct/scan");
  }

  static smc_status ccommit(const DevModel &m, int64_t P, const double *theta, void *state,
                            double *logw, double *loglik, int64_t t0, int64_t t1,
                            bool zero_first, const int64_t *t1_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_ccommit<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, state, logw,
                       loglik, t0, t1, (int32_t)zero_first, t1_dev, Eval<M>::host_y(m));
    return launch_status("correct/commit");
  }

  static smc_status mutate_rw(const DevModel &m, int64_t P, int64_t t, double *theta,
                              double *logprior, double *loglik, void *state, const double *hchol,
                              uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter,
                              int64_t *n_accept, uint8_t *accepted, const KernelTimer *timer,
                              const MomFuse *fuse, hipStream_t s) {
    return launch_rw_shape<M, 64, kUnroll>(m, P, t, theta, logprior, loglik, state, hchol, seed,
                                           run, cycle, iter, n_accept, accepted, timer, fuse, s);
  }

  static smc_status mutate_indep(const DevModel &m, int64_t P, int64_t t, double *theta,
                                 double *logprior, double *loglik, void *state,
                                 const double *chol, const double *mean, uint64_t seed,
                                 uint64_t run, uint64_t cycle, uint64_t iter, int64_t *n_accept,
                                 uint8_t *accepted, const KernelTimer *timer, hipStream_t s) {
    auto *acc = reinterpret_cast<unsigned long long *>(n_accept);
    const typename M::Y *yd = Eval<M>::host_y(m);
    if (timer)
      hipExtLaunchKernelGGL(k_mutate_indep<M>, grid_for(P, 64), dim3(64), 0, s, timer->start,
                            timer->stop, 0, m, P, t, theta, logprior, loglik, state, chol, mean,
                            seed, run, cycle, iter, acc, accepted, yd);
    else
      hipLaunchKernelGGL(k_mutate_indep<M>, grid_for(P, 64), dim3(64), 0, s, m, P, t, theta,
                         logprior, loglik, state, chol, mean, seed, run, cycle, iter, acc,
                         accepted, yd);
    return launch_status("mutate/independent");
  }

  static smc_status loglik(const DevModel &m, int64_t P, const double *theta, int64_t t,
                           double *out, void *state_out, hipStream_t s) {
    hipLaunchKernelGGL(k_loglik<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, t, out,
                       state_out);
    return launch_status("loglik");
  }

  static size_t ckpt_bytes(const DevModel &, int64_t P, int64_t t) {
    if constexpr (IsLinreg<M>::value || !HasAdjoint<M>::value) {
      return 0;
    } else {
      using A = Adjoint<M>;
      const int64_t ns = (t + A::SEG - 1) / A::SEG;
      return (size_t)ns * M::K * (size_t)P * sizeof(typename M::R);
    }
  }

  static smc_status loglik_backward(const DevModel &m, int64_t P, const double *theta, int64_t t,
                                    const double *dloglik, double *dtheta, void *ckpt,
                                    hipStream_t s) {
    if constexpr (!HasAdjoint<M>::value) {
      return set_error(SMC_E_UNSUPPORTED, "no adjoint for normal-mixture shocks");
    } else {
      hipLaunchKernelGGL(k_loglik_backward<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m,
                         P, theta, t, dloglik, dtheta, ckpt);
      return launch_status("loglik_backward");
    }
  }

  static smc_status grad_post(const DevModel &m, int64_t P, const double *theta, int64_t t,
                              double *grad, void *ckpt, hipStream_t s) {
    if constexpr (!HasAdjoint<M>::value) {
      return set_error(SMC_E_UNSUPPORTED, "no adjoint for normal-mixture shocks");
    } else {
      hipLaunchKernelGGL(k_grad_post<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m, P,
                         theta, t, grad, ckpt);
      return launch_status("posterior_grad");
    }
  }

  static int32_t num_tests(int32_t which) { return which == 0 ? M::D : M::kTests; }

  static smc_status test_fns(const DevModel &m, int64_t P, const double *theta, const void *state,
                             int64_t t, int32_t which, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_test_fns<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, state, t,
                       which, out);
    return launch_status("test_functions");
  }

  static smc_status mutate_mala(const DevModel &m, int64_t P, int64_t t, double *theta,
                                double *logprior, double *loglik, void *state, double *grad,
                                const double *hchol, uint64_t seed, uint64_t run, uint64_t cycle,
                                uint64_t iter, int64_t *n_accept, uint8_t *accepted, void *ckpt,
                                hipStream_t s) {
    if constexpr (!HasAdjoint<M>::value) {
      return set_error(SMC_E_UNSUPPORTED, "no adjoint for normal-mixture shocks");
    } else {
      hipLaunchKernelGGL(k_mutate_mala<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m, P,
                         t, theta, logprior, loglik, state, grad, hchol, seed, run, cycle, iter,
                         reinterpret_cast<unsigned long long *>(n_accept), accepted, ckpt);
      return launch_status("mutate/mala");
    }
  }
};

template <class M>
const ModelOps *ops_table() {
  static const ModelOps o{&OpsOf<M>::init,       &OpsOf<M>::cscan,
                          &OpsOf<M>::ccommit,    &OpsOf<M>::mutate_rw,
                          &OpsOf<M>::loglik,     &OpsOf<M>::ckpt_bytes,
                          &OpsOf<M>::loglik_backward, &OpsOf<M>::grad_post,
                          &OpsOf<M>::mutate_mala, &OpsOf<M>::num_tests,
                          &OpsOf<M>::test_fns,   &OpsOf<M>::mutate_indep};
  return &o;
}

}  // namespace smc
