// Model-independent HIP kernels of the sequential posterior simulator for
// gfx950 (CDNA4) and the host-side launchers, including the routing of the
// model-templated launchers (model_kernels.h) to each model's table.
//
// The bandwidth-shaped kernels (reductions, resampling, gathers) use
// 256-thread blocks.  Every reduction combines in a fixed order, so results
// do not depend on timing.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include <algorithm>

#include "common.h"
#include "launch.h"
#include "model.h"
#include "chol.h"
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

}  // namespace

// ------------------------------------------------------------------ fills --
__global__ void k_fill_f64(double *a, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
__global__ void k_fill_i64(int64_t *a, int64_t n, int64_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

smc_status fill_f64(double *a, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return SMC_OK;
  hipLaunchKernelGGL(k_fill_f64, grid_for(n, kBlock), dim3(kBlock), 0, s, a, n, v);
  return launch_status("fill_f64");
}
smc_status fill_i64(int64_t *a, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return SMC_OK;
  hipLaunchKernelGGL(k_fill_i64, grid_for(n, kBlock), dim3(kBlock), 0, s, a, n, v);
  return launch_status("fill_i64");
}
smc_status fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return SMC_OK;
  hipLaunchKernelGGL(k_fill_i32, grid_for(n, kBlock), dim3(kBlock), 0, s, a, n, v);
  return launch_status("fill_i32");
}

constexpr int kRssBlock = 1024;
constexpr int kRssRegs = 16;  // values per thread held in registers: P <= 16,384 per column

// Reduction over a block of kRssBlock threads, the 16 wave values combined in
// wave order by every thread.
template <class Op>
__device__ __forceinline__ double rss_block_reduce(double v, double *lds /* >= 16 */) {
  v = wave_reduce<Op>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int i = 1; i < kRssBlock / 64; ++i) r = Op::apply(r, lds[i]);
  return r;
}
// Two sums at once (one pair of barriers), each in the order above.
__device__ __forceinline__ void rss_block_sum2(double &a, double &b, double *lds /* >= 32 */) {
  a = wave_reduce<OpSum<double>>(a);
  b = wave_reduce<OpSum<double>>(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6] = a;
    lds[kRssBlock / 64 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  double ra = lds[0], rb = lds[kRssBlock / 64];
#pragma unroll
  for (int i = 1; i < kRssBlock / 64; ++i) {
    ra += lds[i];
    rb += lds[kRssBlock / 64 + i];
  }
  a = ra;
  b = rb;
}

// RSS of one column of running log weights (Section 3.3):
// (sum e)^2 / (P sum e^2) with e = exp(logw - max).  Columns of up to
// kRssRegs * kRssBlock values: the maximum first, then the sums, the values
// held in registers between the two passes.
// Block b takes columns b, b + gridDim.x, ... below ncols (or *ncols_dev, the
// count of a device-driven chunk).
__global__ void __launch_bounds__(1024) k_rss_cols(const double *W, int64_t P, double *rss,
                                                   int32_t ncols, const int32_t *ncols_dev) {
  __shared__ double sh[2 * (kRssBlock / 64)];
  const int32_t nc = ncols_dev ? *ncols_dev : ncols;
  for (int32_t col = blockIdx.x; col < nc; col += gridDim.x) {
  const double *w = W + (int64_t)col * P;
  double v[kRssRegs];
  double mx = -INFINITY;
#pragma unroll
  for (int u = 0; u < kRssRegs; ++u) {
    const int64_t p = threadIdx.x + (int64_t)u * kRssBlock;
    v[u] = p < P ? w[p] : -INFINITY;
  }
#pragma unroll
  for (int u = 0; u < kRssRegs; ++u) mx = fmax(mx, v[u]);
  mx = rss_block_reduce<OpMax<double>>(mx, sh);
  double s1 = 0.0, s2 = 0.0;
  if (mx > -INFINITY) {
#pragma unroll
    for (int u = 0; u < kRssRegs; ++u) {
      const double e = exp_nonpos(v[u] - mx);
      s1 += e;
      s2 = fma(e, e, s2);
    }
  }
  rss_block_sum2(s1, s2, sh);
  if (threadIdx.x == 0) rss[col] = (mx > -INFINITY) ? s1 * s1 / ((double)P * s2) : 0.0;
  }  // every LDS write above follows a barrier, so the columns need none between them
}

// Longer columns in slices of kRssSlice values (8 per thread, so more blocks
// overlap their loads with other blocks' exponentials): block (column, slice) takes
// its slice's maximum m and s1 = sum exp(w - m), s2 = sum exp(2 (w - m)) as
// k_rss_cols does a whole column (values in registers, two passes), and
// k_rss_merge combines a column's slices in slice order, rescaling by
// exp(m_slice - m).  Blocks loop over (column, slice) pairs below
// ncols * S (or *ncols_dev * S in a device-driven chunk).
struct Lse3 {
  double m, s1, s2;
};
__device__ __forceinline__ Lse3 lse3_merge(Lse3 a, Lse3 b) {
  const double m = fmax(a.m, b.m);
  if (!(m > -INFINITY)) return Lse3{m, 0.0, 0.0};
  const double ea = exp_nonpos(a.m - m), eb = exp_nonpos(b.m - m);
  return Lse3{m, a.s1 * ea + b.s1 * eb, a.s2 * ea * ea + b.s2 * eb * eb};
}

constexpr int kSliceRegs = 8;  // values per thread in a slice: more blocks in flight per CU
constexpr int64_t kRssSlice = (int64_t)kSliceRegs * kRssBlock;

__global__ void __launch_bounds__(1024) k_rss_slices(const double *W, int64_t P, int32_t S,
                                                     double *part, int32_t ncols,
                                                     const int32_t *ncols_dev) {
  __shared__ double sh[2 * (kRssBlock / 64)];
  const int32_t total = (ncols_dev ? *ncols_dev : ncols) * S;
  for (int32_t b = blockIdx.x; b < total; b += gridDim.x) {
    const int32_t col = b / S, sl = b - col * S;
    const int64_t p0 = (int64_t)sl * kRssSlice;
    const int64_t n = min(kRssSlice, P - p0);
    const double *w = W + (int64_t)col * P + p0;
    double v[kSliceRegs];
#pragma unroll
    for (int u = 0; u < kSliceRegs; ++u) {
      const int64_t p = threadIdx.x + (int64_t)u * kRssBlock;
      v[u] = p < n ? w[p] : -INFINITY;
    }
    double mx = v[0];
#pragma unroll
    for (int u = 1; u < kSliceRegs; ++u) mx = fmax(mx, v[u]);
    mx = rss_block_reduce<OpMax<double>>(mx, sh);
    double s1 = 0.0, s2 = 0.0;
    if (mx > -INFINITY) {
#pragma unroll
      for (int u = 0; u < kSliceRegs; ++u) {
        const double e = exp_nonpos(v[u] - mx);
        s1 += e;
        s2 = fma(e, e, s2);
      }
    }
    rss_block_sum2(s1, s2, sh);
    if (threadIdx.x == 0) {
      part[3 * (int64_t)b] = mx;
      part[3 * (int64_t)b + 1] = s1;
      part[3 * (int64_t)b + 2] = s2;
    }
  }  // every LDS write above follows a barrier
}

__global__ void __launch_bounds__(256) k_rss_merge(const double *part, int64_t P, int32_t S,
                                                   double *rss, int32_t ncols,
                                                   const int32_t *ncols_dev) {
  const int32_t nc = ncols_dev ? *ncols_dev : ncols;
  const int32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  const double *q = part + 3 * (int64_t)c * S;
  Lse3 acc{q[0], q[1], q[2]};
  for (int32_t sl = 1; sl < S; ++sl) acc = lse3_merge(acc, Lse3{q[3 * sl], q[3 * sl + 1], q[3 * sl + 2]});
  rss[c] = (acc.m > -INFINITY) ? acc.s1 * acc.s1 / ((double)P * acc.s2) : 0.0;
}

// RSS of the C-phase scan's dates from its per-wave triples (k_cscan):
// block b takes dates b, b + gridDim.x, ... below ncols (or *ncols_dev); each
// thread merges the triples of waves tid, tid + 256, ... in order, then the
// block merges the threads' results in a fixed tree (lanes ^1 .. ^32 within
// each wave, then the four waves in order).
__device__ __forceinline__ Lse3 lse3_shfl_xor(const Lse3 &a, int off) {
  return Lse3{__shfl_xor(a.m, off, 64), __shfl_xor(a.s1, off, 64), __shfl_xor(a.s2, off, 64)};
}

__global__ void __launch_bounds__(256) k_rss_scan(const double *trip, int64_t P, int32_t nw,
                                                  double *rss, int32_t ncols,
                                                  const int32_t *ncols_dev) {
  __shared__ Lse3 sh[4];
  const int32_t nc = ncols_dev ? *ncols_dev : ncols;
  for (int32_t col = blockIdx.x; col < nc; col += gridDim.x) {
    const double *q = trip + (int64_t)col * nw * 3;
    Lse3 acc{-INFINITY, 0.0, 0.0};
    for (int32_t w = threadIdx.x; w < nw; w += 256)
      acc = lse3_merge(acc, Lse3{q[3 * w], q[3 * w + 1], q[3 * w + 2]});
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc = lse3_merge(acc, lse3_shfl_xor(acc, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const Lse3 t = lse3_merge(lse3_merge(sh[0], sh[1]), lse3_merge(sh[2], sh[3]));
      rss[col] = (t.m > -INFINITY) ? t.s1 * t.s1 / ((double)P * t.s2) : 0.0;
    }
    __syncthreads();  // sh is rewritten by the next date
  }
}

// The chunk's stopping decision (Section 3.3: the first checked date whose
// RSS is below rss_min): one wave scans the RSS values 64 at a time.  Value c
// is that of date first + c * check_every, the multiples of check_every after
// t up to t1, and t_max last when it is not a multiple.  With host_slot, the
// decision and the flags word also go to host memory, every 32-bit word of
// them paired with seq in an 8-byte word (DecisionSlot).  With cyc (a
// device-driven chunk) the chunk comes from there, a chunk without checked
// dates commits to t1 and does not end the phase, and the decision opens the
// S and M phases of a phase that ended: R = kappa Rbar iterations when the
// RSS is below D2, else Rbar (Section 3.3).
__global__ void __launch_bounds__(64) k_find_stop(const double *rss, int32_t nc, int64_t t,
                                                  int64_t t1, int64_t check_every, int64_t t_max,
                                                  double rss_min, StopInfo *out,
                                                  DecisionSlot *host_slot, uint32_t seq,
                                                  const int32_t *flags, CycleDyn *cyc) {
  if (cyc) {
    if (!cyc->go_c) return;
    nc = cyc->nc;
    t = cyc->t;
    t1 = cyc->t1;
    t_max = cyc->t_stop;
  }
  int first = -1;
  for (int base = 0; base < nc; base += 64) {
    const int c = base + (int)threadIdx.x;
    const uint64_t below = __ballot(c < nc && rss[c] < rss_min);
    if (below) {
      first = base + __builtin_ctzll(below);
      break;
    }
  }
  if (threadIdx.x == 0) {
    const int64_t first_date = (t / check_every + 1) * check_every;
    const int64_t n_regular = t1 >= first_date ? (t1 - first_date) / check_every + 1 : 0;
    const int col = first >= 0 ? first : nc - 1;
    StopInfo o;
    o.t_commit = first < 0 ? t1 : (first < n_regular ? first_date + first * check_every : t_max);
    o.rss = nc > 0 ? rss[col] : (cyc ? cyc->rss : 1.0);
    o.below = first >= 0;
    o.ends = nc > 0 && (first >= 0 || t1 >= t_max);
    *out = o;
    if (cyc) {
      const int32_t R = o.ends ? (o.rss < cyc->D2 ? cyc->kR : cyc->Rbar) : 0;
      cyc->t_new = o.t_commit;
      cyc->rss = o.rss;
      cyc->R = R;
      cyc->r0 = 0;
      cyc->go_s = o.ends;
      cyc->go_m = o.ends;
    }
    if (host_slot) {
      const int32_t fl = *flags;
      const uint64_t tc = (uint64_t)o.t_commit;
      const uint64_t rb = __builtin_bit_cast(uint64_t, o.rss);
      uint4 *dst = reinterpret_cast<uint4 *>(host_slot);
      dst[0] = make_uint4(seq, (uint32_t)tc, seq, (uint32_t)(tc >> 32));
      dst[1] = make_uint4(seq, (uint32_t)rb, seq, (uint32_t)(rb >> 32));
      dst[2] = make_uint4(seq, (uint32_t)fl, seq, (uint32_t)(o.ends | (o.below << 1)));
    }
  }
}

// ------------------------------------------------ device-driven cycles --
// Last date of the C phase that starts at t: T, the next multiple of
// force_every, or the burn-in date, whichever comes first.
__device__ __forceinline__ int64_t cycle_stop(const CycleDyn &c, int64_t t) {
  int64_t ts = c.T;
  if (c.force_every > 0) ts = min(ts, (t / c.force_every + 1) * c.force_every);
  if (c.burn_in > t) ts = min(ts, c.burn_in);
  return ts;
}

// The chunk (t, t1] of length at most c.chunk, and its checked dates: the
// multiples of check_every, and the phase's last date.
__device__ __forceinline__ void cycle_open_chunk(CycleDyn &c) {
  c.t1 = min(c.t + c.chunk, c.t_stop);
  const int64_t ce = c.check_every;
  c.nc = (int32_t)(c.t1 / ce - c.t / ce + ((c.t1 == c.t_stop && c.t_stop % ce != 0) ? 1 : 0));
  c.go_c = 1;
  c.go_scan = c.nc > 0;
}

// Start of a device-driven run: the fixed fields come from the host, the
// first chunk opens at t = 0.
__global__ void k_cycle_init(CycleDyn *c, CycleDyn init) {
  if (threadIdx.x != 0) return;
  init.t = 0;
  init.t_phase = 0;
  init.l = 0;
  init.zero_first = 1;
  init.last_len = 0;
  init.evals = 0;
  init.steps = 0;
  init.rss = 1.0;
  init.go_s = init.go_m = 0;
  init.r0 = init.R = 0;
  init.done = init.err = init.flags = 0;
  init.progress = 0;
  init.t_stop = cycle_stop(init, 0);
  init.chunk = min<int64_t>(16, init.cap);
  cycle_open_chunk(init);
  *c = init;
}

// End of a device-driven step.  After the last M slot of a cycle: record the
// cycle (date, iterations, RSS), count its evaluations, stop on a raised
// flag, at T or with the record full, else open the next cycle's C phase
// with a chunk twice the last phase's length plus 16 (the eager driver's
// speculation, so the chunks and their rounding are the same).  After M
// slots that leave iterations over: the next step runs only M slots.  After
// a chunk that did not end the phase: the next chunk, twice as long.  The
// host follows the run through *host: progress << 2 | err << 1 | done.
__global__ void k_cycle_end(CycleDyn *cp, int64_t *t_end, int32_t *r_rec, double *rss_rec,
                            const int32_t *flags, uint32_t *host, AccSink acc) {
  // the last M slot's accept counts (the slots' own moment launches add
  // those of the slots before them)
  if (acc.pending) acc_flush(acc, cp->P);
  if (threadIdx.x != 0) return;
  CycleDyn c = *cp;
  if (c.done || c.err) return;
  if (c.go_m) {
    const int32_t r_done = c.r0 + c.m_slots;
    if (r_done < c.R) {
      c.r0 = r_done;
      c.go_c = c.go_scan = c.go_s = 0;
    } else {
      const int32_t l = c.l;
      t_end[l] = c.t_new;
      r_rec[l] = c.R;
      rss_rec[l] = c.rss;
      c.evals += c.P * (c.t_new - c.t_phase) + (int64_t)c.R * c.P * c.t_new;
      c.steps += c.R;
      c.last_len = c.t_new - c.t_phase;
      c.t = c.t_phase = c.t_new;
      c.l = l + 1;
      c.zero_first = 1;
      c.go_c = c.go_scan = c.go_s = c.go_m = 0;
      c.r0 = c.R = 0;
      const int32_t fl = *flags;
      if (fl) {
        c.err = 2;
        c.flags = fl;
      } else if (c.t >= c.T) {
        c.done = 1;
      } else if (c.l >= c.Lmax) {
        c.err = 1;
      } else {
        c.t_stop = cycle_stop(c, c.t);
        c.chunk = min(max<int64_t>(16, 2 * c.last_len + 16), c.cap);
        cycle_open_chunk(c);
      }
    }
  } else if (c.go_c) {
    c.t = c.t_new;
    c.zero_first = 0;
    c.chunk = min(2 * c.chunk, c.cap);
    cycle_open_chunk(c);
  }
  c.progress += 1;
  *cp = c;
  __threadfence_system();
  __hip_atomic_store(host, (c.progress << 2) | (c.err ? 2u : 0u) | (c.done ? 1u : 0u),
                     __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A C phase driven on the device (smc_correct_async): the state opens its
// first chunk; after each chunk the phase either has ended (its date and RSS
// stay in the state) or opens the next chunk, twice as long; at the end the
// date and RSS are copied to the caller's outputs.
__global__ void k_phase_init(CycleDyn *c, CycleDyn init) {
  if (threadIdx.x != 0) return;
  cycle_open_chunk(init);
  *c = init;
}

__global__ void k_phase_step(CycleDyn *cp) {
  if (threadIdx.x != 0) return;
  CycleDyn c = *cp;
  if (!c.go_c) return;
  if (c.go_s) {  // the decision ended the phase
    c.go_c = c.go_scan = 0;
    c.done = 1;
  } else {
    c.t = c.t_new;
    c.zero_first = 0;
    c.chunk = min(2 * c.chunk, c.cap);
    cycle_open_chunk(c);
  }
  *cp = c;
}

__global__ void k_phase_out(const CycleDyn *c, const double *rss_src, int64_t t_fixed,
                            int64_t *t_to, double *rss) {
  if (threadIdx.x != 0) return;
  if (c) {
    t_to[0] = c->t_new;
    if (rss) rss[0] = c->rss;
  } else {
    t_to[0] = t_fixed;
    if (rss) rss[0] = rss_src[0];
  }
}

// ------------------------------------------------------------ S phase (a3) --
// One block of kSBlock threads (16 waves) per group.  The group's weights,
// then their running residual sums, live in LDS when they fit (kCumLdsMax),
// else in the workspace; the copy counts, then the ancestors' first output
// slots, in LDS.  Residual: floor(N W_n) copies, then the remaining draws
// from the residuals; multinomial: N draws from W_n; stratified / systematic
// (Section 3.3's experimental schemes): the k-th of N draws at (k + U_k)/N,
// respectively (k + U)/N, of the running sum.  A group's block is
// latency-bound, so the scans work within waves and every search runs a
// fixed number of steps, four of them interleaved per thread.
constexpr int kSBlock = 1024;         // threads per group
constexpr int kSWaves = kSBlock / 64;
constexpr int kCumLdsMax = 2048;      // groups up to this size keep their sums in LDS
constexpr int kResampleMaxN = 16384;  // the counts alone fill 64 KB of LDS here
constexpr int kGatherQ = 2;           // particles per thread per gather pass (global path)
constexpr int kGatherRows = 6;        // rows per batch of gather loads (global path)
constexpr int kGatherLdsBytes = 98304;  // LDS staging of source rows (groups <= kCumLdsMax)
constexpr int kStageRows = 8;          // rows of staging loads in flight together
constexpr int kStageQ = kCumLdsMax / kSBlock;  // particles per thread in an LDS-held group

// Reduction over the group's block: wave_reduce within each wave, then the
// wave values combined in one fixed pairwise tree, the same in every thread.
template <class Op>
__device__ __forceinline__ double sblock_reduce(double v, double *lds /* >= kSWaves */) {
  v = wave_reduce<Op>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double x[kSWaves];
#pragma unroll
  for (int i = 0; i < kSWaves; ++i) x[i] = lds[i];
#pragma unroll
  for (int s = 1; s < kSWaves; s <<= 1)
#pragma unroll
    for (int i = 0; i < kSWaves; i += 2 * s) x[i] = Op::apply(x[i], x[i + s]);
  return x[0];
}

// Exclusive scan over the group's block (DPP scans within the waves, then the
// totals of the preceding waves); `total` receives the block sum.
template <typename T>
__device__ __forceinline__ T sblock_exclusive_scan(T v, T *lds /* >= kSWaves */, T &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(v);
  const T up = __shfl_up(inc, 1, 64);
  const T ex = lane ? up : T(0);  // the wave's exclusive prefix
  __syncthreads();
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  T pre = T(0), tot = T(0);
#pragma unroll
  for (int i = 0; i < kSWaves; ++i) {
    const T x = lds[i];
    if (i < w) pre += x;
    tot += x;
  }
  total = tot;
  return pre + ex;
}

// Largest power of two not above n (n >= 1): the first step of the searches.
__device__ __forceinline__ int top_step(int n) { return 1 << (31 - __clz(n)); }

// Group maximum of logw and sum of exp(logw - max), in one order that the
// S-phase kernel and k_group_logwbar share (so both give the same bits).
// `keep`, when given, receives the log weights, then their exponentials.
__device__ __forceinline__ void group_max_sum(const double *lw, int32_t N, double *keep,
                                              double *sh, double &mx, double &se) {
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int n = tid; n < N; n += kSBlock) {
    const double v = lw[n];
    if (keep) keep[n] = v;
    m = fmax(m, v);
  }
  m = sblock_reduce<OpMax<double>>(m, sh);
  double s = 0.0;
  if (m > -INFINITY)
    for (int n = tid; n < N; n += kSBlock) {
      const double e = exp_nonpos((keep ? keep[n] : lw[n]) - m);
      if (keep) keep[n] = e;
      s += e;
    }
  se = sblock_reduce<OpSum<double>>(s, sh);  // its barriers publish `keep`
  mx = m;
}

// log wbar_j = log(N^-1 sum_n exp(logw_jn)) per group (Section 4.2).
__global__ void __launch_bounds__(kSBlock) k_group_logwbar(const double *logw, int32_t N,
                                                           double *out) {
  __shared__ double sh[kSWaves];
  double mx, s;
  group_max_sum(logw + (int64_t)blockIdx.x * N, N, nullptr, sh, mx, s);
  if (threadIdx.x == 0) out[blockIdx.x] = (mx > -INFINITY) ? mx + log(s / (double)N) : -INFINITY;
}

struct GatherArgs {
  const int32_t *anc;
  int64_t P;
  int32_t d, S, st_bytes, has_grad;
  double *theta, *logprior, *loglik, *grad;
  void *state;
  double *tmp;  // [2d + S + 2][P]
};

// Row r of the particle arrays in gather order: theta rows, log prior, log
// likelihood, state rows, gradient rows (rows are wave-uniform).
__device__ __forceinline__ double gather_load(const GatherArgs &g, int r, int64_t i) {
  if (r < g.d) return g.theta[r * g.P + i];
  r -= g.d;
  if (r == 0) return g.logprior[i];
  if (r == 1) return g.loglik[i];
  r -= 2;
  if (r < g.S)
    return g.st_bytes == 8 ? typed<double>(g.state)[r * g.P + i]
                           : (double)typed<float>(g.state)[r * g.P + i];
  r -= g.S;
  return g.grad[r * g.P + i];
}
// Start of row r and whether it holds floats (an FP32 model's state).
__device__ __forceinline__ const void *gather_row(const GatherArgs &g, int r, bool &f32) {
  f32 = false;
  if (r < g.d) return g.theta + r * g.P;
  r -= g.d;
  if (r == 0) return g.logprior;
  if (r == 1) return g.loglik;
  r -= 2;
  if (r < g.S) {
    f32 = g.st_bytes == 4;
    return f32 ? static_cast<const void *>(typed<float>(g.state) + r * g.P)
               : static_cast<const void *>(typed<double>(g.state) + r * g.P);
  }
  r -= g.S;
  return g.grad + r * g.P;
}
__device__ __forceinline__ void gather_store(const GatherArgs &g, int r, int64_t i, double v) {
  if (r < g.d) { g.theta[r * g.P + i] = v; return; }
  r -= g.d;
  if (r == 0) { g.logprior[i] = v; return; }
  if (r == 1) { g.loglik[i] = v; return; }
  r -= 2;
  if (r < g.S) {
    if (g.st_bytes == 8) typed<double>(g.state)[r * g.P + i] = v;
    else typed<float>(g.state)[r * g.P + i] = (float)v;
    return;
  }
  r -= g.S;
  g.grad[r * g.P + i] = v;
}

// In-place gather held in registers (N <= kSBlock, rows <= kRegRows): every
// thread loads all rows of its particle's ancestor, the block synchronises,
// then every thread stores them at its own position.
constexpr int kRegRows = 16;
__device__ __forceinline__ void gather_in_registers(const GatherArgs &g, int64_t base, int32_t N,
                                                    int rows, const int32_t *anc_l) {
  double v[kRegRows];
  const int n = threadIdx.x;
  const int64_t a = base + (n < N ? anc_l[n] : 0);
#pragma unroll
  for (int r = 0; r < kRegRows; ++r)
    if (r < rows) v[r] = gather_load(g, r, a);
  __syncthreads();
  if (n < N)
#pragma unroll
    for (int r = 0; r < kRegRows; ++r)
      if (r < rows) gather_store(g, r, base + n, v[r]);
}

// Copy counts and ancestors of group j.  Its weights, then their running
// sums, go to ev (LDS, or the workspace for large groups), the counts, then
// every n's first output slot, to cnt (LDS), and the group-local ancestors
// also to anc_l when given.  Returns false for a dead group (no positive
// weight), whose ancestors are the identity.
__device__ __forceinline__ bool select_ancestors(const double *lw, int32_t N, int32_t scheme,
                                                 uint64_t seed, uint64_t run, uint64_t cycle,
                                                 int j, int64_t base, int32_t *anc,
                                                 int32_t *flags, double *group_logwbar,
                                                 double *ev, int32_t *cnt, int32_t *anc_l,
                                                 double *shd, int32_t *shi) {
  const int tid = threadIdx.x;
  double mx, se;
  group_max_sum(lw, N, ev, shd, mx, se);
  if (!(mx > -INFINITY)) {
    for (int n = tid; n < N; n += kSBlock) anc[base + n] = (int32_t)(base + n);
    if (tid == 0) {
      atomicOr(flags, SMC_FLAG_DEAD_GROUP);
      if (group_logwbar) group_logwbar[j] = -INFINITY;
    }
    return false;
  }
  // log wbar_j from the same maximum and sum as k_group_logwbar
  if (group_logwbar && tid == 0) group_logwbar[j] = mx + log(se / (double)N);

  // Thread-contiguous chunks: copy counts and running residual sums.
  const int m = (N + kSBlock - 1) / kSBlock;
  const int lo = min(tid * m, N), hi = min(lo + m, N);
  double rsum = 0.0;
  int32_t csum = 0;
  for (int n = lo; n < hi; ++n) {
    const double nw = ((double)N * ev[n]) / se;  // N W_n
    const double c = (scheme == SMC_RESAMPLE_RESIDUAL) ? floor(nw) : 0.0;
    rsum += nw - c;
    ev[n] = rsum;
    cnt[n] = (int32_t)c;
    csum += (int32_t)c;
  }
  double rtot;
  const double roff = sblock_exclusive_scan<double>(rsum, shd, rtot);
  for (int n = lo; n < hi; ++n) ev[n] += roff;
  int32_t ctot;
  (void)sblock_exclusive_scan<int32_t>(csum, shi, ctot);
  __syncthreads();
  const double *cum = ev;
  const double total = cum[N - 1];
  const int R = N - ctot;
  const int top = top_step(N);
  // Draws k = 4q..4q+3 share the Philox block q; each draw's ancestor is the
  // first n with cum[n] > u * total, found in top_step(N) halvings with the
  // four draws' loads issued together.
  const double u_sys = scheme == SMC_RESAMPLE_SYSTEMATIC
                           ? u01_co(draw4(seed, run, (uint64_t)j, cycle, 0, kResample).x0)
                           : 0.0;
  for (int q = tid; 4 * q < R; q += kSBlock) {
    const U64x4 w = draw4(seed, run, (uint64_t)j, cycle, (uint64_t)q, kResample);
    const uint64_t xs[4] = {w.x0, w.x1, w.x2, w.x3};
    double tg[4];
    int pos[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * q + i;
      double u = u01_co(xs[i]);
      if (scheme == SMC_RESAMPLE_STRATIFIED) u = ((double)k + u) / (double)N;
      else if (scheme == SMC_RESAMPLE_SYSTEMATIC) u = ((double)k + u_sys) / (double)N;
      tg[i] = u * total;
      pos[i] = 0;
    }
    for (int step = top; step > 0; step >>= 1) {
      double c[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = cum[min(pos[i] + step, N) - 1];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (pos[i] + step <= N && !(c[i] > tg[i])) pos[i] += step;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (4 * q + i >= R) break;
      int a = pos[i];
      if (a >= N) {  // u * total rounded up to the last sum: the last positive residual
        a = N - 1;
        while (a > 0 && !(cum[a] > cum[a - 1])) --a;
      }
      atomicAdd(&cnt[a], 1);
    }
  }
  __syncthreads();
  // Copy counts -> first output slot of every n (in place); the ancestor of
  // slot s is the last n whose first slot is <= s.
  int32_t my = 0;
  for (int n = lo; n < hi; ++n) my += cnt[n];
  int32_t tot2;
  int32_t at = sblock_exclusive_scan<int32_t>(my, shi, tot2);
  for (int n = lo; n < hi; ++n) {
    const int32_t c = cnt[n];
    cnt[n] = at;
    at += c;
  }
  __syncthreads();
  for (int s = tid; s < N; s += kSBlock) {
    int a = 0;
    for (int step = top; step > 0; step >>= 1) {
      const int nx = a + step;
      const int32_t first = cnt[min(nx, N) - 1];
      if (nx <= N && first <= s) a = nx;
    }
    --a;
    if (anc_l) anc_l[s] = a;
    anc[base + s] = (int32_t)(base + a);
  }
  __syncthreads();
  return true;
}

__global__ void __launch_bounds__(kSBlock) k_resample(const double *logw, int32_t N,
                                                      int32_t scheme, uint64_t seed, uint64_t run,
                                                      uint64_t cycle, int32_t *anc,
                                                      double *cum_ws, int32_t *flags,
                                                      GatherArgs g, const int32_t *go,
                                                      double *group_logwbar,
                                                      const CycleDyn *cyc) {
  if (go && *go == 0) return;  // enqueued ahead of a C phase that did not end
  if (cyc) {  // a device-driven cycle: its S phase, key, counter and record row
    if (!cyc->go_s) return;
    seed = cyc->seed;
    run = cyc->run;
    cycle = (uint64_t)(cyc->l + 1);
    group_logwbar += (int64_t)cyc->l * gridDim.x;
  }
  extern __shared__ double lds_dyn[];
  __shared__ double shd[kSWaves];
  __shared__ int32_t shi[kSWaves];
  const int j = blockIdx.x;
  const int64_t base = (int64_t)j * N;
  // LDS layout for groups up to kCumLdsMax: [N] doubles (weights, then the
  // running sums), [kGatherLdsBytes] of row staging, [N] int32 counts, [N]
  // int32 ancestors; larger groups keep the sums in the workspace and only
  // the counts in LDS.  The two cases are separate calls, so that every LDS
  // access compiles to an LDS instruction.
  const bool in_lds = N <= kCumLdsMax;
  double *stage = lds_dyn + N;
  int32_t *anc_l = reinterpret_cast<int32_t *>(stage + kGatherLdsBytes / 8) + N;
  if (in_lds) {
    if (!select_ancestors(logw + base, N, scheme, seed, run, cycle, j, base, anc, flags,
                          group_logwbar, lds_dyn, anc_l - N, anc_l, shd, shi))
      return;
  } else {
    if (!select_ancestors(logw + base, N, scheme, seed, run, cycle, j, base, anc, flags,
                          group_logwbar, cum_ws + base, reinterpret_cast<int32_t *>(lds_dyn),
                          nullptr, shd, shi))
      return;
  }
  const int tid = threadIdx.x;
  const int64_t P = g.P;
  const int rows = g.d + 2 + g.S + (g.has_grad ? g.d : 0);
  if (in_lds && rows <= kRegRows && N <= kSBlock) {
    gather_in_registers(g, base, N, rows, anc_l);
    return;
  }
  if (in_lds) {
    // Replace the group's particles by their ancestors through LDS: stage
    // B source rows of the whole group (coalesced loads, kStageRows rows of
    // every particle of the thread in flight together), then write every
    // particle's row values from its ancestor's slot.
    const int B = max(1, min(rows, kGatherLdsBytes / (8 * N)));
    for (int r0 = 0; r0 < rows; r0 += B) {
      const int nr = min(B, rows - r0);
      for (int rr0 = 0; rr0 < nr; rr0 += kStageRows) {
        const void *rp[kStageRows];
        bool f32[kStageRows];
#pragma unroll
        for (int u = 0; u < kStageRows; ++u)
          rp[u] = gather_row(g, r0 + min(rr0 + u, nr - 1), f32[u]);
        double v[kStageRows][kStageQ];
#pragma unroll
        for (int u = 0; u < kStageRows; ++u)
#pragma unroll
          for (int q = 0; q < kStageQ; ++q) {
            const int n = tid + q * kSBlock;
            const int64_t i = base + (n < N ? n : 0);
            v[u][q] = f32[u] ? (double)static_cast<const float *>(rp[u])[i]
                             : static_cast<const double *>(rp[u])[i];
          }
#pragma unroll
        for (int u = 0; u < kStageRows; ++u)
#pragma unroll
          for (int q = 0; q < kStageQ; ++q) {
            const int n = tid + q * kSBlock;
            if (rr0 + u < nr && n < N) stage[(rr0 + u) * N + n] = v[u][q];
          }
      }
      __syncthreads();
      for (int rr = 0; rr < nr; ++rr)
        for (int n = tid; n < N; n += kSBlock)
          gather_store(g, r0 + rr, base + n, stage[rr * N + anc_l[n]]);
      __syncthreads();
    }
    return;
  }
  // Larger groups: copy the ancestors' values to the workspace, then back,
  // with kGatherQ particles x kGatherRows rows of loads in flight per batch.
  for (int n0 = 0; n0 < N; n0 += kSBlock * kGatherQ) {
    int64_t pp[kGatherQ], aa[kGatherQ];
    bool ok[kGatherQ];
#pragma unroll
    for (int q = 0; q < kGatherQ; ++q) {
      const int n = n0 + q * kSBlock + tid;
      ok[q] = n < N;
      pp[q] = base + (ok[q] ? n : 0);
    }
#pragma unroll
    for (int q = 0; q < kGatherQ; ++q) aa[q] = anc[pp[q]];
    for (int r0 = 0; r0 < rows; r0 += kGatherRows) {
      double v[kGatherRows][kGatherQ];
#pragma unroll
      for (int rr = 0; rr < kGatherRows; ++rr)
        if (r0 + rr < rows)
#pragma unroll
          for (int q = 0; q < kGatherQ; ++q) v[rr][q] = gather_load(g, r0 + rr, aa[q]);
#pragma unroll
      for (int rr = 0; rr < kGatherRows; ++rr)
        if (r0 + rr < rows)
#pragma unroll
          for (int q = 0; q < kGatherQ; ++q)
            if (ok[q]) g.tmp[(r0 + rr) * P + pp[q]] = v[rr][q];
    }
  }
  __syncthreads();
  for (int n0 = 0; n0 < N; n0 += kSBlock * kGatherQ) {
    int64_t pp[kGatherQ];
    bool ok[kGatherQ];
#pragma unroll
    for (int q = 0; q < kGatherQ; ++q) {
      const int n = n0 + q * kSBlock + tid;
      ok[q] = n < N;
      pp[q] = base + (ok[q] ? n : 0);
    }
    for (int r0 = 0; r0 < rows; r0 += kGatherRows) {
      double v[kGatherRows][kGatherQ];
#pragma unroll
      for (int rr = 0; rr < kGatherRows; ++rr)
        if (r0 + rr < rows)
#pragma unroll
          for (int q = 0; q < kGatherQ; ++q) v[rr][q] = g.tmp[(r0 + rr) * P + pp[q]];
#pragma unroll
      for (int rr = 0; rr < kGatherRows; ++rr)
        if (r0 + rr < rows)
#pragma unroll
          for (int q = 0; q < kGatherQ; ++q)
            if (ok[q]) gather_store(g, r0 + rr, pp[q], v[rr][q]);
    }
  }
}

// ----------------------------------------------- particle moments (a4) ----
// Pass 1: every wave accumulates sum_p x_p x_p' on the matrix cores with
// x_p = (theta_p - s, 1, 0, ...) padded to W = 16 or 32 (s = particle 0, a
// shift that keeps the one-pass sums well conditioned; the constant slot d
// carries the first moments and the count).  v_mfma_f64_16x16x4f64 takes four
// particles per instruction.  Operand layout (measured on gfx950): lane l
// supplies element (row l%16, k = l/16) of A and (k = l/16, col l%16) of B,
// so A = B' = a 16x4 block of shifted particles; accumulator register r of
// lane l holds element (4r + l/16, l%16) of the 16x16 result.  With W = 32
// each lane holds rows i and 16 + i, and three products per step give the
// (0,0), (1,0) and (1,1) tiles of the symmetric result.  Each block writes
// one W x W partial matrix.  With sink.pending, one block more, the last,
// adds the previous Metropolis step's accept counts to their counter
// (acc_flush) while the others form the partials.
template <int W>
__global__ void __launch_bounds__(256) k_mom_partial(const double *theta, int64_t P, int32_t d,
                                                     int64_t chunk, double *part,
                                                     const CycleDyn *cyc, int32_t slot,
                                                     AccSink sink) {
  if (m_slot_off(cyc, slot)) return;  // an unused M slot of a device-driven cycle
  if (sink.pending && blockIdx.x == gridDim.x - 1) {
    if (threadIdx.x < 64) acc_flush(sink, P);
    return;
  }
  constexpr int NT = W / 16;
  constexpr int NA = NT == 1 ? 1 : 3;  // tiles accumulated
  __shared__ double red[4][W * W];
  typedef double double4v __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int i = l & 15, k = l >> 4;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + wv) * chunk;
  const int64_t p1 = min(P, p0 + chunk);
  int ir[NT];
  double si[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ir[t] = 16 * t + i < d ? 16 * t + i : 0;  // a valid row to load from
    si[t] = theta[(int64_t)ir[t] * P];
  }
  double4v acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = double4v{0.0, 0.0, 0.0, 0.0};
  // Batches of eight MFMA steps (32 particles).  Each batch's loads are
  // issued before the previous batch is consumed, so their latency overlaps
  // the matrix-core work (addresses are clamped into the wave's range and
  // the values masked afterwards).
  auto load = [&](int64_t q0, double (&x)[NT][8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = q0 + 4 * u + k;
      const int64_t pc = p < p1 ? p : p1 - 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) x[t][u] = theta[(int64_t)ir[t] * P + pc];
    }
  };
  auto consume = [&](int64_t q0, const double (&x)[NT][8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = q0 + 4 * u + k;
      double xm[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int row = 16 * t + i;
        const double v = (row < d) ? x[t][u] - si[t] : (row == d ? 1.0 : 0.0);
        xm[t] = p < p1 ? v : 0.0;
      }
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(xm[0], xm[0], acc[0], 0, 0, 0);
      if constexpr (NT == 2) {
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(xm[1], xm[0], acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(xm[1], xm[1], acc[2], 0, 0, 0);
      }
    }
  };
  double xa[NT][8], xb[NT][8];
  if (p0 < p1) load(p0, xa);
  for (int64_t q0 = p0; q0 < p1; q0 += 64) {
    const int64_t q1 = q0 + 32;
    if (q1 < p1) load(q1, xb);
    consume(q0, xa);
    if (q1 < p1) {
      if (q1 + 32 < p1) load(q1 + 32, xa);
      consume(q1, xb);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * r + k;
    red[wv][row * W + i] = acc[0][r];
    if constexpr (NT == 2) {
      red[wv][(16 + row) * W + i] = acc[1][r];   // tile (1,0)
      red[wv][i * W + 16 + row] = acc[1][r];     // its mirror (0,1)
      red[wv][(16 + row) * W + 16 + i] = acc[2][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < W * W; e += 256)
    part[(int64_t)blockIdx.x * W * W + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// The partial matrices are first added entry by entry across a few blocks,
// so the final step reads one matrix.  A block takes 64
// entries; each of its four waves adds a quarter of the partials in block
// order (its loads in flight together), and the four subtotals are added in
// wave order.
__global__ void __launch_bounds__(256) k_mom_sum(const double *part, int32_t nb, int32_t n,
                                                 double *out, const CycleDyn *cyc, int32_t slot) {
  if (m_slot_off(cyc, slot)) return;
  __shared__ double sub[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int per = (nb + 3) / 4;
  const int b_lo = min(nb, wv * per), b_hi = min(nb, b_lo + per);
  constexpr int kBatch = 32;
  double sum = 0.0;
  if (e < n) {
    for (int b0 = b_lo; b0 < b_hi; b0 += kBatch) {
      double x[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        x[q] = (b0 + q < b_hi) ? part[(int64_t)(b0 + q) * n + e] : 0.0;
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        if (b0 + q < b_hi) sum += x[q];
    }
  }
  sub[wv][lane] = sum;
  __syncthreads();
  if (wv == 0 && e < n) out[e] = ((sub[0][lane] + sub[1][lane]) + sub[2][lane]) + sub[3][lane];
}

// Pass 2 (one block of W * W threads, one entry each): add the partial
// matrices in block order, optionally apply the step-size rule to mh, form
// the mean and V (divisor P - 1), factor V = L L' and write h L.  A variance
// that is not positive definite raises the flag and yields h L = 0.
template <int W>
__global__ void __launch_bounds__(W * W) k_mom_final(MomArgs a, int32_t nb) {
  __shared__ double Ms[W * W];
  __shared__ double Ls[W * chol_ld<W>()];
  __shared__ double sh_h;
  const int e = threadIdx.x;  // entry (r, c) = (e / W, e % W)
  const int d = a.d;
  const int64_t P = a.P;
  // the step-size inputs are read first so their latency overlaps the sums
  int32_t m = 0;
  int64_t nacc = 0;
  if (e == 0) {
    m = *a.mh;
    if (a.mh_reset <= 0 && a.prev_nacc) nacc = *a.prev_nacc;
  }
  // Partials are added in block order, up to 32 loads in flight per thread.
  constexpr int kBatch = 32;
  const double *pp = a.part + e;
  double sum = 0.0;
  for (int b0 = 0; b0 < nb; b0 += kBatch) {
    double x[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) x[q] = (b0 + q < nb) ? pp[(int64_t)(b0 + q) * W * W] : 0.0;
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
      if (b0 + q < nb) sum += x[q];
  }
  Ms[e] = sum;
  if (e == 0) {
    if (a.mh_reset > 0) {
      m = a.mh_reset;
    } else if (a.prev_nacc) {
      m += (nacc * 1000 > (int64_t)a.target_permille * P) ? 1 : -1;
      m = m < 1 ? 1 : (m > 10 ? 10 : m);
    }
    *a.mh = m;
    sh_h = (double)m / 10.0;
  }
  __syncthreads();
  const double invP = 1.0 / (double)P;
  const int r = e / W, c = e % W;
  double v = 0.0;
  if (r < d && c < d) {
    v = (Ms[r * W + c] - Ms[r * W + d] * Ms[c * W + d] * invP) / (double)(P - 1);
    if (a.cov_out) a.cov_out[r * d + c] = v;
  }
  if (a.mean_out && e < d) a.mean_out[e] = a.theta[(int64_t)e * P] + Ms[e * W + d] * invP;
  __syncthreads();
  if (r < d && c < d) Ms[e] = v;
  __syncthreads();
  if (e < 64) wave_cholesky<W>(Ms, Ls, d, sh_h, a.hchol, a.flags);
}

// ------------------------------------------------ step size, RNE, log-ML --
__global__ void k_adapt(const int64_t *n_accept, int64_t P, int32_t target_permille, int32_t *mh) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t n = *n_accept;
  int32_t v = *mh + ((n * 1000 > (int64_t)target_permille * P) ? 1 : -1);
  *mh = v < 1 ? 1 : (v > 10 ? 10 : v);
}

// Per group j and parameter i: the group mean and the within-group sum of
// squared deviations.
__global__ void __launch_bounds__(256) k_rne_group(const double *theta, int64_t P, int32_t N,
                                                   int32_t d, double *part) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  for (int i = 0; i < d; ++i) {
    const double *x = theta + i * P + (int64_t)j * N;
    double s = 0.0;
    for (int n = threadIdx.x; n < N; n += kBlock) s += x[n];
    const double mean = block_reduce<OpSum<double>>(s, sh) / (double)N;
    double q = 0.0;
    for (int n = threadIdx.x; n < N; n += kBlock) {
      const double e = x[n] - mean;
      q = fma(e, e, q);
    }
    q = block_reduce<OpSum<double>>(q, sh);
    if (threadIdx.x == 0) {
      part[(int64_t)j * 2 * kDMax + i] = mean;
      part[(int64_t)j * 2 * kDMax + kDMax + i] = q;
    }
  }
}

// RNE_i = var-hat / v-hat with var-hat = (within SS + N sum_j (gbar_j - gbar)^2)
// / (NJ - 1) and v-hat = N / (J - 1) sum_j (gbar_j - gbar)^2; mean over i.
__global__ void k_rne_final(const double *part, int32_t J, int32_t N, int32_t d, double *rne) {
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int i = 0; i < d; ++i) {
    double g = 0.0, w = 0.0;
    for (int j = 0; j < J; ++j) {
      g += part[(int64_t)j * 2 * kDMax + i];
      w += part[(int64_t)j * 2 * kDMax + kDMax + i];
    }
    g /= (double)J;
    double b = 0.0;
    for (int j = 0; j < J; ++j) {
      const double e = part[(int64_t)j * 2 * kDMax + i] - g;
      b += e * e;
    }
    const double var = (w + (double)N * b) / ((double)N * J - 1.0);
    const double vhat = (double)N * b / (double)(J - 1);
    acc += var / vhat;
  }
  *rne = acc / (double)d;
}

// Moment report from k_rne_group's group means and within-group sums of
// squares (Section 2.3): mean, sd = var-hat^(1/2), NSE (eq NSE_def), RNE =
// var-hat / v-hat (eq vhat); and the mean RNE over the G functions.
__global__ void k_report_final(const double *part, int32_t J, int32_t N, int32_t G, double *out,
                               double *rne_mean) {
  if (threadIdx.x != 0) return;
  double acc = 0.0;
  for (int i = 0; i < G; ++i) {
    double g = 0.0, w = 0.0;
    for (int j = 0; j < J; ++j) {
      g += part[(int64_t)j * 2 * kDMax + i];
      w += part[(int64_t)j * 2 * kDMax + kDMax + i];
    }
    g /= (double)J;
    double b = 0.0;
    for (int j = 0; j < J; ++j) {
      const double e = part[(int64_t)j * 2 * kDMax + i] - g;
      b += e * e;
    }
    const double var = (w + (double)N * b) / ((double)N * J - 1.0);
    const double vhat = (double)N * b / (double)(J - 1);
    out[i * 4 + 0] = g;
    out[i * 4 + 1] = sqrt(var);
    out[i * 4 + 2] = sqrt(b / ((double)J * (J - 1)));
    out[i * 4 + 3] = var / vhat;
    acc += var / vhat;
  }
  if (rne_mean) *rne_mean = acc / (double)G;
}

// log wbar, its delta-method NSE and log wtilde from group_logwbar[L][J].
__global__ void __launch_bounds__(256) k_log_ml(int32_t L, int32_t J, const double *g,
                                                double *out) {
  __shared__ double sh[4];
  const int tid = threadIdx.x;
  // log wbar_j = sum_l log wbar_j(l): each thread owns groups j = tid + 256 k
  // and sums over the cycles in order.
  auto lw = [&](int j) {
    double s = 0.0;
    for (int l = 0; l < L; ++l) s += g[(int64_t)l * J + j];
    return s;
  };
  double m = -INFINITY;
  for (int j = tid; j < J; j += kBlock) m = fmax(m, lw(j));
  const double mx = block_reduce<OpMax<double>>(m, sh);
  double r = 0.0;
  for (int j = tid; j < J; j += kBlock) r += exp(lw(j) - mx);
  const double rbar = block_reduce<OpSum<double>>(r, sh) / (double)J;
  double q = 0.0;
  for (int j = tid; j < J; j += kBlock) {
    const double e = exp(lw(j) - mx) - rbar;
    q = fma(e, e, q);
  }
  const double ss = block_reduce<OpSum<double>>(q, sh);
  // log wtilde = sum_l log mean_j wbar_j(l): each thread owns cycles.
  double lt = 0.0;
  for (int l = tid; l < L; l += kBlock) {
    const double *gl = g + (int64_t)l * J;
    double ml = -INFINITY;
    for (int j = 0; j < J; ++j) ml = fmax(ml, gl[j]);
    double sl = 0.0;
    for (int j = 0; j < J; ++j) sl += exp(gl[j] - ml);
    lt += (ml > -INFINITY) ? ml + log(sl / (double)J) : -INFINITY;
  }
  lt = block_reduce<OpSum<double>>(lt, sh);
  if (tid == 0) {
    out[0] = mx + log(rbar);
    out[1] = sqrt(ss / ((double)J * (J - 1))) / rbar;
    out[2] = lt;
  }
}

// ============================================================ launchers ====

// ---------------------------------------------- model-templated launchers --
const ModelOps *ops_for(const DevModel &m) {
  const ModelOps *o = nullptr;
  if (m.kind == SMC_MODEL_LINREG) o = ops_linreg(m);
  else if (m.shock != SMC_SHOCK_MIXTURE) o = ops_egarch(m);
  else if (m.prec == SMC_FP64) o = ops_mixture64(m);
  else o = ops_mixture32(m);
  if (!o)
    set_error(SMC_E_UNSUPPORTED, "model kind %d, K=%d, shock %d, I=%d, nreg %d", m.kind, m.K,
              m.shock, m.ncomp, m.nreg);
  return o;
}

smc_status launch_init(const DevModel &m, int64_t P, uint64_t seed, uint64_t run, double *theta,
                       double *logprior, double *loglik, void *state, double *logw,
                       hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->init(m, P, seed, run, theta, logprior, loglik, state, logw, s) : SMC_E_UNSUPPORTED;
}

smc_status launch_cscan(const DevModel &m, int64_t P, const double *theta, const void *state,
                        const double *logw, int64_t t0, int64_t t1, int64_t check_every,
                        int64_t t_max, bool zero_first, double *W, hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->cscan(m, P, theta, state, logw, t0, t1, check_every, t_max, zero_first, W, s)
           : SMC_E_UNSUPPORTED;
}

smc_status launch_ccommit(const DevModel &m, int64_t P, const double *theta, void *state,
                          double *logw, double *loglik, int64_t t0, int64_t t1, bool zero_first,
                          hipStream_t s, const int64_t *t1_dev) {
  const ModelOps *o = ops_for(m);
  return o ? o->ccommit(m, P, theta, state, logw, loglik, t0, t1, zero_first, t1_dev, s)
           : SMC_E_UNSUPPORTED;
}

bool has_launch_shapes(const DevModel &m) {
  return m.kind == SMC_MODEL_EGARCH &&
         ((m.K == 1 && m.shock == SMC_SHOCK_GAUSS) || (m.K == 2 && m.shock == SMC_SHOCK_STUDENT_T) ||
          (m.K == 2 && m.shock == SMC_SHOCK_MIXTURE && m.ncomp == 3));
}

smc_status launch_mutate_rw(const DevModel &m, int64_t P, int64_t t, double *theta,
                            double *logprior, double *loglik, void *state, const double *hchol,
                            uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter,
                            int64_t *n_accept, uint8_t *accepted, hipStream_t s,
                            const KernelTimer *timer, const MomFuse *fuse) {
  const bool shaped = (m.block != 0 && m.block != 64) || (m.unroll != 0 && m.unroll != kUnroll);
  if (shaped && m.shock == SMC_SHOCK_MIXTURE) {
    return m.prec == SMC_FP32
               ? launch_mutate_rw_shaped_mix32(m, P, t, theta, logprior, loglik, state, hchol,
                                               seed, run, cycle, iter, n_accept, accepted, timer,
                                               fuse, s)
               : launch_mutate_rw_shaped_mix64(m, P, t, theta, logprior, loglik, state, hchol,
                                               seed, run, cycle, iter, n_accept, accepted, timer,
                                               fuse, s);
  }
  if (shaped) {
    return m.prec == SMC_FP32
               ? launch_mutate_rw_shaped32(m, P, t, theta, logprior, loglik, state, hchol, seed,
                                           run, cycle, iter, n_accept, accepted, timer, fuse, s)
               : launch_mutate_rw_shaped64(m, P, t, theta, logprior, loglik, state, hchol, seed,
                                           run, cycle, iter, n_accept, accepted, timer, fuse, s);
  }
  const ModelOps *o = ops_for(m);
  return o ? o->mutate_rw(m, P, t, theta, logprior, loglik, state, hchol, seed, run, cycle, iter,
                          n_accept, accepted, timer, fuse, s)
           : SMC_E_UNSUPPORTED;
}

smc_status launch_mutate_indep(const DevModel &m, int64_t P, int64_t t, double *theta,
                               double *logprior, double *loglik, void *state, const double *chol,
                               const double *mean, uint64_t seed, uint64_t run, uint64_t cycle,
                               uint64_t iter, int64_t *n_accept, uint8_t *accepted,
                               hipStream_t s, const KernelTimer *timer) {
  const ModelOps *o = ops_for(m);
  return o ? o->mutate_indep(m, P, t, theta, logprior, loglik, state, chol, mean, seed, run,
                             cycle, iter, n_accept, accepted, timer, s)
           : SMC_E_UNSUPPORTED;
}

smc_status launch_loglik(const DevModel &m, int64_t P, const double *theta, int64_t t,
                         double *out, void *state_out, hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->loglik(m, P, theta, t, out, state_out, s) : SMC_E_UNSUPPORTED;
}

size_t adjoint_ckpt_bytes(const DevModel &m, int64_t P, int64_t t) {
  const ModelOps *o = ops_for(m);
  return o ? o->ckpt_bytes(m, P, t) : 0;
}

smc_status launch_loglik_backward(const DevModel &m, int64_t P, const double *theta, int64_t t,
                                  const double *dloglik, double *dtheta, void *ckpt,
                                  hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->loglik_backward(m, P, theta, t, dloglik, dtheta, ckpt, s) : SMC_E_UNSUPPORTED;
}

smc_status launch_grad_post(const DevModel &m, int64_t P, const double *theta, int64_t t,
                            double *grad, void *ckpt, hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->grad_post(m, P, theta, t, grad, ckpt, s) : SMC_E_UNSUPPORTED;
}

smc_status launch_mutate_mala(const DevModel &m, int64_t P, int64_t t, double *theta,
                              double *logprior, double *loglik, void *state, double *grad,
                              const double *hchol, uint64_t seed, uint64_t run, uint64_t cycle,
                              uint64_t iter, int64_t *n_accept, uint8_t *accepted, void *ckpt,
                              hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->mutate_mala(m, P, t, theta, logprior, loglik, state, grad, hchol, seed, run,
                            cycle, iter, n_accept, accepted, ckpt, s)
           : SMC_E_UNSUPPORTED;
}

int32_t num_test_fns(const DevModel &m, int32_t which) {
  const ModelOps *o = ops_for(m);
  return o ? o->num_tests(which) : -1;
}

smc_status launch_test_fns(const DevModel &m, int64_t P, const double *theta, const void *state,
                           int64_t t, int32_t which, double *out, hipStream_t s) {
  const ModelOps *o = ops_for(m);
  return o ? o->test_fns(m, P, theta, state, t, which, out, s) : SMC_E_UNSUPPORTED;
}

// ------------------------------------------------- model-independent ones --
int64_t rss_slice_doubles(int64_t P) {
  return P <= (int64_t)kRssRegs * kRssBlock ? 0
                                            : kMaxChunk * 3 * ((P + kRssSlice - 1) / kRssSlice);
}

smc_status launch_rss_cols(const double *W, int64_t P, int64_t ncols, double *rss,
                           hipStream_t s, const int32_t *ncols_dev) {
  if (ncols <= 0) return SMC_OK;
  if (ncols > kMaxChunk)
    return set_error(SMC_E_INVALID_ARG, "RSS of %lld columns", (long long)ncols);
  if (P <= (int64_t)kRssRegs * kRssBlock) {
    // a device-driven chunk: up to ncols columns, a block per column up to a
    // few per CU
    const unsigned grid = (unsigned)(ncols_dev ? std::min<int64_t>(ncols, 512) : ncols);
    hipLaunchKernelGGL(k_rss_cols, dim3(grid), dim3(kRssBlock), 0, s, W, P, rss, (int32_t)ncols,
                       ncols_dev);
    return launch_status("correct/rss");
  }
  const int64_t S = (P + kRssSlice - 1) / kRssSlice;
  if (S * ncols > INT32_MAX)
    return set_error(SMC_E_UNSUPPORTED, "RSS of %lld slices", (long long)(S * ncols));
  double *part = rss + kMaxChunk;  // the slices' sums follow the RSS values
  const unsigned grid =
      (unsigned)(ncols_dev ? std::min<int64_t>(ncols * S, 2048) : ncols * S);
  hipLaunchKernelGGL(k_rss_slices, dim3(grid), dim3(kRssBlock), 0, s, W, P, (int32_t)S, part,
                     (int32_t)ncols, ncols_dev);
  smc_status st = launch_status("correct/rss slices");
  if (st) return st;
  hipLaunchKernelGGL(k_rss_merge, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s, part, P,
                     (int32_t)S, rss, (int32_t)ncols, ncols_dev);
  return launch_status("correct/rss merge");
}

smc_status launch_rss_scan(const double *trip, int64_t P, int64_t ncols, double *rss,
                           hipStream_t s, const int32_t *ncols_dev) {
  if (ncols <= 0) return SMC_OK;
  if (ncols > kMaxChunk)
    return set_error(SMC_E_INVALID_ARG, "RSS of %lld dates", (long long)ncols);
  const int64_t nw = (P + 63) / 64;
  if (nw > INT32_MAX) return set_error(SMC_E_UNSUPPORTED, "%lld waves", (long long)nw);
  const unsigned grid = (unsigned)(ncols_dev ? std::min<int64_t>(ncols, 1024) : ncols);
  hipLaunchKernelGGL(k_rss_scan, dim3(grid), dim3(256), 0, s, trip, P, (int32_t)nw, rss,
                     (int32_t)ncols, ncols_dev);
  return launch_status("correct/rss");
}

smc_status launch_find_stop(const double *rss, int64_t nc, int64_t t, int64_t t1,
                            int64_t check_every, int64_t t_max, double rss_min, StopInfo *out,
                            hipStream_t s, DecisionSlot *host_slot, uint32_t seq,
                            const int32_t *flags, CycleDyn *cyc) {
  if (!cyc && (nc < 1 || nc > kMaxChunk))
    return set_error(SMC_E_INVALID_ARG, "stop search over %lld columns", (long long)nc);
  hipLaunchKernelGGL(k_find_stop, dim3(1), dim3(64), 0, s, rss, (int32_t)nc, t, t1, check_every,
                     t_max, rss_min, out, host_slot, seq, flags, cyc);
  return launch_status("correct/find_stop");
}

smc_status launch_cycle_init(CycleDyn *c, const CycleDyn &init, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, s, c, init);
  return launch_status("cycle/init");
}

smc_status launch_cycle_end(CycleDyn *c, int64_t *t_end, int32_t *r_rec, double *rss_rec,
                            const int32_t *flags, uint32_t *host, const AccSink &acc,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_end, dim3(1), dim3(64), 0, s, c, t_end, r_rec, rss_rec, flags, host,
                     acc);
  return launch_status("cycle/end");
}

__global__ void k_acc_flush(AccSink acc, int64_t P) { acc_flush(acc, P); }

smc_status launch_acc_flush(const AccSink &acc, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_acc_flush, dim3(1), dim3(64), 0, s, acc, P);
  return launch_status("accept counts");
}

smc_status launch_phase_init(CycleDyn *c, const CycleDyn &init, hipStream_t s) {
  hipLaunchKernelGGL(k_phase_init, dim3(1), dim3(64), 0, s, c, init);
  return launch_status("correct/phase init");
}

smc_status launch_phase_step(CycleDyn *c, hipStream_t s) {
  hipLaunchKernelGGL(k_phase_step, dim3(1), dim3(64), 0, s, c);
  return launch_status("correct/phase step");
}

smc_status launch_phase_out(const CycleDyn *c, const double *rss_src, int64_t t_fixed,
                            int64_t *t_to, double *rss, hipStream_t s) {
  hipLaunchKernelGGL(k_phase_out, dim3(1), dim3(64), 0, s, c, rss_src, t_fixed, t_to, rss);
  return launch_status("correct/phase out");
}

smc_status launch_group_logwbar(const double *logw, int32_t J, int32_t N, double *out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_group_logwbar, dim3(J), dim3(kSBlock), 0, s, logw, N, out);
  return launch_status("correct/group_logwbar");
}

smc_status launch_resample(const double *logw, int32_t J, int32_t N, int32_t scheme,
                           uint64_t seed, uint64_t run, uint64_t cycle, int32_t *anc,
                           double *cum_ws, int32_t *flags, int32_t d, int32_t S, int32_t st_bytes,
                           double *theta, double *logprior, double *loglik, void *state,
                           double *grad, double *tmp, hipStream_t s, const int32_t *go,
                           double *group_logwbar, const CycleDyn *cyc) {
  const int64_t P = (int64_t)J * N;
  GatherArgs g{anc, P, d, S, st_bytes, grad != nullptr ? 1 : 0, theta, logprior, loglik, grad,
               state, tmp};
  if (N > kResampleMaxN)
    return set_error(SMC_E_UNSUPPORTED, "resampling needs N <= %d", kResampleMaxN);
  const size_t lds = N <= kCumLdsMax ? (size_t)N * (sizeof(double) + 2 * sizeof(int32_t)) +
                                           kGatherLdsBytes
                                     : (size_t)N * sizeof(int32_t);
  hipLaunchKernelGGL(k_resample, dim3(J), dim3(kSBlock), lds, s, logw, N, scheme, seed, run, cycle,
                     anc, cum_ws, flags, g, go, group_logwbar, cyc);
  return launch_status("resample");
}

// Blocks of four waves (their loads pipelined), about 128 of them, so each
// wave's chain of loads is short (four batches of 32 particles at 65,536
// particles); k_mom_sum then adds the partial matrices entry by entry (a
// quarter of them per wave, the quarters in wave order) and the final step
// reads one matrix.  Each wave takes `chunk` particles (a multiple of 32).
// The batched moments use the same partition and order, so a run gives the
// same sums alone or in a batch.
void moment_partition(int64_t P, int32_t d, int64_t &chunk, int64_t &nb) {
  (void)d;
  const int64_t target = 128;
  chunk = (P + 4 * target - 1) / (4 * target);
  chunk = ((chunk + 31) / 32) * 32;
  nb = (P + 4 * chunk - 1) / (4 * chunk);
}

smc_status launch_moments(const MomArgs &a, hipStream_t s) {
  if (a.d + 1 > kDMax) return set_error(SMC_E_UNSUPPORTED, "moments need d < %d", kDMax);
  int64_t chunk = 0, nb = 0;
  moment_partition(a.P, a.d, chunk, nb);
  if (nb > kMomBlocks)
    return set_error(SMC_E_WORKSPACE, "moments need %lld partials", (long long)nb);
  const int64_t xb = a.acc.pending ? 1 : 0;  // the accept-count flush
  const int n = a.d + 1 <= 16 ? 256 : 1024;  // entries of a partial matrix
  if (n == 256) {
    hipLaunchKernelGGL(k_mom_partial<16>, dim3((unsigned)(nb + xb)), dim3(kBlock), 0, s, a.theta,
                       a.P, a.d, chunk, a.part, a.cyc, a.slot, a.acc);
  } else {
    hipLaunchKernelGGL(k_mom_partial<32>, dim3((unsigned)(nb + xb)), dim3(kBlock), 0, s, a.theta,
                       a.P, a.d, chunk, a.part, a.cyc, a.slot, a.acc);
  }
  smc_status st = launch_status("particle_moments/partial");
  if (st) return st;
  // sums into the slot after the partials, then the final block reads them
  double *sums = a.part + nb * n;
  hipLaunchKernelGGL(k_mom_sum, dim3(n / 64), dim3(256), 0, s, a.part, (int32_t)nb, n, sums,
                     a.cyc, a.slot);
  if ((st = launch_status("particle_moments/sum"))) return st;
  MomArgs f = a;
  f.part = sums;
  if (n == 256)
    hipLaunchKernelGGL(k_mom_final<16>, dim3(1), dim3(256), 0, s, f, 1);
  else
    hipLaunchKernelGGL(k_mom_final<32>, dim3(1), dim3(1024), 0, s, f, 1);
  return launch_status("particle_moments/final");
}

smc_status launch_moment_partials(const MomArgs &a, const double **part, int64_t &nb,
                                  hipStream_t s) {
  if (a.d + 1 > kDMax) return set_error(SMC_E_UNSUPPORTED, "moments need d < %d", kDMax);
  int64_t chunk = 0;
  moment_partition(a.P, a.d, chunk, nb);
  if (nb > kMomBlocks)
    return set_error(SMC_E_WORKSPACE, "moments need %lld partials", (long long)nb);
  const int64_t xb = a.acc.pending ? 1 : 0;  // the accept-count flush
  const int n = a.d + 1 <= 16 ? 256 : 1024;
  if (n == 256)
    hipLaunchKernelGGL(k_mom_partial<16>, dim3((unsigned)(nb + xb)), dim3(kBlock), 0, s, a.theta,
                       a.P, a.d, chunk, a.part, a.cyc, a.slot, a.acc);
  else
    hipLaunchKernelGGL(k_mom_partial<32>, dim3((unsigned)(nb + xb)), dim3(kBlock), 0, s, a.theta,
                       a.P, a.d, chunk, a.part, a.cyc, a.slot, a.acc);
  smc_status st = launch_status("particle_moments/partial");
  if (st) return st;
  // summed into the slot after the partials, as launch_moments does
  double *sums = a.part + nb * n;
  hipLaunchKernelGGL(k_mom_sum, dim3(n / 64), dim3(256), 0, s, a.part, (int32_t)nb, n, sums,
                     a.cyc, a.slot);
  *part = sums;
  nb = 1;
  return launch_status("particle_moments/sum");
}

smc_status launch_adapt(const int64_t *n_accept, int64_t P, int32_t target_permille,
                        int32_t *mh, hipStream_t s) {
  hipLaunchKernelGGL(k_adapt, dim3(1), dim3(64), 0, s, n_accept, P, target_permille, mh);
  return launch_status("adapt_scale");
}

smc_status launch_rne(const double *theta, int32_t J, int32_t N, int32_t d, double *part,
                      double *rne, hipStream_t s) {
  const int64_t P = (int64_t)J * N;
  hipLaunchKernelGGL(k_rne_group, dim3(J), dim3(kBlock), 0, s, theta, P, N, d, part);
  smc_status st = launch_status("rne/group");
  if (st) return st;
  hipLaunchKernelGGL(k_rne_final, dim3(1), dim3(64), 0, s, part, J, N, d, rne);
  return launch_status("rne/final");
}

smc_status launch_report(const double *g, int32_t J, int32_t N, int32_t G, double *part,
                         double *out, double *rne_mean, hipStream_t s) {
  if (G < 1 || G > kDMax) return set_error(SMC_E_UNSUPPORTED, "report of %d functions", G);
  const int64_t P = (int64_t)J * N;
  hipLaunchKernelGGL(k_rne_group, dim3(J), dim3(kBlock), 0, s, g, P, N, G, part);
  smc_status st = launch_status("report/group");
  if (st) return st;
  hipLaunchKernelGGL(k_report_final, dim3(1), dim3(64), 0, s, part, J, N, G, out, rne_mean);
  return launch_status("report/final");
}

smc_status launch_log_ml(int32_t L, int32_t J, const double *g, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_log_ml, dim3(1), dim3(kBlock), 0, s, L, J, g, out);
  return launch_status("log_ml");
}

}  // namespace smc
