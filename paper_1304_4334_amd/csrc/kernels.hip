// HIP kernels of the sequential posterior simulator for gfx950 (CDNA4) and
// their host-side launchers.
//
// Geometry: the likelihood kernels map one particle to one lane and launch
// 64-thread blocks (one wave each), so a population spreads over as many
// compute units as it has waves; observations are wave-uniform and reach the
// lanes through scalar loads into SGPRs.  The bandwidth-shaped kernels
// (reductions, resampling, gathers) use 256-thread blocks.  Every reduction
// combines in a fixed order, so results do not depend on timing.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "adjoint.h"
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
// t0+1..t1 and record the running log weight at every check date, without
// committing anything.
template <class M>
__global__ void __launch_bounds__(64) k_cscan(DevModel dm, int64_t P, const double *theta,
                                              const void *state, const double *logw, int64_t t0,
                                              int64_t t1, int64_t check_every, int64_t t_max,
                                              int32_t zero_first, double *W) {
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
  for (int k = 0; k < SR; ++k) st[k] = (k < StoredS<M>::value) ? typed<R>(state)[k * P + p] : (R)0;
  double lw = zero_first ? 0.0 : logw[p];
  int64_t col = 0;
  for (int64_t s = t0 + 1; s <= t1; ++s) {
    double lp = Eval<M>::advance(dm, par, st, s - 1, s);
    if (isnan(lp)) lp = -INFINITY;
    lw += lp;
    if (s % check_every == 0 || s == t_max) {
      W[col * P + p] = lw;
      ++col;
    }
  }
}

// Commit: advance from t0 to t1, adding the log densities to logw and loglik.
template <class M>
__global__ void __launch_bounds__(64) k_ccommit(DevModel dm, int64_t P, const double *theta,
                                                void *state, double *logw, double *loglik,
                                                int64_t t0, int64_t t1, int32_t zero_first) {
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  if (p >= P) return;
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
  double lp = Eval<M>::advance(dm, par, st, t0, t1);
  if (isnan(lp)) lp = -INFINITY;
  logw[p] = (zero_first ? 0.0 : logw[p]) + lp;
  loglik[p] += lp;
#pragma unroll
  for (int k = 0; k < SS; ++k) typed<R>(state)[k * P + p] = st[k];
}

// RSS of each recorded column: (sum e)^2 / (P sum e^2), e = exp(w - max w).
// One block of 1024 threads per column, one pass: each thread keeps a running
// maximum m with s1 = sum exp(w - m), s2 = sum exp(2(w - m)), rescaled when
// m grows; the block merges the triples the same way in a fixed order.
struct Lse3 {
  double m, s1, s2;
};
__device__ __forceinline__ Lse3 lse3_merge(Lse3 a, Lse3 b) {
  const double m = fmax(a.m, b.m);
  if (!(m > -INFINITY)) return Lse3{m, 0.0, 0.0};
  const double ea = exp(a.m - m), eb = exp(b.m - m);
  return Lse3{m, a.s1 * ea + b.s1 * eb, a.s2 * ea * ea + b.s2 * eb * eb};
}

constexpr int kRssBlock = 1024;

__global__ void __launch_bounds__(1024) k_rss_cols(const double *W, int64_t P, double *rss) {
  __shared__ Lse3 sh[kRssBlock / 64];
  const double *w = W + blockIdx.x * P;
  Lse3 acc{-INFINITY, 0.0, 0.0};
  for (int64_t p0 = threadIdx.x; p0 < P; p0 += 8 * kRssBlock) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = p0 + (int64_t)u * kRssBlock;
      v[u] = p < P ? w[p] : -INFINITY;
    }
    double m = v[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) m = fmax(m, v[u]);
    Lse3 c{m, 0.0, 0.0};
    if (m > -INFINITY) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double e = exp(v[u] - m);
        c.s1 += e;
        c.s2 = fma(e, e, c.s2);
      }
    }
    acc = lse3_merge(acc, c);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Lse3 o{__shfl_xor(acc.m, off, 64), __shfl_xor(acc.s1, off, 64), __shfl_xor(acc.s2, off, 64)};
    acc = lse3_merge(acc, o);
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Lse3 t = sh[0];
    for (int q = 1; q < kRssBlock / 64; ++q) t = lse3_merge(t, sh[q]);
    rss[blockIdx.x] = (t.m > -INFINITY) ? t.s1 * t.s1 / ((double)P * t.s2) : 0.0;
  }
}

// log wbar_j = log(N^-1 sum_n exp(logw_jn)) per group (Section 4.2).
__global__ void __launch_bounds__(256) k_group_logwbar(const double *logw, int32_t N,
                                                       double *out) {
  __shared__ double sh[4];
  const double *w = logw + (int64_t)blockIdx.x * N;
  double mx = -INFINITY;
  for (int n = threadIdx.x; n < N; n += kBlock) mx = fmax(mx, w[n]);
  mx = block_reduce<OpMax<double>>(mx, sh);
  double s = 0.0;
  if (mx > -INFINITY)
    for (int n = threadIdx.x; n < N; n += kBlock) s += exp(w[n] - mx);
  s = block_reduce<OpSum<double>>(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = (mx > -INFINITY) ? mx + log(s / (double)N) : -INFINITY;
}

// ------------------------------------------------------------ S phase (a3) --
// One block per group.  Counts live in LDS (dynamic, N int32); the running
// residual sums in the workspace.  Residual: floor(N W_n) copies, then the
// remaining draws from the residuals; multinomial: N draws from W_n;
// stratified / systematic (Section 3.3's experimental schemes): the k-th of N
// draws at (k + U_k)/N, respectively (k + U)/N, of the running sum.
struct GatherArgs {
  const int32_t *anc;
  int64_t P;
  int32_t d, S, st_bytes, has_grad;
  double *theta, *logprior, *loglik, *grad;
  void *state;
  double *tmp;  // [2d + S + 2][P]
};

__global__ void __launch_bounds__(256) k_resample(const double *logw, int32_t N, int32_t scheme,
                                                  uint64_t seed, uint64_t run, uint64_t cycle,
                                                  int32_t *anc, double *cum_ws, int32_t *flags,
                                                  GatherArgs g) {
  extern __shared__ int32_t cnt[];
  __shared__ double shd[kBlock];
  __shared__ int64_t shi[kBlock];
  const int j = blockIdx.x;
  const int64_t base = (int64_t)j * N;
  const double *lw = logw + base;
  double *cum = cum_ws + base;
  const int tid = threadIdx.x;

  double mx = -INFINITY;
  for (int n = tid; n < N; n += kBlock) mx = fmax(mx, lw[n]);
  mx = block_reduce<OpMax<double>>(mx, shd);
  if (!(mx > -INFINITY)) {
    for (int n = tid; n < N; n += kBlock) anc[base + n] = (int32_t)(base + n);
    if (tid == 0) atomicOr(flags, SMC_FLAG_DEAD_GROUP);
    return;
  }
  double se = 0.0;
  for (int n = tid; n < N; n += kBlock) se += exp(lw[n] - mx);
  se = block_reduce<OpSum<double>>(se, shd);

  // Thread-contiguous chunks for the scans.
  const int m = (N + kBlock - 1) / kBlock;
  const int lo = min(tid * m, N), hi = min(lo + m, N);
  double rsum = 0.0;
  int64_t csum = 0;
  for (int n = lo; n < hi; ++n) {
    const double nw = ((double)N * exp(lw[n] - mx)) / se;  // N W_n
    const double c = (scheme == SMC_RESAMPLE_RESIDUAL) ? floor(nw) : 0.0;
    rsum += nw - c;
    cum[n] = rsum;
    cnt[n] = (int32_t)c;
    csum += (int64_t)c;
  }
  double rtot;
  const double roff = block_inclusive_scan<double>(rsum, shd, rtot) - rsum;
  for (int n = lo; n < hi; ++n) cum[n] += roff;
  int64_t ctot;
  (void)block_inclusive_scan<int64_t>(csum, shi, ctot);
  __syncthreads();
  const double total = cum[N - 1];
  const int64_t R = (int64_t)N - ctot;
  const double u_sys = u01_co(draw4(seed, run, (uint64_t)j, cycle, 0, kResample).x0);
  for (int64_t k = tid; k < R; k += kBlock) {
    const U64x4 w = draw4(seed, run, (uint64_t)j, cycle, (uint64_t)(k >> 2), kResample);
    const uint64_t x = (k & 3) == 0 ? w.x0 : (k & 3) == 1 ? w.x1 : (k & 3) == 2 ? w.x2 : w.x3;
    double u = u01_co(x);
    if (scheme == SMC_RESAMPLE_STRATIFIED) u = ((double)k + u) / (double)N;
    else if (scheme == SMC_RESAMPLE_SYSTEMATIC) u = ((double)k + u_sys) / (double)N;
    const double target = u * total;
    int a_lo = 0, a_hi = N;  // first n with cum[n] > target
    while (a_lo < a_hi) {
      const int mid = (a_lo + a_hi) >> 1;
      if (cum[mid] > target) a_hi = mid;
      else a_lo = mid + 1;
    }
    int a = a_lo;
    if (a >= N) {
      a = N - 1;
      while (a > 0 && !(cum[a] > cum[a - 1])) --a;
    }
    atomicAdd(&cnt[a], 1);
  }
  __syncthreads();
  int64_t my = 0;
  for (int n = lo; n < hi; ++n) my += cnt[n];
  int64_t tot2;
  int64_t pos = block_inclusive_scan<int64_t>(my, shi, tot2) - my;
  for (int n = lo; n < hi; ++n)
    for (int c = 0; c < cnt[n] && pos < N; ++c) anc[base + pos++] = (int32_t)(base + n);
  __syncthreads();
  // Replace the group's particles by their ancestors (all inside this
  // group): copy the ancestors' values to the workspace, then back.
  const int64_t P = g.P;
  for (int n = tid; n < N; n += kBlock) {
    const int64_t p = base + n;
    const int64_t a = anc[p];
    int r = 0;
    for (int i = 0; i < g.d; ++i, ++r) g.tmp[r * P + p] = g.theta[i * P + a];
    g.tmp[r++ * P + p] = g.logprior[a];
    g.tmp[r++ * P + p] = g.loglik[a];
    for (int k = 0; k < g.S; ++k, ++r)
      g.tmp[r * P + p] = g.st_bytes == 8 ? typed<double>(g.state)[k * P + a]
                                         : (double)typed<float>(g.state)[k * P + a];
    if (g.has_grad)
      for (int i = 0; i < g.d; ++i, ++r) g.tmp[r * P + p] = g.grad[i * P + a];
  }
  __syncthreads();
  for (int n = tid; n < N; n += kBlock) {
    const int64_t p = base + n;
    int r = 0;
    for (int i = 0; i < g.d; ++i, ++r) g.theta[i * P + p] = g.tmp[r * P + p];
    g.logprior[p] = g.tmp[r++ * P + p];
    g.loglik[p] = g.tmp[r++ * P + p];
    for (int k = 0; k < g.S; ++k, ++r) {
      if (g.st_bytes == 8) typed<double>(g.state)[k * P + p] = g.tmp[r * P + p];
      else typed<float>(g.state)[k * P + p] = (float)g.tmp[r * P + p];
    }
    if (g.has_grad)
      for (int i = 0; i < g.d; ++i, ++r) g.grad[i * P + p] = g.tmp[r * P + p];
  }
}

// ----------------------------------------------- particle moments (a4) ----
// Pass 1: every wave accumulates sum_p x_p x_p' on the matrix cores with
// x_p = (theta_p - s, 1, 0, ...) padded to 16 (s = particle 0, a shift that
// keeps the one-pass sums well conditioned; the constant slot d carries the
// first moments and the count).  v_mfma_f64_16x16x4f64 takes four particles
// per instruction.  Operand layout (measured on gfx950): lane l supplies
// element (row l%16, k = l/16) of A and (k = l/16, col l%16) of B, so
// A = B' = the 16x4 block of shifted particles; accumulator register r of
// lane l holds element (4r + l/16, l%16) of the 16x16 result.  Each block
// writes one partial matrix.
__global__ void __launch_bounds__(256) k_mom_partial(const double *theta, int64_t P, int32_t d,
                                                     int64_t chunk, double *part) {
  __shared__ double red[4][256];
  typedef double double4v __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int i = l & 15, k = l >> 4;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + wv) * chunk;
  const int64_t p1 = min(P, p0 + chunk);
  const int ir = i < d ? i : 0;  // a valid row to load from when i >= d
  const double si = theta[(int64_t)ir * P];
  double4v acc = {0.0, 0.0, 0.0, 0.0};
  // Eight MFMA steps per batch with all loads issued first (addresses are
  // clamped into the wave's range and masked afterwards).
  for (int64_t q0 = p0; q0 < p1; q0 += 32) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = q0 + 4 * u + k;
      const int64_t pc = p < p1 ? p : p1 - 1;
      x[u] = theta[(int64_t)ir * P + pc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = q0 + 4 * u + k;
      const double v = (i < d) ? x[u] - si : (i == d ? 1.0 : 0.0);
      const double xm = p < p1 ? v : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xm, xm, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv][(4 * r + k) * 16 + i] = acc[r];
  __syncthreads();
  part[blockIdx.x * 256 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// Pass 2 (one block): add the partial matrices in block order, optionally
// apply the step-size rule to mh, form the mean and V (divisor P - 1),
// factor V = L L' and write h L.  A variance that is not positive definite
// raises the flag and yields h L = 0.
__global__ void __launch_bounds__(256) k_mom_final(MomArgs a, int32_t nb) {
  __shared__ double Ms[256];
  __shared__ double Ls[kDMax * kDMax];
  __shared__ double sh_h;
  __shared__ int sh_ok;
  const int tid = threadIdx.x;
  const int d = a.d;
  const int64_t P = a.P;
  double sum = 0.0;
#pragma unroll 16
  for (int b = 0; b < nb; ++b) sum += a.part[b * 256 + tid];
  Ms[tid] = sum;
  if (tid == 0) {
    int32_t m = *a.mh;
    if (a.mh_reset > 0) {
      m = a.mh_reset;
    } else if (a.prev_nacc) {
      m += ((*a.prev_nacc) * 1000 > (int64_t)a.target_permille * P) ? 1 : -1;
      m = m < 1 ? 1 : (m > 10 ? 10 : m);
    }
    *a.mh = m;
    sh_h = (double)m / 10.0;
    sh_ok = 1;
  }
  __syncthreads();
  const double invP = 1.0 / (double)P;
  const int r = tid >> 4, c = tid & 15;
  double v = 0.0;
  if (r < d && c < d) {
    v = (Ms[r * 16 + c] - Ms[r * 16 + d] * Ms[c * 16 + d] * invP) / (double)(P - 1);
    if (a.cov_out) a.cov_out[r * d + c] = v;
  }
  if (a.mean_out && tid < d) a.mean_out[tid] = a.theta[(int64_t)tid * P] + Ms[tid * 16 + d] * invP;
  __syncthreads();
  if (r < d && c < d) Ms[r * 16 + c] = v;
  Ls[tid] = 0.0;
  __syncthreads();
  // Cholesky, column by column: the diagonal by one thread, the column below
  // it by one thread per row.
  for (int col = 0; col < d; ++col) {
    if (tid == 0) {
      double q = Ms[col * 16 + col];
      for (int t = 0; t < col; ++t) q -= Ls[col * kDMax + t] * Ls[col * kDMax + t];
      if (q > 0.0 && sh_ok) Ls[col * kDMax + col] = sqrt(q);
      else sh_ok = 0;
    }
    __syncthreads();
    if (sh_ok && tid > col && tid < d) {
      double q = Ms[tid * 16 + col];
      for (int t = 0; t < col; ++t) q -= Ls[tid * kDMax + t] * Ls[col * kDMax + t];
      Ls[tid * kDMax + col] = q / Ls[col * kDMax + col];
    }
    __syncthreads();
  }
  if (r < d && c < d) a.hchol[r * d + c] = (sh_ok && c <= r) ? sh_h * Ls[r * kDMax + c] : 0.0;
  if (tid == 0 && !sh_ok) atomicOr(a.flags, SMC_FLAG_NOT_PD);
}

// ------------------------------------------------------------ M phase (a5) --
template <class M>
__global__ void __launch_bounds__(64) k_mutate_rw(DevModel dm, int64_t P, int64_t t, double *theta,
                                                  double *logprior, double *loglik, void *state,
                                                  const double *__restrict__ hchol, uint64_t seed,
                                                  uint64_t run, uint64_t cycle, uint64_t iter,
                                                  unsigned long long *n_accept, uint8_t *accepted) {
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
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k <= i; ++k) s = fma(hchol[i * D + k], z[k], s);
      pr[i] = th[i] + s;
    }
    const double lp1 = M::logprior(pr);
    R st[SR];
#pragma unroll
    for (int k = 0; k < SR; ++k) st[k] = (R)0;
    double ll1 = -INFINITY;
    if (lp1 > -INFINITY) {
      const auto par = M::params(pr);
      ll1 = Eval<M>::advance(dm, par, st, 0, t);
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
  const unsigned long long mask = __ballot(acc);
  if (threadIdx.x == 0 && mask) atomicAdd(n_accept, (unsigned long long)__popcll(mask));
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

// log wbar, its delta-method NSE and log wtilde from group_logwbar[L][J].
__global__ void k_log_ml(int32_t L, int32_t J, const double *g, double *out) {
  if (threadIdx.x != 0) return;
  double mx = -INFINITY;
  for (int j = 0; j < J; ++j) {
    double s = 0.0;
    for (int l = 0; l < L; ++l) s += g[(int64_t)l * J + j];
    mx = fmax(mx, s);
  }
  double rbar = 0.0;
  for (int j = 0; j < J; ++j) {
    double s = 0.0;
    for (int l = 0; l < L; ++l) s += g[(int64_t)l * J + j];
    rbar += exp(s - mx);
  }
  rbar /= (double)J;
  double ss = 0.0;
  for (int j = 0; j < J; ++j) {
    double s = 0.0;
    for (int l = 0; l < L; ++l) s += g[(int64_t)l * J + j];
    const double e = exp(s - mx) - rbar;
    ss += e * e;
  }
  double lt = 0.0;
  for (int l = 0; l < L; ++l) {
    double m = -INFINITY;
    for (int j = 0; j < J; ++j) m = fmax(m, g[(int64_t)l * J + j]);
    double s = 0.0;
    for (int j = 0; j < J; ++j) s += exp(g[(int64_t)l * J + j] - m);
    lt += (m > -INFINITY) ? m + log(s / (double)J) : -INFINITY;
  }
  out[0] = mx + log(rbar);
  out[1] = sqrt(ss / ((double)J * (J - 1))) / rbar;
  out[2] = lt;
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

// One preconditioned Langevin (MALA) Metropolis iteration: proposal mean
// theta + (1/2)(hL)(hL)' grad, noise hL z; the acceptance test adds
// log q(theta | theta') - log q(theta' | theta) = -|w|^2/2 + |z|^2/2 with
// (hL) w = theta - theta' - (1/2)(hL)(hL)' grad'.
template <class M>
__global__ void __launch_bounds__(64) k_mutate_mala(DevModel dm, int64_t P, int64_t t, double *theta,
                                                    double *logprior, double *loglik, void *state,
                                                    double *grad, const double *__restrict__ hchol,
                                                    uint64_t seed, uint64_t run, uint64_t cycle,
                                                    uint64_t iter, unsigned long long *n_accept,
                                                    uint8_t *accepted, void *ckpt) {
  extern __shared__ double lds_dyn[];
  constexpr int D = M::D;
  using R = typename M::R;
  constexpr int SR = Eval<M>::SR;
  constexpr int SS = StoredS<M>::value;
  const int64_t p = blockIdx.x * 64ll + threadIdx.x;
  int acc = 0;
  if (p < P) {
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
      ll1 = ll_and_grad<M>(dm, pr, t, ckpt, P, p, lds_dyn, 1.0, g1, stv);
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
      const double delta =
          (lp1 + ll1) - (logprior[p] + loglik[p]) + (-0.5 * ww + 0.5 * zz);
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
    if (accepted) accepted[p] = (uint8_t)acc;
  }
  const unsigned long long mask = __ballot(acc);
  if (threadIdx.x == 0 && mask) atomicAdd(n_accept, (unsigned long long)__popcll(mask));
}

// ============================================================ launchers ====

template <class F>
smc_status dispatch(const DevModel &m, F &&f) {
  if (m.kind == SMC_MODEL_LINREG) {
    switch (m.nreg) {
      case 1: return f(Tag<Linreg<1>>{});
      case 2: return f(Tag<Linreg<2>>{});
      case 3: return f(Tag<Linreg<3>>{});
      case 4: return f(Tag<Linreg<4>>{});
      default: return set_error(SMC_E_UNSUPPORTED, "regression with %d regressors", m.nreg);
    }
  }
  const bool t = m.shock == SMC_SHOCK_STUDENT_T;
  if (m.prec == SMC_FP64) {
    if (m.K == 1) return t ? f(Tag<Egarch<1, 1, double>>{}) : f(Tag<Egarch<1, 0, double>>{});
    if (m.K == 2) return t ? f(Tag<Egarch<2, 1, double>>{}) : f(Tag<Egarch<2, 0, double>>{});
  } else {
    if (m.K == 1) return t ? f(Tag<Egarch<1, 1, float>>{}) : f(Tag<Egarch<1, 0, float>>{});
    if (m.K == 2) return t ? f(Tag<Egarch<2, 1, float>>{}) : f(Tag<Egarch<2, 0, float>>{});
  }
  return set_error(SMC_E_UNSUPPORTED, "EGARCH with K=%d", m.K);
}

smc_status launch_init(const DevModel &m, int64_t P, uint64_t seed, uint64_t run, double *theta,
                       double *logprior, double *loglik, void *state, double *logw,
                       hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_init<M>, grid_for(P, 64), dim3(64), 0, s, m, P, seed, run, theta,
                       logprior, loglik, state, logw);
    return launch_status("init_from_prior");
  });
}

smc_status launch_cscan(const DevModel &m, int64_t P, const double *theta, const void *state,
                        const double *logw, int64_t t0, int64_t t1, int64_t check_every,
                        int64_t t_max, bool zero_first, double *W, hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_cscan<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, state, logw, t0,
                       t1, check_every, t_max, (int32_t)zero_first, W);
    return launch_status("correct/scan");
  });
}

smc_status launch_ccommit(const DevModel &m, int64_t P, const double *theta, void *state,
                          double *logw, double *loglik, int64_t t0, int64_t t1, bool zero_first,
                          hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_ccommit<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, state, logw,
                       loglik, t0, t1, (int32_t)zero_first);
    return launch_status("correct/commit");
  });
}

smc_status launch_rss_cols(const double *W, int64_t P, int64_t ncols, double *rss,
                           hipStream_t s) {
  if (ncols <= 0) return SMC_OK;
  hipLaunchKernelGGL(k_rss_cols, dim3((unsigned)ncols), dim3(kRssBlock), 0, s, W, P, rss);
  return launch_status("correct/rss");
}

smc_status launch_group_logwbar(const double *logw, int32_t J, int32_t N, double *out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_group_logwbar, dim3(J), dim3(kBlock), 0, s, logw, N, out);
  return launch_status("correct/group_logwbar");
}

smc_status launch_resample(const double *logw, int32_t J, int32_t N, int32_t scheme,
                           uint64_t seed, uint64_t run, uint64_t cycle, int32_t *anc,
                           double *cum_ws, int32_t *flags, int32_t d, int32_t S, int32_t st_bytes,
                           double *theta, double *logprior, double *loglik, void *state,
                           double *grad, double *tmp, hipStream_t s) {
  const int64_t P = (int64_t)J * N;
  GatherArgs g{anc, P, d, S, st_bytes, grad != nullptr ? 1 : 0, theta, logprior, loglik, grad,
               state, tmp};
  hipLaunchKernelGGL(k_resample, dim3(J), dim3(kBlock), (size_t)N * sizeof(int32_t), s, logw, N,
                     scheme, seed, run, cycle, anc, cum_ws, flags, g);
  return launch_status("resample");
}

smc_status launch_moments(const MomArgs &a, hipStream_t s) {
  if (a.d + 1 > kDMax) return set_error(SMC_E_UNSUPPORTED, "moments need d < 16");
  // About 64 particles per wave (two load batches); at most kMomBlocks
  // blocks of four waves.
  const int64_t waves = std::max<int64_t>(1, (a.P + 63) / 64);
  int64_t nb = std::min<int64_t>(kMomBlocks, (waves + 3) / 4);
  int64_t chunk = (a.P + 4 * nb - 1) / (4 * nb);
  chunk = ((chunk + 31) / 32) * 32;
  nb = (a.P + 4 * chunk - 1) / (4 * chunk);
  hipLaunchKernelGGL(k_mom_partial, dim3((unsigned)nb), dim3(kBlock), 0, s, a.theta, a.P, a.d,
                     chunk, a.part);
  smc_status st = launch_status("particle_moments/partial");
  if (st) return st;
  hipLaunchKernelGGL(k_mom_final, dim3(1), dim3(kBlock), 0, s, a, (int32_t)nb);
  return launch_status("particle_moments/final");
}

smc_status launch_mutate_rw(const DevModel &m, int64_t P, int64_t t, double *theta,
                            double *logprior, double *loglik, void *state, const double *hchol,
                            uint64_t seed, uint64_t run, uint64_t cycle, uint64_t iter,
                            int64_t *n_accept, uint8_t *accepted, hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_mutate_rw<M>, grid_for(P, 64), dim3(64), 0, s, m, P, t, theta, logprior,
                       loglik, state, hchol, seed, run, cycle, iter,
                       reinterpret_cast<unsigned long long *>(n_accept), accepted);
    return launch_status("mutate");
  });
}

smc_status launch_loglik(const DevModel &m, int64_t P, const double *theta, int64_t t,
                         double *out, void *state_out, hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_loglik<M>, grid_for(P, 64), dim3(64), 0, s, m, P, theta, t, out,
                       state_out);
    return launch_status("loglik");
  });
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

smc_status launch_log_ml(int32_t L, int32_t J, const double *g, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_log_ml, dim3(1), dim3(64), 0, s, L, J, g, out);
  return launch_status("log_ml");
}

size_t adjoint_ckpt_bytes(const DevModel &m, int64_t P, int64_t t) {
  size_t out = 0;
  (void)dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    if constexpr (!IsLinreg<M>::value) {
      using A = Adjoint<M>;
      const int64_t ns = (t + A::SEG - 1) / A::SEG;
      out = (size_t)ns * M::K * (size_t)P * sizeof(typename M::R);
    }
    return SMC_OK;
  });
  return out;
}

smc_status launch_loglik_backward(const DevModel &m, int64_t P, const double *theta, int64_t t,
                                  const double *dloglik, double *dtheta, void *ckpt,
                                  hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_loglik_backward<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m,
                       P, theta, t, dloglik, dtheta, ckpt);
    return launch_status("loglik_backward");
  });
}

smc_status launch_grad_post(const DevModel &m, int64_t P, const double *theta, int64_t t,
                            double *grad, void *ckpt, hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_grad_post<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m, P,
                       theta, t, grad, ckpt);
    return launch_status("posterior_grad");
  });
}

smc_status launch_mutate_mala(const DevModel &m, int64_t P, int64_t t, double *theta,
                              double *logprior, double *loglik, void *state, double *grad,
                              const double *hchol, uint64_t seed, uint64_t run, uint64_t cycle,
                              uint64_t iter, int64_t *n_accept, uint8_t *accepted, void *ckpt,
                              hipStream_t s) {
  return dispatch(m, [&](auto tag) {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL(k_mutate_mala<M>, grid_for(P, 64), dim3(64), lds_bytes_of<M>(), s, m, P, t,
                       theta, logprior, loglik, state, grad, hchol, seed, run, cycle, iter,
                       reinterpret_cast<unsigned long long *>(n_accept), accepted, ckpt);
    return launch_status("mutate/mala");
  });
}

}  // namespace smc
