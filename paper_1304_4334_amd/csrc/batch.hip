// Many independent runs advanced together (the batched workload).
//
// At each step of the batch driver (abi.hip) every run is in a C-phase chunk
// or in an M iteration.  The M iterations of all runs go to
//   k_batch_mom_partial  one 256-thread block per (run, particle chunk),
//   k_batch_mom_final    one block per run (h rule, V, Cholesky, h L),
//   k_batch_mutate       one persistent launch: each block takes the next
//                        (run, block of particles) item from a device counter,
//                        items ordered by decreasing cost t_r.
// Static per-run data (arrays, keys, sizes) sits in a device table written
// once per batch call; what changes from step to step (date, cycle,
// iteration, record slots) travels by value in the kernel arguments, so a
// batch with no host decisions (replay) can be captured in a graph.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "batch.h"
#include "chol.h"
#include "model.h"
#include "model_kernels.h"
#include "rng.h"

namespace smc {

namespace {

inline dim3 grid_of(int64_t n) { return dim3((unsigned)n); }

inline smc_status launch_ok(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SMC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return SMC_OK;
}

// Which active run (index into a.dyn, ordered by item offsets) owns item i.
__device__ __forceinline__ int owner(const BatchArgs &a, int32_t i, bool mom) {
  int r = 0;
  for (int q = 1; q < a.n_active; ++q) {
    const int32_t b = mom ? a.dyn[q].mom_begin : a.dyn[q].mut_begin;
    if (i >= b) r = q;
  }
  return r;
}

}  // namespace

__global__ void __launch_bounds__(256) k_batch_mom_partial(BatchArgs a) {
  __shared__ double red[4][256];
  typedef double double4v __attribute__((ext_vector_type(4)));
  const int ri = owner(a, (int32_t)blockIdx.x, true);
  const BatchDyn &dy = a.dyn[ri];
  const BatchStatic &st = a.runs[dy.idx];
  const int lb = (int)blockIdx.x - dy.mom_begin;
  const double *theta = st.theta;
  const int64_t P = st.P;
  const int d = st.d;
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int i = l & 15, k = l >> 4;
  const int64_t p0 = ((int64_t)lb * 4 + wv) * dy.mom_chunk;
  const int64_t p1 = min(P, p0 + dy.mom_chunk);
  const int ir = i < d ? i : 0;
  const double si = theta[(int64_t)ir * P];
  double4v acc = {0.0, 0.0, 0.0, 0.0};
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
  st.part[lb * 256 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

__global__ void __launch_bounds__(256) k_batch_mom_final(BatchArgs a) {
  __shared__ double Ms[256];
  __shared__ double Ls[16 * chol_ld<16>()];
  __shared__ double sh_h;
  const BatchDyn &dy = a.dyn[blockIdx.x];
  const BatchStatic &st = a.runs[dy.idx];
  const int tid = threadIdx.x;
  const int d = st.d;
  const int64_t P = st.P;
  // the partials added as k_mom_sum adds them: four quarters in block order,
  // then the quarters in order; each quarter's loads issued 32 at a time
  const int nb = dy.mom_nb, per = (nb + 3) / 4;
  constexpr int kBatch = 32;
  double q[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int lo = min(nb, w * per), hi = min(nb, lo + per);
    double s = 0.0;
    for (int b0 = lo; b0 < hi; b0 += kBatch) {
      double x[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) x[u] = (b0 + u < hi) ? st.part[(b0 + u) * 256 + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < kBatch; ++u)
        if (b0 + u < hi) s += x[u];
    }
    q[w] = s;
  }
  Ms[tid] = ((q[0] + q[1]) + q[2]) + q[3];
  if (tid == 0) {
    int32_t m = *st.mh;
    if (dy.mh_reset > 0) {
      m = dy.mh_reset;
    } else if (dy.prev_nacc) {
      m += ((*dy.prev_nacc) * 1000 > (int64_t)a.target_permille * P) ? 1 : -1;
      m = m < 1 ? 1 : (m > 10 ? 10 : m);
    }
    *st.mh = m;
    sh_h = (double)m / 10.0;
  }
  __syncthreads();
  const double invP = 1.0 / (double)P;
  const int r = tid >> 4, c = tid & 15;
  double v = 0.0;
  if (r < d && c < d)
    v = (Ms[r * 16 + c] - Ms[r * 16 + d] * Ms[c * 16 + d] * invP) / (double)(P - 1);
  __syncthreads();
  if (r < d && c < d) Ms[r * 16 + c] = v;
  __syncthreads();
  if (tid < 64) wave_cholesky<16>(Ms, Ls, d, sh_h, dy.hchol, st.flags);
}

// The random-walk M step of one particle of run `st` (as k_mutate_rw).
template <class M, int U = kUnroll>
__device__ __forceinline__ int mstep_one(const BatchStatic &st, const BatchDyn &dy, int64_t p,
                                         const typename M::Y *__restrict__ y) {
  constexpr int D = M::D;
  using R = typename M::R;
  constexpr int S = M::S;
  const int64_t P = st.P;
  double th[D], z[D], pr[D];
#pragma unroll
  for (int i = 0; i < D; ++i) th[i] = st.theta[i * P + p];
  normals<D>(st.seed, st.run, (uint64_t)p, (uint64_t)dy.cycle, (uint64_t)dy.iter, kProposal, z,
             D);
  const double *__restrict__ hl = dy.hchol;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k <= i; ++k) s = fma(hl[i * D + k], z[k], s);
    pr[i] = th[i] + s;
  }
  const double lp1 = M::logprior(pr);
  R stv[S];
#pragma unroll
  for (int k = 0; k < S; ++k) stv[k] = (R)0;
  int acc = 0;
  double ll1 = -INFINITY;
  if (lp1 > -INFINITY) {
    const auto par = M::params(pr);
    ll1 = M::template advance<U>(par, stv, 0, dy.t, y);
    const double delta = (lp1 + ll1) - (st.logprior[p] + st.loglik[p]);
    const U64x4 w = draw4(st.seed, st.run, (uint64_t)p, (uint64_t)dy.cycle, (uint64_t)dy.iter,
                          kAccept);
    acc = (log(u01_oo(w.x0)) < delta) ? 1 : 0;
  }
  if (acc) {
#pragma unroll
    for (int i = 0; i < D; ++i) st.theta[i * P + p] = pr[i];
    st.logprior[p] = lp1;
    st.loglik[p] = ll1;
#pragma unroll
    for (int k = 0; k < S; ++k) reinterpret_cast<R *>(st.state)[k * P + p] = stv[k];
  }
  return acc;
}

// The Langevin step of one particle of run `st` (as k_mutate_mala).
template <class M>
__device__ __forceinline__ int mala_batch_one(const BatchStatic &st, const BatchDyn &dy, int64_t p,
                                              void *lds) {
  DevModel dm{};
  if constexpr (sizeof(typename M::Y) == 4) dm.y32 = static_cast<const float *>(st.y);
  else dm.y = static_cast<const double *>(st.y);
  return mala_one<M>(dm, st.P, p, dy.t, st.theta, st.logprior, st.loglik, st.state, st.grad,
                     dy.hchol, st.seed, st.run, (uint64_t)dy.cycle, (uint64_t)dy.iter, st.ckpt,
                     lds);
}

// Persistent M step over every active run: blocks of B threads pull
// (run, B-particle block) items until the counter passes the item count
// (every block reaches that exit).  kMala: the Langevin step (the block's
// dynamic LDS is the adjoint's buffer); U: observations per load batch.
template <class M0, class M1, bool kMala, int B = 64, int U = kUnroll>
__global__ void __launch_bounds__(B) k_batch_mutate(BatchArgs a) {
  extern __shared__ double lds_dyn[];
  __shared__ int sh_item;
  for (;;) {
    if (threadIdx.x == 0) sh_item = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int item = sh_item;
    __syncthreads();
    if (item >= a.n_mut_items) break;
    const int ri = owner(a, item, false);
    const BatchDyn &dy = a.dyn[ri];
    const BatchStatic &st = a.runs[dy.idx];
    const int64_t p = (int64_t)(item - dy.mut_begin) * B + threadIdx.x;
    int acc = 0;
    if (p < st.P) {
      if constexpr (kMala) {
        if (st.tag == 0) acc = mala_batch_one<M0>(st, dy, p, lds_dyn);
        else acc = mala_batch_one<M1>(st, dy, p, lds_dyn);
      } else {
        if (st.tag == 0)
          acc = mstep_one<M0, U>(st, dy, p, static_cast<const typename M0::Y *>(st.y));
        else
          acc = mstep_one<M1, U>(st, dy, p, static_cast<const typename M1::Y *>(st.y));
      }
    }
    const unsigned long long mask = __ballot(acc);
    if ((threadIdx.x & 63) == 0 && mask)
      atomicAdd(dy.n_accept, (unsigned long long)__popcll(mask));
  }
}

__global__ void k_batch_static(BatchStaticArgs a) {
  if (threadIdx.x < (unsigned)a.n) a.dst[threadIdx.x] = a.src[threadIdx.x];
}

smc_status launch_batch_static(const BatchStaticArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_static, dim3(1), dim3(64), 0, s, a);
  return launch_ok("batch/static table");
}

__global__ void k_batch_queue_reset(unsigned int *q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0u;
}

smc_status launch_batch_m(const BatchArgs &a, bool moments, int32_t family, int32_t waves,
                          hipStream_t s, const KernelTimer *timer, int32_t block,
                          int32_t unroll) {
  smc_status st;
  if (a.n_active <= 0) return SMC_OK;
  if (moments) {
    hipLaunchKernelGGL(k_batch_mom_partial, grid_of(a.n_mom_items), dim3(256), 0, s, a);
    if ((st = launch_ok("batch/moments partial"))) return st;
    hipLaunchKernelGGL(k_batch_mom_final, grid_of(a.n_active), dim3(256), 0, s, a);
    if ((st = launch_ok("batch/moments final"))) return st;
  }
  hipLaunchKernelGGL(k_batch_queue_reset, dim3(1), dim3(64), 0, s, a.queue);
  if ((st = launch_ok("batch/queue reset"))) return st;
  // `waves` persistent waves, in blocks of `block` threads
  const int32_t B = block ? block : 64;
  const int64_t blocks =
      std::max<int64_t>(1, std::min<int64_t>(a.n_mut_items, std::max(1, waves * 64 / B)));
  auto go = [&](auto kern, int32_t threads, size_t lds) {
    if (timer)
      hipExtLaunchKernelGGL(kern, grid_of(blocks), dim3(threads), lds, s, timer->start,
                            timer->stop, 0, a);
    else
      hipLaunchKernelGGL(kern, grid_of(blocks), dim3(threads), lds, s, a);
  };
  using F1 = Egarch<1, 0, float>;
  using F2 = Egarch<2, 1, float>;
  using D1 = Egarch<1, 0, double>;
  using D2 = Egarch<2, 1, double>;
  const bool mala = a.kernel == SMC_KERNEL_MALA;
  const int32_t U = unroll ? unroll : kUnroll;
  if (family == kFamilyFp32) {
    if (mala) {
      go(k_batch_mutate<F1, F2, true>, 64, std::max(lds_bytes_of<F1>(), lds_bytes_of<F2>()));
    } else {
      // the tuned shapes of FP32 random-walk batches
#define SMC_BATCH_SHAPE(b, u) \
  if (B == b && U == u) go(k_batch_mutate<F1, F2, false, b, u>, b, 0); else
      SMC_BATCH_SHAPE(64, 4) SMC_BATCH_SHAPE(64, 8) SMC_BATCH_SHAPE(64, 16)
      SMC_BATCH_SHAPE(128, 4) SMC_BATCH_SHAPE(128, 8) SMC_BATCH_SHAPE(128, 16)
      SMC_BATCH_SHAPE(256, 4) SMC_BATCH_SHAPE(256, 8) SMC_BATCH_SHAPE(256, 16)
      return set_error(SMC_E_UNSUPPORTED, "batch launch shape %d x %d", B, U);
#undef SMC_BATCH_SHAPE
    }
  } else {
    if (mala) go(k_batch_mutate<D1, D2, true>, 64, std::max(lds_bytes_of<D1>(), lds_bytes_of<D2>()));
    else go(k_batch_mutate<D1, D2, false>, 64, 0);
  }
  return launch_ok("batch/mutate");
}

}  // namespace smc
