// C ABI of the simulator (declared in include/smc.h): argument validation,
// workspace carve-up, the adaptive C-phase chunking, and the native driver
// of Algorithms 1 and 2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "common.h"
#include "launch.h"
#include "smc.h"

namespace smc {

namespace {
thread_local char g_err[512] = "";

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline char *wsb(const smc_particles *pop) { return reinterpret_cast<char *>(pop->ws); }

template <typename T>
inline T *ws_at(const smc_particles *pop, size_t off) {
  return reinterpret_cast<T *>(wsb(pop) + off);
}

}  // namespace

smc_status set_error(smc_status status, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return status;
}

WsLayout ws_layout(const DevModel &m, int32_t J, int32_t N) {
  const size_t P = (size_t)J * (size_t)N;
  WsLayout L{};
  size_t off = 0;
  L.small = off;
  off += align256(kSmallBytes);
  L.rsscols = off;
  off += align256((kMaxChunk + rss_slice_doubles((int64_t)P)) * sizeof(double));
  L.gather = off;
  off += align256((size_t)(2 * m.d + m.S + 2) * P * sizeof(double));
  L.cum = off;
  off += align256(P * sizeof(double));
  L.mpart = off;
  const size_t mw = m.d + 1 <= 16 ? 16 : 32;  // padded moments width
  off += align256((size_t)(kMomBlocks + 1) * mw * mw * sizeof(double));  // + the sums
  L.rpart = off;
  off += align256((size_t)J * 2 * kDMax * sizeof(double));
  L.cyc = off;
  off += align256(sizeof(CycleDyn)) +
         align256((size_t)kGraphMaxCycles * (sizeof(int64_t) + sizeof(int32_t) + sizeof(double)));
  L.acc = off;
  off += 256 + align256((P + 63) / 64 * sizeof(int32_t));
  L.wcols = off;
  L.fixed = off;
  return L;
}

namespace {

smc_status check_model(const smc_model *m) {
  if (!m) return set_error(SMC_E_INVALID_ARG, "model handle is NULL");
  return SMC_OK;
}

smc_status check_pop(const smc_model *m, const smc_particles *pop, bool need_ws = true) {
  if (!pop) return set_error(SMC_E_INVALID_ARG, "particles is NULL");
  if (pop->J < 2 || pop->N < 2) return set_error(SMC_E_INVALID_ARG, "need J >= 2 and N >= 2");
  if (pop->N > 16384) return set_error(SMC_E_UNSUPPORTED, "N > 16384 per group");
  if ((int64_t)pop->J * pop->N > (int64_t)1 << 30)
    return set_error(SMC_E_UNSUPPORTED, "more than 2^30 particles");
  if (!pop->theta || !pop->logprior || !pop->loglik || !pop->logw || !pop->ancestor)
    return set_error(SMC_E_INVALID_ARG, "a particle array is NULL");
  if (m->dev.S > 0 && !pop->state) return set_error(SMC_E_INVALID_ARG, "state is NULL");
  if (need_ws) {
    if (!pop->ws) return set_error(SMC_E_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(pop->ws) & 255)
      return set_error(SMC_E_INVALID_ARG, "workspace is not 256-byte aligned");
    const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
    if (pop->ws_bytes < L.fixed)
      return set_error(SMC_E_WORKSPACE, "workspace of %zu bytes < %zu", pop->ws_bytes, L.fixed);
  }
  return SMC_OK;
}

// The workspace's accept-count sink (AccSink), or none when the workspace
// does not hold the layout.
AccSink acc_sink(const smc_model *m, const smc_particles *pop) {
  if (!pop->ws || (reinterpret_cast<uintptr_t>(pop->ws) & 255)) return AccSink{};
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  if (pop->ws_bytes < L.fixed) return AccSink{};
  char *base = static_cast<char *>(pop->ws) + L.acc;
  return AccSink{reinterpret_cast<int32_t *>(base + 256),
                 reinterpret_cast<unsigned long long *>(base)};
}

int64_t chunk_capacity(const smc_model *m, const smc_particles *pop) {
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  const size_t P = (size_t)pop->J * pop->N;
  if (pop->ws_bytes <= L.wcols) return 0;
  return std::min<int64_t>(kMaxChunk, (int64_t)((pop->ws_bytes - L.wcols) / (P * sizeof(double))));
}

int32_t state_bytes(const smc_model *m) { return m->dev.prec == SMC_FP32 ? 4 : 8; }

// Page-locked, coherent host slot where the C-phase decision kernel stores
// each chunk's decision and the numerical flags word (one per host thread,
// kept for the life of the process); NULL if it cannot be had.  Device
// stores to coherent host memory bypass the device caches, so the host needs
// neither a fence nor an event: it watches the slot until every word carries
// the call's sequence number while the work queued after the kernel runs on.
DecisionSlot *decision_slot() {
  thread_local DecisionSlot *buf = nullptr;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void *p = nullptr;
    const unsigned flags = hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable;
    if (hipHostMalloc(&p, sizeof(DecisionSlot), flags) == hipSuccess) {
      buf = static_cast<DecisionSlot *>(p);
      *buf = DecisionSlot{};
    }
  }
  return buf;
}

// The calling thread's page-locked readback area for batched C phases, at
// least n doubles; grown (reallocated) on demand and kept for the life of
// the process; NULL if it cannot be had.
double *batch_readback(size_t n) {
  thread_local double *buf = nullptr;
  thread_local size_t cap = 0;
  if (cap < n) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    void *p = nullptr;
    if (hipHostMalloc(&p, n * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
    buf = static_cast<double *>(p);
    cap = n;
  }
  return buf;
}

// An event (no timing) of the calling thread for the current device, marking
// the completion of a copy back so the host can wait for it alone while
// later work stays queued; kept for the life of the process.
smc_status readback_event(hipEvent_t *out) {
  thread_local hipEvent_t ev[16] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16)
    return set_error(SMC_E_DEVICE, "readback event: device %d not supported", dev);
  if (!ev[dev] && hipEventCreateWithFlags(&ev[dev], hipEventDisableTiming) != hipSuccess) {
    ev[dev] = nullptr;
    return set_error(SMC_E_DEVICE, "creating a readback event failed");
  }
  *out = ev[dev];
  return SMC_OK;
}

// Waits until the slot holds this call's whole decision for the chunk
// (t, t1] (read_decision: every word tagged with `seq`, two reads agreeing,
// the date inside the chunk).  The stream is polled every millisecond: once
// all its work has completed the slot gets 10 more ms, then the wait fails
// (false).
bool await_decision(const DecisionSlot *slot, uint32_t seq, int64_t t, int64_t t1, hipStream_t s,
                    StopInfo *out, int32_t *flags) {
  const volatile DecisionSlot *v = slot;
  using clock = std::chrono::steady_clock;
  auto next_poll = clock::now() + std::chrono::milliseconds(1);
  clock::time_point idle_since{};
  bool idle = false;
  while (!read_decision(v, seq, t, t1, out, flags)) {
    const auto now = clock::now();
    if (now < next_poll) continue;
    next_poll = now + std::chrono::milliseconds(1);
    if (!idle) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return false;
      idle = true;
      idle_since = now;
    } else if (now - idle_since > std::chrono::milliseconds(10)) {
      return false;
    }
  }
  return true;
}

// Event i of the calling thread's pool for the current device.  The pools
// grow on demand and keep their events for the life of the process, so timed
// runs create events only the first time.  No system-scope fences: the stamps
// are read only after the stream has been synchronised (a timed launch then
// costs about 2 us more instead of about 6).
constexpr int kEventPoolDevices = 16;
smc_status timing_event(size_t i, hipEvent_t *out) {
  thread_local std::vector<hipEvent_t> pools[kEventPoolDevices];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kEventPoolDevices)
    return set_error(SMC_E_DEVICE, "timing events: device %d not supported", dev);
  std::vector<hipEvent_t> &v = pools[dev];
  while (v.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
      return set_error(SMC_E_DEVICE, "creating a timing event failed");
    v.push_back(e);
  }
  *out = v[i];
  return SMC_OK;
}


// Page-locked, coherent host word through which a device-driven run reports
// its progress (k_cycle_end); one per host thread, kept for the life of the
// process; NULL if it cannot be had.
uint32_t *progress_word() {
  thread_local uint32_t *w = nullptr;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void *p = nullptr;
    const unsigned flags = hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable;
    if (hipHostMalloc(&p, 256, flags) == hipSuccess) w = static_cast<uint32_t *>(p);
  }
  return w;
}

// The executable step graphs of device-driven runs, keyed by every value
// their kernels take by value (model, arrays, sizes, rules; the key and the
// dates come from the device state), so a run with the same set-up launches
// the graph it captured before.  A few per host thread, the oldest replaced
// first; kept for the life of the process.
struct StepKey {
  int32_t device;
  int32_t J, N, check_every, Rbar, scheme;
  int64_t cap;
  double D1;
  DevModel dm;
  const void *arrays[14];
};
struct StepGraph {
  StepKey key;
  hipGraphExec_t exec;
};
constexpr size_t kStepGraphs = 4;

}  // namespace

// The S phase that an adaptive C phase may enqueue ahead of its last host
// decision (it runs only if the phase ended; see correct_impl).
struct ResampleAhead {
  int32_t scheme;
  int32_t cycle;
  smc_rng rng;
};
smc_status correct_impl(const smc_model *m, smc_particles *pop, int64_t t_from, int64_t t_max,
                        int64_t check_every, double rss_min, double *group_logwbar,
                        int64_t *t_to, double *rss, void *stream, int64_t first_chunk,
                        const ResampleAhead *ahead = nullptr, bool *resampled = nullptr,
                        int32_t *flags_seen = nullptr);

}  // namespace smc

using namespace smc;

smc_status run_device_driven(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                             smc_run_record *rec, hipStream_t s);

extern "C" {

const char *smc_status_string(smc_status s) {
  switch (s) {
    case SMC_OK: return "ok";
    case SMC_E_INVALID_ARG: return "invalid argument";
    case SMC_E_UNSUPPORTED: return "unsupported";
    case SMC_E_DEVICE: return "device error";
    case SMC_E_NUMERIC: return "numerical failure";
    case SMC_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char *smc_last_error(void) { return g_err; }

smc_status smc_model_create(const smc_model_desc *desc, smc_model **out) {
  if (!desc || !out) return set_error(SMC_E_INVALID_ARG, "NULL description or output");
  *out = nullptr;
  if (desc->T < 1) return set_error(SMC_E_INVALID_ARG, "T must be >= 1");
  if (!desc->y) return set_error(SMC_E_INVALID_ARG, "y is NULL");
  if (desc->precision != SMC_FP64 && desc->precision != SMC_FP32)
    return set_error(SMC_E_INVALID_ARG, "precision %d", desc->precision);
  DevModel d{};
  d.kind = desc->kind;
  d.K = desc->K;
  d.shock = desc->shock;
  d.nreg = desc->nreg;
  d.prec = desc->precision;
  d.T = desc->T;
  d.y = desc->y;
  d.y32 = desc->y32;
  d.X = desc->X;
  if (desc->kind == SMC_MODEL_LINREG) {
    if (desc->ncomp != 0) return set_error(SMC_E_INVALID_ARG, "ncomp must be 0 for the regression");
    if (desc->nreg < 1 || desc->nreg > 4)
      return set_error(SMC_E_UNSUPPORTED, "regression needs 1..4 regressors");
    if (!desc->X) return set_error(SMC_E_INVALID_ARG, "X is NULL");
    if (desc->precision != SMC_FP64)
      return set_error(SMC_E_UNSUPPORTED, "the regression runs in FP64 only");
    d.d = desc->nreg + 1;
    d.S = 0;
  } else if (desc->kind == SMC_MODEL_EGARCH) {
    if (desc->shock != SMC_SHOCK_GAUSS && desc->shock != SMC_SHOCK_STUDENT_T &&
        desc->shock != SMC_SHOCK_MIXTURE)
      return set_error(SMC_E_INVALID_ARG, "shock %d", desc->shock);
    if (desc->shock == SMC_SHOCK_MIXTURE) {
      if (desc->K < 1 || desc->K > 4) return set_error(SMC_E_UNSUPPORTED, "mixture needs K in 1..4");
      if (desc->ncomp < 2 || desc->ncomp > 4)
        return set_error(SMC_E_UNSUPPORTED, "mixture needs I in 2..4 components");
    } else {
      if (desc->K < 1 || desc->K > 2) return set_error(SMC_E_UNSUPPORTED, "EGARCH needs K in {1,2}");
      if (desc->ncomp != 0) return set_error(SMC_E_INVALID_ARG, "ncomp must be 0 without a mixture");
    }
    if (desc->precision == SMC_FP32 && !desc->y32)
      return set_error(SMC_E_INVALID_ARG, "FP32 recursion needs y32");
    d.d = 2 + 3 * desc->K + (desc->shock == SMC_SHOCK_STUDENT_T ? 1 : 0) +
          (desc->shock == SMC_SHOCK_MIXTURE ? 3 * desc->ncomp : 0);
    d.S = desc->K + 1;
    d.ncomp = desc->shock == SMC_SHOCK_MIXTURE ? desc->ncomp : 0;
  } else {
    return set_error(SMC_E_INVALID_ARG, "model kind %d", desc->kind);
  }
  smc_model *m = new (std::nothrow) smc_model;
  if (!m) return set_error(SMC_E_INVALID_ARG, "out of host memory");
  m->dev = d;
  *out = m;
  return SMC_OK;
}

smc_status smc_model_destroy(smc_model *m) {
  delete m;
  return SMC_OK;
}

smc_status smc_model_set_launch(smc_model *m, int32_t block, int32_t unroll) {
  if (!m) return set_error(SMC_E_INVALID_ARG, "model handle is NULL");
  if (block != 0 && block != 64 && block != 128 && block != 256)
    return set_error(SMC_E_INVALID_ARG, "threads per block %d (0, 64, 128 or 256)", block);
  if (unroll != 0 && unroll != 4 && unroll != 8 && unroll != 16)
    return set_error(SMC_E_INVALID_ARG, "observations per load batch %d (0, 4, 8 or 16)", unroll);
  const bool dflt = (block == 0 || block == 64) && (unroll == 0 || unroll == 8);
  if (!dflt && !has_launch_shapes(m->dev))
    return set_error(SMC_E_UNSUPPORTED, "no tuned launch shapes for this model");
  m->dev.block = block == 64 ? 0 : block;
  m->dev.unroll = unroll == 8 ? 0 : unroll;
  return SMC_OK;
}

int32_t smc_model_dim(const smc_model *m) { return m ? m->dev.d : -1; }
int32_t smc_model_state_dim(const smc_model *m) { return m ? m->dev.S : -1; }

size_t smc_workspace_bytes(const smc_model *m, int32_t J, int32_t N, int64_t max_chunk) {
  if (!m || J < 1 || N < 1) return 0;
  if (max_chunk <= 0) max_chunk = kDefaultChunk;
  if (max_chunk > kMaxChunk) max_chunk = kMaxChunk;
  const WsLayout L = ws_layout(m->dev, J, N);
  return L.wcols + (size_t)max_chunk * (size_t)J * (size_t)N * sizeof(double);
}

smc_status smc_init_from_prior(const smc_model *m, smc_particles *pop, smc_rng rng,
                               void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop, false))) return st;
  const int64_t P = (int64_t)pop->J * pop->N;
  return launch_init(m->dev, P, rng.seed, rng.run, pop->theta, pop->logprior, pop->loglik,
                     pop->state, pop->logw, as_stream(stream));
}

smc_status smc_correct(const smc_model *m, smc_particles *pop, int64_t t_from, int64_t t_max,
                       int64_t check_every, double rss_min, double *group_logwbar,
                       int64_t *t_to, double *rss, void *stream) {
  return correct_impl(m, pop, t_from, t_max, check_every, rss_min, group_logwbar, t_to, rss,
                      stream, 16);
}

smc_status smc_correct_async(const smc_model *m, smc_particles *pop, int64_t t_from,
                             int64_t t_max, int64_t check_every, double rss_min,
                             double *group_logwbar, int64_t *t_to, double *rss, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!group_logwbar || !t_to) return set_error(SMC_E_INVALID_ARG, "NULL output");
  if (t_from < 0 || t_max > m->dev.T || t_from > t_max)
    return set_error(SMC_E_INVALID_ARG, "dates 0 <= t_from <= t_max <= T violated");
  if (check_every < 1) return set_error(SMC_E_INVALID_ARG, "check_every < 1");
  hipStream_t s = as_stream(stream);
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  double *rsscols = ws_at<double>(pop, L.rsscols);
  if (!(rss_min > 0.0 && t_from < t_max)) {
    // the whole range, then the RSS of the final weights
    if (t_max == t_from) {
      if ((st = fill_f64(pop->logw, P, 0.0, s))) return st;
    } else if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik,
                                    t_from, t_max, true, s))) {
      return st;
    }
    if ((rss && (st = launch_rss_cols(pop->logw, P, 1, rsscols, s))) ||
        (st = launch_group_logwbar(pop->logw, pop->J, pop->N, group_logwbar, s)))
      return st;
    return launch_phase_out(nullptr, rsscols, t_max, t_to, rss, s);
  }
  const int64_t cap = chunk_capacity(m, pop);
  if (cap < 1) return set_error(SMC_E_WORKSPACE, "workspace has no room for C-phase chunks");
  CycleDyn *cyc = ws_at<CycleDyn>(pop, L.cyc);
  StopInfo *stop_dev = ws_at<StopInfo>(pop, L.small + kSmallStop);
  DevModel dm = m->dev;
  dm.cyc = cyc;
  // The chunks of smc_correct (16 observations, doubling up to the
  // workspace's capacity), enough of them to reach t_max; those after the
  // phase's end return at once.
  CycleDyn init{};
  init.T = m->dev.T;
  init.P = P;
  init.check_every = check_every;
  init.cap = cap;
  init.t = init.t_phase = t_from;
  init.t_stop = t_max;
  init.chunk = std::min<int64_t>(16, cap);
  init.zero_first = 1;
  init.rss = 1.0;
  init.J = pop->J;
  if ((st = launch_phase_init(cyc, init, s))) return st;
  double *W = ws_at<double>(pop, L.wcols);
  for (int64_t covered = 0, chunk = init.chunk; covered < t_max - t_from;
       covered += chunk, chunk = std::min(2 * chunk, cap)) {
    if ((st = launch_cscan(dm, P, pop->theta, pop->state, pop->logw, 0, 0, check_every, 0, false,
                           W, s)) ||
        (st = launch_rss_scan(W, P, std::min<int64_t>(chunk, kMaxChunk), rsscols, s, &cyc->nc)) ||
        (st = launch_find_stop(rsscols, 0, 0, 0, check_every, 0, rss_min, stop_dev, s, nullptr, 0,
                               nullptr, cyc)) ||
        (st = launch_ccommit(dm, P, pop->theta, pop->state, pop->logw, pop->loglik, 0, 0, false,
                             s, &stop_dev->t_commit)) ||
        (st = launch_phase_step(cyc, s)))
      return st;
  }
  if ((st = launch_group_logwbar(pop->logw, pop->J, pop->N, group_logwbar, s))) return st;
  return launch_phase_out(cyc, nullptr, 0, t_to, rss, s);
}

}  // extern "C"

// The C phase with a first speculative chunk of `first_chunk` observations
// (the driver passes a length predicted from the previous cycle).  Adaptive
// chunks: scan every checked date (the scan reduces each wave's weights to
// RSS sums on the fly), merge them into each date's RSS, decide the stop
// on the device, and queue the commit to the decided date before the host
// reads the decision back; with `ahead`, the S phase (which does nothing
// unless the phase ended, and then also writes the group weights) is queued
// too, so the device has that work in hand while the host waits.
// *resampled tells whether the S phase was queued that way; *flags_seen
// receives the workspace's flags word as the last decision carried it (-1
// when no decision came through the host slot).
smc_status smc::correct_impl(const smc_model *m, smc_particles *pop, int64_t t_from,
                             int64_t t_max, int64_t check_every, double rss_min,
                             double *group_logwbar, int64_t *t_to, double *rss, void *stream,
                             int64_t first_chunk, const ResampleAhead *ahead, bool *resampled,
                             int32_t *flags_seen) {
  smc_status st;
  if (resampled) *resampled = false;
  if (flags_seen) *flags_seen = -1;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!group_logwbar || !t_to) return set_error(SMC_E_INVALID_ARG, "NULL output");
  if (t_from < 0 || t_max > m->dev.T || t_from > t_max)
    return set_error(SMC_E_INVALID_ARG, "dates 0 <= t_from <= t_max <= T violated");
  if (check_every < 1) return set_error(SMC_E_INVALID_ARG, "check_every < 1");
  hipStream_t s = as_stream(stream);
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  double *rsscols = ws_at<double>(pop, L.rsscols);
  double *W = ws_at<double>(pop, L.wcols);
  int64_t t_stop = t_max;
  double rss_at_stop = 1.0;
  const bool adaptive = rss_min > 0.0 && t_from < t_max;
  // logw = 0 at the start of the phase: folded into the first kernel that
  // touches the weights (or a fill when no observation is added).
  if (t_max == t_from && (st = fill_f64(pop->logw, P, 0.0, s))) return st;
  bool zero_first = true;
  if (!adaptive) {
    if (t_max > t_from &&
        (st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik, t_from,
                             t_max, true, s)))
      return st;
    if (rss) {
      if ((st = launch_rss_cols(pop->logw, P, 1, rsscols, s))) return st;
      if (hipMemcpyAsync(&rss_at_stop, rsscols, sizeof(double), hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "correct: reading the RSS failed");
    }
  } else {
    const int64_t cap = chunk_capacity(m, pop);
    if (cap < 1) return set_error(SMC_E_WORKSPACE, "workspace has no room for C-phase chunks");
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(first_chunk, cap));
    int64_t t = t_from;
    StopInfo *stop_dev = ws_at<StopInfo>(pop, L.small + kSmallStop);
    // With the host slot the decision kernel stores the decision and the
    // flags word there itself (no copy); else the decision is copied back.
    DecisionSlot *slot = decision_slot();
    thread_local uint32_t slot_seq = 0;
    StopInfo got{};
    hipEvent_t ev = nullptr;
    if (!slot && (st = readback_event(&ev))) return st;
    bool stopped = false, queued_ahead = false;
    while (!stopped) {
      const int64_t t1 = std::min(t + chunk, t_max);
      // checked dates in (t, t1]: the multiples of check_every, and t_max
      const int64_t nc = t1 / check_every - t / check_every +
                         ((t1 == t_max && t_max % check_every != 0) ? 1 : 0);
      if (nc == 0) {
        if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik, t,
                                 t1, zero_first, s)))
          return st;
        zero_first = false;
        t = t1;
        stopped = t >= t_max;
        queued_ahead = false;
        chunk = std::min(2 * chunk, cap);
        continue;
      }
      if ((st = launch_cscan(m->dev, P, pop->theta, pop->state, pop->logw, t, t1, check_every,
                             t_max, zero_first, W, s)) ||
          (st = launch_rss_scan(W, P, nc, rsscols, s)) ||
          (st = launch_find_stop(rsscols, nc, t, t1, check_every, t_max, rss_min, stop_dev, s,
                                 slot, ++slot_seq, ws_at<int32_t>(pop, L.small + kSmallFlags))))
        return st;
      if (!slot && (hipMemcpyAsync(&got, stop_dev, sizeof(StopInfo), hipMemcpyDeviceToHost, s) !=
                        hipSuccess ||
                    hipEventRecord(ev, s) != hipSuccess))
        return set_error(SMC_E_DEVICE, "correct: reading the stop decision failed");
      if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik, t, t1,
                               zero_first, s, &stop_dev->t_commit)))
        return st;
      if (ahead) {
        // the S phase also writes the group weights of the phase's end
        if ((st = launch_resample(pop->logw, pop->J, pop->N, ahead->scheme, ahead->rng.seed,
                                  ahead->rng.run, (uint64_t)ahead->cycle, pop->ancestor,
                                  ws_at<double>(pop, L.cum),
                                  ws_at<int32_t>(pop, L.small + kSmallFlags), m->dev.d, m->dev.S,
                                  state_bytes(m), pop->theta, pop->logprior, pop->loglik,
                                  pop->state, pop->grad, ws_at<double>(pop, L.gather), s,
                                  &stop_dev->ends, group_logwbar)))
          return st;
      }
      int32_t fl = -1;
      if (slot ? !await_decision(slot, slot_seq, t, t1, s, &got, &fl)
               : hipEventSynchronize(ev) != hipSuccess)
        return set_error(SMC_E_DEVICE, "correct: the stop decision did not reach the host");
      if (flags_seen) *flags_seen = fl;
      zero_first = false;
      rss_at_stop = got.rss;
      t = got.t_commit;
      stopped = got.ends != 0;
      queued_ahead = ahead != nullptr;
      chunk = std::min(2 * chunk, cap);
    }
    t_stop = t;
    if (queued_ahead) {
      *t_to = t_stop;
      if (rss) *rss = rss_at_stop;
      if (resampled) *resampled = true;
      return SMC_OK;
    }
  }
  if ((st = launch_group_logwbar(pop->logw, pop->J, pop->N, group_logwbar, s))) return st;
  *t_to = t_stop;
  if (rss) *rss = rss_at_stop;
  return SMC_OK;
}

extern "C" {

smc_status smc_resample(const smc_model *m, smc_particles *pop, int32_t scheme, smc_rng rng,
                        int32_t cycle, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (scheme < SMC_RESAMPLE_RESIDUAL || scheme > SMC_RESAMPLE_SYSTEMATIC)
    return set_error(SMC_E_INVALID_ARG, "resampling scheme %d", scheme);
  hipStream_t s = as_stream(stream);
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  (void)P;
  return launch_resample(pop->logw, pop->J, pop->N, scheme, rng.seed, rng.run, (uint64_t)cycle,
                         pop->ancestor, ws_at<double>(pop, L.cum),
                         ws_at<int32_t>(pop, L.small + kSmallFlags), m->dev.d, m->dev.S,
                         state_bytes(m), pop->theta, pop->logprior, pop->loglik, pop->state,
                         pop->grad, ws_at<double>(pop, L.gather), s);
}

smc_status smc_particle_moments(const smc_model *m, const smc_particles *pop, const int32_t *mh,
                                double *mean, double *cov, double *hchol, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!mh || !hchol) return set_error(SMC_E_INVALID_ARG, "mh and hchol are required");
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  MomArgs a{};
  a.theta = pop->theta;
  a.P = P;
  a.d = m->dev.d;
  a.part = ws_at<double>(pop, L.mpart);
  a.mh = const_cast<int32_t *>(mh);
  a.mean_out = mean;
  a.cov_out = cov;
  a.hchol = hchol;
  a.flags = ws_at<int32_t>(pop, L.small + kSmallFlags);
  return launch_moments(a, as_stream(stream));
}

smc_status smc_mutate(const smc_model *m, smc_particles *pop, int64_t t, int32_t kernel,
                      const double *hchol, smc_rng rng, int32_t cycle, int32_t iter,
                      int64_t *n_accept, uint8_t *accepted, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop, false))) return st;
  if (!hchol || !n_accept) return set_error(SMC_E_INVALID_ARG, "hchol and n_accept are required");
  if (t < 0 || t > m->dev.T) return set_error(SMC_E_INVALID_ARG, "date t out of range");
  const int64_t P = (int64_t)pop->J * pop->N;
  hipStream_t s = as_stream(stream);
  // with a workspace, the counts go through its sink and are added at once
  DevModel dm = m->dev;
  dm.acc = acc_sink(m, pop);
  auto flushed = [&](smc_status e) {
    return (e || !dm.acc.part) ? e : launch_acc_flush(dm.acc, P, s);
  };
  if (kernel == SMC_KERNEL_RW)
    return flushed(launch_mutate_rw(dm, P, t, pop->theta, pop->logprior, pop->loglik,
                                    pop->state, hchol, rng.seed, rng.run, (uint64_t)cycle,
                                    (uint64_t)iter, n_accept, accepted, s));
  if (kernel == SMC_KERNEL_MALA) {
    if (!pop->grad) return set_error(SMC_E_INVALID_ARG, "the Langevin kernel needs pop->grad");
    if ((st = check_pop(m, pop))) return st;
    const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
    const size_t need = adjoint_ckpt_bytes(m->dev, P, t);
    if (pop->ws_bytes < L.wcols + need)
      return set_error(SMC_E_WORKSPACE, "Langevin step needs %zu workspace bytes",
                       L.wcols + need);
    return flushed(launch_mutate_mala(dm, P, t, pop->theta, pop->logprior, pop->loglik,
                                      pop->state, pop->grad, hchol, rng.seed, rng.run,
                                      (uint64_t)cycle, (uint64_t)iter, n_accept, accepted,
                                      ws_at<char>(pop, L.wcols), s));
  }
  if (kernel == SMC_KERNEL_INDEPENDENT) {
    const int32_t d = m->dev.d;
    return flushed(launch_mutate_indep(dm, P, t, pop->theta, pop->logprior, pop->loglik,
                                       pop->state, hchol, hchol + (int64_t)d * d, rng.seed,
                                       rng.run, (uint64_t)cycle, (uint64_t)iter, n_accept,
                                       accepted, s));
  }
  return set_error(SMC_E_INVALID_ARG, "kernel %d", kernel);
}

smc_status smc_loglik(const smc_model *m, int64_t P, const double *theta, int64_t t,
                      double *loglik, void *state_out, void *stream) {
  smc_status st;
  if ((st = check_model(m))) return st;
  if (t < 0 || t > m->dev.T) return set_error(SMC_E_INVALID_ARG, "date t out of range");
  if (P == 0) return SMC_OK;
  if (P < 0 || !theta || !loglik) return set_error(SMC_E_INVALID_ARG, "bad loglik arguments");
  return launch_loglik(m->dev, P, theta, t, loglik, state_out, as_stream(stream));
}

size_t smc_backward_ws_bytes(const smc_model *m, int64_t P, int64_t t) {
  if (!m || P < 0 || t < 0) return 0;
  return adjoint_ckpt_bytes(m->dev, P, t);
}

smc_status smc_loglik_backward(const smc_model *m, int64_t P, const double *theta, int64_t t,
                               const double *dloglik, double *dtheta, void *ws, size_t ws_bytes,
                               void *stream) {
  smc_status st;
  if ((st = check_model(m))) return st;
  if (t < 0 || t > m->dev.T) return set_error(SMC_E_INVALID_ARG, "date t out of range");
  if (P == 0) return SMC_OK;
  if (P < 0 || !theta || !dloglik || !dtheta)
    return set_error(SMC_E_INVALID_ARG, "bad loglik_backward arguments");
  const size_t need = adjoint_ckpt_bytes(m->dev, P, t);
  if (need > 0 && (!ws || ws_bytes < need))
    return set_error(SMC_E_WORKSPACE, "adjoint needs %zu workspace bytes", need);
  return launch_loglik_backward(m->dev, P, theta, t, dloglik, dtheta, ws, as_stream(stream));
}

size_t smc_mala_workspace_bytes(const smc_model *m, int32_t J, int32_t N, int64_t max_chunk) {
  if (!m || J < 1 || N < 1) return 0;
  const size_t base = smc_workspace_bytes(m, J, N, max_chunk);
  const WsLayout L = ws_layout(m->dev, J, N);
  const size_t ck = L.wcols + adjoint_ckpt_bytes(m->dev, (int64_t)J * N, m->dev.T);
  return base > ck ? base : ck;
}

smc_status smc_posterior_grad(const smc_model *m, smc_particles *pop, int64_t t, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!pop->grad) return set_error(SMC_E_INVALID_ARG, "pop->grad is NULL");
  if (t < 0 || t > m->dev.T) return set_error(SMC_E_INVALID_ARG, "date t out of range");
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  const size_t need = adjoint_ckpt_bytes(m->dev, P, t);
  if (pop->ws_bytes < L.wcols + need)
    return set_error(SMC_E_WORKSPACE, "posterior gradient needs %zu workspace bytes",
                     L.wcols + need);
  return launch_grad_post(m->dev, P, pop->theta, t, pop->grad, ws_at<char>(pop, L.wcols),
                          as_stream(stream));
}

smc_status smc_log_ml(int32_t L, int32_t J, const double *group_logwbar, double *out,
                      void *stream) {
  if (L < 1 || J < 2 || !group_logwbar || !out)
    return set_error(SMC_E_INVALID_ARG, "need L >= 1, J >= 2 and device arrays");
  return launch_log_ml(L, J, group_logwbar, out, as_stream(stream));
}

smc_status smc_adapt_scale(const int64_t *n_accept, int64_t P, int32_t target_permille,
                           int32_t *mh, void *stream) {
  if (!n_accept || !mh || P < 1 || target_permille < 0 || target_permille > 1000)
    return set_error(SMC_E_INVALID_ARG, "bad adapt_scale arguments");
  return launch_adapt(n_accept, P, target_permille, mh, as_stream(stream));
}

int32_t smc_num_test_functions(const smc_model *m, int32_t which) {
  if (!m || (which != SMC_TEST_PARAMS && which != SMC_TEST_MODEL)) return -1;
  return num_test_fns(m->dev, which);
}

smc_status smc_test_moments(const smc_model *m, smc_particles *pop, int64_t t, int32_t which,
                            double *out, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!out) return set_error(SMC_E_INVALID_ARG, "NULL output");
  if (t < 0 || t > m->dev.T) return set_error(SMC_E_INVALID_ARG, "date %lld", (long long)t);
  const int32_t G = smc_num_test_functions(m, which);
  if (G < 1) return set_error(SMC_E_INVALID_ARG, "test functions %d", which);
  hipStream_t s = as_stream(stream);
  const int64_t P = (int64_t)pop->J * pop->N;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  double *g = ws_at<double>(pop, L.gather);  // [G][P], G <= 2d + S + 2 rows
  if ((st = launch_test_fns(m->dev, P, pop->theta, pop->state, t, which, g, s))) return st;
  return launch_report(g, pop->J, pop->N, G, ws_at<double>(pop, L.rpart), out, nullptr, s);
}

smc_status smc_log_score(int32_t L, int32_t J, const double *group_logwbar, const int64_t *t_end,
                         int64_t burn_in, double *out, void *stream) {
  if (L < 1 || J < 2 || !group_logwbar || !t_end || !out)
    return set_error(SMC_E_INVALID_ARG, "log score needs L >= 1, J >= 2 and arrays");
  int32_t l0 = 0;
  while (l0 < L && (l0 == 0 ? 0 : t_end[l0 - 1]) < burn_in) ++l0;
  if (l0 == 0 || l0 >= L || t_end[l0 - 1] != burn_in)
    return set_error(SMC_E_INVALID_ARG, "no cycle ends at the burn-in date %lld",
                     (long long)burn_in);
  return smc_log_ml(L - l0, J, group_logwbar + (int64_t)l0 * J, out, stream);
}

smc_status smc_rne(const smc_model *m, const smc_particles *pop, double *rne, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!rne) return set_error(SMC_E_INVALID_ARG, "rne is NULL");
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  return launch_rne(pop->theta, pop->J, pop->N, m->dev.d, ws_at<double>(pop, L.rpart), rne,
                    as_stream(stream));
}

smc_status smc_flags(const smc_particles *pop, int32_t *flags, void *stream) {
  if (!pop || !pop->ws || !flags) return set_error(SMC_E_INVALID_ARG, "bad flags arguments");
  hipStream_t s = as_stream(stream);
  int32_t *dflags = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(pop->ws) + kSmallFlags);
  if (hipMemcpyAsync(flags, dflags, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "reading flags failed");
  return fill_i32(dflags, 1, 0, s);
}

smc_status smc_run(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                   smc_run_record *rec, void *stream) {
  smc_status st;
  if ((st = check_model(m)) || (st = check_pop(m, pop))) return st;
  if (!cfg || !rec) return set_error(SMC_E_INVALID_ARG, "NULL config or record");
  if (cfg->J != pop->J || cfg->N != pop->N)
    return set_error(SMC_E_INVALID_ARG, "config and population shapes differ");
  if (!rec->t_end || !rec->R || !rec->rss || !rec->n_accept || !rec->hchol ||
      !rec->group_logwbar || !rec->log_ml)
    return set_error(SMC_E_INVALID_ARG, "a record array is NULL");
  if (cfg->Lmax < 1 || cfg->RmaxRec < 1 || cfg->check_every < 1 || cfg->force_every < 0)
    return set_error(SMC_E_INVALID_ARG, "bad record capacity or check spacing");
  if (cfg->kernel != SMC_KERNEL_RW && cfg->kernel != SMC_KERNEL_MALA &&
      cfg->kernel != SMC_KERNEL_INDEPENDENT)
    return set_error(SMC_E_INVALID_ARG, "kernel %d", cfg->kernel);
  if (cfg->scheme < SMC_RESAMPLE_RESIDUAL || cfg->scheme > SMC_RESAMPLE_SYSTEMATIC)
    return set_error(SMC_E_INVALID_ARG, "resampling scheme %d", cfg->scheme);
  const bool indep = cfg->kernel == SMC_KERNEL_INDEPENDENT;
  if (indep && !rec->mean)
    return set_error(SMC_E_INVALID_ARG, "the independent sampler records its means");
  if (cfg->kernel == SMC_KERNEL_MALA && !pop->grad)
    return set_error(SMC_E_INVALID_ARG, "the Langevin kernel needs pop->grad");
  if (cfg->graph != 0 && cfg->graph != 1)
    return set_error(SMC_E_INVALID_ARG, "graph must be 0 or 1");
  const int32_t G = smc_num_test_functions(m, cfg->test_fn);
  if (G < 1) return set_error(SMC_E_INVALID_ARG, "test functions %d", cfg->test_fn);
  if (cfg->burn_in < 0 || cfg->burn_in >= m->dev.T)
    return set_error(SMC_E_INVALID_ARG, "burn-in date %lld", (long long)cfg->burn_in);
  hipStream_t s = as_stream(stream);
  if (cfg->graph) return run_device_driven(m, pop, cfg, rec, s);
  const int64_t P = (int64_t)pop->J * pop->N;
  const int32_t d = m->dev.d;
  const int64_t T = m->dev.T;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  int32_t *mh = ws_at<int32_t>(pop, L.small + kSmallMh);
  int32_t *dflags = ws_at<int32_t>(pop, L.small + kSmallFlags);
  if ((st = fill_i32(dflags, 1, 0, s))) return st;
  if ((st = fill_i64(rec->n_accept, (int64_t)cfg->Lmax * cfg->RmaxRec, 0, s))) return st;
  // Each Metropolis step leaves its accept counts in the workspace's sink;
  // the next iteration's moment partials add them to the record (those of a
  // phase's last step the next phase's first moments, and after the run's
  // last step a launch of its own).
  DevModel dm = m->dev;
  dm.acc = acc_sink(m, pop);
  if ((st = fill_i64(reinterpret_cast<int64_t *>(dm.acc.pending), 1, 0, s))) return st;
  // Moments with the step-size rule folded in: no separate launch for it.
  MomArgs ma{};
  ma.theta = pop->theta;
  ma.P = P;
  ma.d = d;
  ma.acc = dm.acc;
  ma.target_permille = cfg->kernel == SMC_KERNEL_MALA ? 574 : 250;
  ma.part = ws_at<double>(pop, L.mpart);
  ma.mh = mh;
  ma.flags = dflags;
  if ((st = smc_init_from_prior(m, pop, cfg->rng, stream))) return st;
  int64_t t = 0, evals = 0, steps = 0, last_len = 0;
  int32_t l = 0;
  // Optional per-launch timing of the mutation kernel (every time_every-th
  // iteration): pairs of pooled events, resolved after the run.  The random-walk and independent kernels
  // carry the events on their own dispatch; the Langevin step (several
  // kernels) is bracketed by two event records.
  struct Timed {
    hipEvent_t a = nullptr, b = nullptr;
    int64_t slot = 0;
  };
  std::vector<Timed> timed;
  if (rec->mutate_ms)
    std::fill(rec->mutate_ms, rec->mutate_ms + (int64_t)cfg->Lmax * cfg->RmaxRec, -1.f);
  while (t < T) {
    if (l >= cfg->Lmax) return set_error(SMC_E_INVALID_ARG, "record holds only %d cycles", cfg->Lmax);
    int64_t t_stop = T;
    if (cfg->force_every > 0) t_stop = std::min(t_stop, (t / cfg->force_every + 1) * cfg->force_every);
    if (cfg->burn_in > t) t_stop = std::min(t_stop, cfg->burn_in);
    if (cfg->replay) {
      t_stop = rec->t_end[l];
      if (t_stop <= t || t_stop > T)
        return set_error(SMC_E_INVALID_ARG, "replayed date %lld out of order", (long long)t_stop);
    }
    // The flags raised by the previous cycle's S and M phases travel back
    // with this cycle's C-phase decisions (the decision kernel stores them in
    // the page-locked slot; one host synchronisation fewer per cycle); a
    // raised flag ends the run after that readback.
    int32_t fl_seen = -1;
    int64_t t_new = t;
    double rss = NAN;
    // Speculate on a cycle twice as long as the previous one, so most C
    // phases need a single host round trip (cycles lengthen as the posterior
    // concentrates; evaluations past the stop date are cheap beside the M
    // phase's).
    const int64_t hint = std::max<int64_t>(16, 2 * last_len + 16);
    // The S phase is queued by the C phase ahead of its last readback.
    const ResampleAhead ahead{cfg->scheme, l + 1, cfg->rng};
    bool resampled = false;
    if ((st = correct_impl(m, pop, t, t_stop, cfg->check_every, cfg->replay ? 0.0 : cfg->D1,
                           rec->group_logwbar + (int64_t)l * cfg->J, &t_new,
                           cfg->replay ? nullptr : &rss, stream, hint,
                           cfg->replay ? nullptr : &ahead, &resampled, &fl_seen)))
      return st;
    // correct_impl has waited for its last decision, which carried the flags
    if (fl_seen > 0 && l > 0) {
      rec->L = l;
      (void)launch_acc_flush(dm.acc, P, s);  // the previous phase's last step
      return set_error(SMC_E_NUMERIC, "numerical flags 0x%x in cycle %d", fl_seen, l);
    }
    last_len = t_new - t;
    evals += P * (t_new - t);
    if (!resampled && (st = smc_resample(m, pop, cfg->scheme, cfg->rng, l + 1, stream)))
      return st;
    int32_t R = cfg->replay ? rec->R[l] : (rss < cfg->D2 ? cfg->kappa * cfg->Rbar : cfg->Rbar);
    if (R < 1) return set_error(SMC_E_INVALID_ARG, "R_l < 1 in cycle %d", l);
    // The Langevin drift needs the posterior gradient at the new date.
    if (cfg->kernel == SMC_KERNEL_MALA && (st = smc_posterior_grad(m, pop, t_new, stream)))
      return st;
    int32_t r = 0;
    for (;;) {
      ++r;
      if (r > cfg->RmaxRec)
        return set_error(SMC_E_INVALID_ARG, "record holds only %d iterations", cfg->RmaxRec);
      double *hl = rec->hchol + ((int64_t)l * cfg->RmaxRec + (r - 1)) * d * d;
      double *mslot = indep ? rec->mean + ((int64_t)l * cfg->RmaxRec + (r - 1)) * d : nullptr;
      int64_t *nacc = rec->n_accept + (int64_t)l * cfg->RmaxRec + (r - 1);
      // The random-walk step folds the proposal scale into its own launch;
      // the partial sums still come from their own kernel.
      const bool fold = !cfg->replay && cfg->kernel == SMC_KERNEL_RW;
      MomFuse fm{};
      if (!cfg->replay) {
        // h starts at 0.5 in each M phase; later iterations first apply the
        // step-size rule to the previous iteration's acceptances.  The
        // independent sampler takes the particle variance unscaled (h = 1).
        ma.mh_reset = indep ? 10 : ((r == 1) ? 5 : 0);
        ma.prev_nacc = (r == 1 || indep) ? nullptr : nacc - 1;
        ma.hchol = hl;
        ma.mean_out = mslot;
        if (fold) {
          int64_t nb = 0;
          if ((st = launch_moment_partials(ma, &fm.part, nb, s))) return st;
          // two step-size slots, alternating, as every block reads the
          // previous iteration's value while block 0 writes this one's
          fm.nb = (int32_t)nb;
          fm.mh_reset = ma.mh_reset;
          fm.mh_in = (r & 1) ? mh + 1 : mh;
          fm.mh_out = (r & 1) ? mh : mh + 1;
          fm.prev_nacc = ma.prev_nacc;
          fm.target_permille = ma.target_permille;
          fm.hchol_out = hl;
          fm.flags = dflags;
        } else if ((st = launch_moments(ma, s))) {
          return st;
        }
      }
      Timed *ev = nullptr;
      const bool bracket = cfg->kernel == SMC_KERNEL_MALA;
      if (rec->mutate_ms && steps % std::max(1, rec->time_every) == 0) {
        timed.emplace_back();
        ev = &timed.back();
        ev->slot = (int64_t)l * cfg->RmaxRec + (r - 1);
        if ((st = timing_event(2 * (timed.size() - 1), &ev->a)) ||
            (st = timing_event(2 * (timed.size() - 1) + 1, &ev->b)))
          return st;
        if (bracket && hipEventRecord(ev->a, s) != hipSuccess)
          return set_error(SMC_E_DEVICE, "event record failed");
      }
      const KernelTimer timer{ev ? ev->a : nullptr, ev ? ev->b : nullptr};
      const KernelTimer *tp = ev && !bracket ? &timer : nullptr;
      if (indep) {
        if ((st = launch_mutate_indep(dm, P, t_new, pop->theta, pop->logprior, pop->loglik,
                                      pop->state, hl, mslot, cfg->rng.seed, cfg->rng.run,
                                      (uint64_t)(l + 1), (uint64_t)r, nacc, nullptr, s, tp)))
          return st;
      } else if (cfg->kernel == SMC_KERNEL_RW) {
        if ((st = launch_mutate_rw(dm, P, t_new, pop->theta, pop->logprior, pop->loglik,
                                   pop->state, fold ? nullptr : hl, cfg->rng.seed, cfg->rng.run,
                                   (uint64_t)(l + 1), (uint64_t)r, nacc, nullptr, s, tp,
                                   fold ? &fm : nullptr)))
          return st;
      } else if ((st = smc_mutate(m, pop, t_new, cfg->kernel, hl, cfg->rng, l + 1, r, nacc,
                                  nullptr, stream))) {
        return st;
      }
      if (ev && bracket && hipEventRecord(ev->b, s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "event record failed");
      // a replayed design computes no moments to carry the counts
      if (cfg->replay && (st = launch_acc_flush(dm.acc, P, s))) return st;
      evals += P * t_new;
      ++steps;
      if (cfg->replay || cfg->stop_rule == 0) {
        if (r >= R) break;
      } else {
        // mean RNE of the test functions; the higher threshold E2 after a C
        // phase that ended at a date of interest (Section 3.3)
        double *rne_d = ws_at<double>(pop, L.small + kSmallRne);
        double *g = ws_at<double>(pop, L.gather);
        double *rep = ws_at<double>(pop, L.small + kSmallCov);  // [G][4] scratch
        if ((st = launch_test_fns(m->dev, P, pop->theta, pop->state, t_new, cfg->test_fn, g, s)) ||
            (st = launch_report(g, pop->J, pop->N, G, ws_at<double>(pop, L.rpart), rep, rne_d,
                                s)))
          return st;
        double rne = 0.0;
        if (hipMemcpyAsync(&rne, rne_d, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return set_error(SMC_E_DEVICE, "reading the RNE failed");
        const bool at_date = t_new == T || t_new == cfg->burn_in ||
                             (cfg->force_every > 0 && t_new % cfg->force_every == 0);
        if (rne > (at_date ? cfg->E2 : cfg->E1) || r >= cfg->Rmax) break;
      }
    }
    if (rec->moments &&
        (st = smc_test_moments(m, pop, t_new, cfg->test_fn, rec->moments + (int64_t)l * G * 4,
                               stream)))
      return st;
    if (!cfg->replay) {
      rec->t_end[l] = t_new;
      rec->R[l] = r;
    }
    rec->rss[l] = rss;
    t = t_new;
    ++l;
    if (t >= T && (st = launch_acc_flush(dm.acc, P, s))) return st;  // the run's last step
    // without the pinned slot (or after the last cycle) the flags are read here
    if (!cfg->replay && (!decision_slot() || t >= T)) {
      int32_t fl = 0;
      if (hipMemcpyAsync(&fl, dflags, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "reading flags failed");
      if (fl) {
        rec->L = l;
        return set_error(SMC_E_NUMERIC, "numerical flags 0x%x in cycle %d", fl, l);
      }
    }
  }
  rec->L = l;
  rec->evals = evals;
  rec->mh_steps = steps;
  if ((st = smc_log_ml(l, pop->J, rec->group_logwbar, rec->log_ml, stream))) return st;
  if (rec->log_score && cfg->burn_in > 0 &&
      (st = smc_log_score(l, pop->J, rec->group_logwbar, rec->t_end, cfg->burn_in, rec->log_score,
                          stream)))
    return st;
  if (!timed.empty()) {
    if (hipStreamSynchronize(s) != hipSuccess)
      return set_error(SMC_E_DEVICE, "synchronising for the timings failed");
    for (auto &e : timed) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess)
        return set_error(SMC_E_DEVICE, "reading a kernel timing failed");
      rec->mutate_ms[e.slot] = ms;
    }
  }
  return SMC_OK;
}

}  // extern "C"

// Device-driven adaptive run (cfg->graph): after the eager set-up (flags,
// counters, the prior draw, k_cycle_init), one captured step -- the C-phase
// chunk (scan, RSS merge, decision, commit), the S phase, Rbar M slots and
// k_cycle_end -- is launched again and again on the stream.  Every decision
// is taken and applied on the device, so the host never waits for one: it
// keeps up to three steps queued, reads the progress word to see how far the
// run is, and stops launching once the run has ended.  The kernels, their
// chunks and counters are those of the host-driven run, so both give the
// same bits.
smc_status run_device_driven(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                             smc_run_record *rec, hipStream_t s) {
  smc_status st;
  const int64_t P = (int64_t)pop->J * pop->N;
  const int32_t d = m->dev.d;
  const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
  const int32_t kR = cfg->kappa * cfg->Rbar;
  if (cfg->kernel != SMC_KERNEL_RW || cfg->replay || cfg->stop_rule != 0 || rec->moments ||
      rec->mutate_ms)
    return set_error(SMC_E_UNSUPPORTED,
                     "device-driven runs take the adaptive random-walk simulator with "
                     "deterministic R_l, without moment reports or timings");
  if (!(cfg->D1 > 0.0) || cfg->Rbar < 1 || cfg->kappa < 1 || kR > cfg->RmaxRec)
    return set_error(SMC_E_INVALID_ARG, "device-driven runs need D1 > 0, Rbar >= 1, kappa >= 1 "
                                        "and kappa Rbar <= RmaxRec");
  if (cfg->Lmax > kGraphMaxCycles)
    return set_error(SMC_E_INVALID_ARG, "device-driven runs record at most %d cycles",
                     kGraphMaxCycles);
  if (d + 1 > kDMax)
    return set_error(SMC_E_UNSUPPORTED, "device-driven runs need d < %d", kDMax);
  const int64_t cap = chunk_capacity(m, pop);
  if (cap < 1) return set_error(SMC_E_WORKSPACE, "workspace has no room for C-phase chunks");
  uint32_t *prog = progress_word();
  if (!prog) return set_error(SMC_E_DEVICE, "no page-locked progress word");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(SMC_E_DEVICE, "hipGetDevice failed");

  CycleDyn *cyc = ws_at<CycleDyn>(pop, L.cyc);
  int64_t *t_end_d = ws_at<int64_t>(pop, L.cyc + align256(sizeof(CycleDyn)));
  int32_t *r_d = reinterpret_cast<int32_t *>(t_end_d + kGraphMaxCycles);
  double *rss_d = reinterpret_cast<double *>(r_d + kGraphMaxCycles);
  int32_t *mh = ws_at<int32_t>(pop, L.small + kSmallMh);
  int32_t *dflags = ws_at<int32_t>(pop, L.small + kSmallFlags);
  StopInfo *stop_dev = ws_at<StopInfo>(pop, L.small + kSmallStop);
  DevModel dm = m->dev;
  dm.cyc = cyc;
  dm.acc = acc_sink(m, pop);

  StepKey key;
  memset(&key, 0, sizeof key);
  key.device = dev;
  key.J = pop->J;
  key.N = pop->N;
  key.check_every = cfg->check_every;
  key.Rbar = cfg->Rbar;
  key.scheme = cfg->scheme;
  key.cap = cap;
  key.D1 = cfg->D1;
  key.dm = dm;
  const void *arrays[14] = {pop->theta, pop->logprior, pop->loglik, pop->state,
                            pop->logw,  pop->grad,     pop->ancestor, pop->ws,
                            rec->n_accept, rec->hchol, rec->group_logwbar, prog,
                            nullptr,    nullptr};
  memcpy(key.arrays, arrays, sizeof arrays);
  thread_local std::vector<StepGraph> graphs;
  hipGraphExec_t exec = nullptr;
  for (const StepGraph &g : graphs)
    if (memcmp(&g.key, &key, sizeof key) == 0) exec = g.exec;
  if (!exec) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
      return set_error(SMC_E_DEVICE, "creating the capture stream failed");
    hipGraph_t graph = nullptr;
    auto capture = [&]() -> smc_status {
      smc_status e;
      double *W = ws_at<double>(pop, L.wcols);
      double *rsscols = ws_at<double>(pop, L.rsscols);
      if ((e = launch_cscan(dm, P, pop->theta, pop->state, pop->logw, 0, 0, cfg->check_every, 0,
                            false, W, cs)) ||
          (e = launch_rss_scan(W, P, cap, rsscols, cs, &cyc->nc)) ||
          (e = launch_find_stop(rsscols, 0, 0, 0, cfg->check_every, 0, cfg->D1, stop_dev, cs,
                                nullptr, 0, nullptr, cyc)) ||
          (e = launch_ccommit(dm, P, pop->theta, pop->state, pop->logw, pop->loglik, 0, 0, false,
                              cs, &stop_dev->t_commit)) ||
          (e = launch_resample(pop->logw, pop->J, pop->N, cfg->scheme, 0, 0, 0, pop->ancestor,
                               ws_at<double>(pop, L.cum), dflags, d, m->dev.S, state_bytes(m),
                               pop->theta, pop->logprior, pop->loglik, pop->state, pop->grad,
                               ws_at<double>(pop, L.gather), cs, nullptr, rec->group_logwbar,
                               cyc)))
        return e;
      for (int32_t k = 1; k <= cfg->Rbar; ++k) {
        MomArgs ma{};
        ma.theta = pop->theta;
        ma.P = P;
        ma.d = d;
        ma.target_permille = 250;
        ma.part = ws_at<double>(pop, L.mpart);
        ma.mh = mh;
        ma.flags = dflags;
        ma.cyc = cyc;
        ma.slot = k;
        ma.acc = dm.acc;  // the moment partials add the previous slot's accept counts
        MomFuse fm{};
        int64_t nb = 0;
        if ((e = launch_moment_partials(ma, &fm.part, nb, cs))) return e;
        fm.nb = (int32_t)nb;
        fm.target_permille = 250;
        fm.mh_out = mh;  // the kernel picks the slot pair and rule for its iteration
        fm.hchol_out = rec->hchol;
        fm.flags = dflags;
        if ((e = launch_mutate_rw(dm, P, m->dev.T, pop->theta, pop->logprior, pop->loglik,
                                  pop->state, nullptr, 0, 0, 0, (uint64_t)k, rec->n_accept,
                                  nullptr, cs, nullptr, &fm)))
          return e;
      }
      return launch_cycle_end(cyc, t_end_d, r_d, rss_d, dflags, prog, dm.acc, cs);
    };
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return set_error(SMC_E_DEVICE, "beginning the step capture failed");
    }
    st = capture();
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return st ? st : set_error(SMC_E_DEVICE, "capturing the step failed");
    }
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return set_error(SMC_E_DEVICE, "instantiating the step failed");
    if (graphs.size() >= kStepGraphs) {
      (void)hipGraphExecDestroy(graphs.front().exec);
      graphs.erase(graphs.begin());
    }
    graphs.push_back(StepGraph{key, exec});
  }

  // eager set-up, as the host-driven run does it
  if ((st = fill_i32(dflags, 1, 0, s)) ||
      (st = fill_i64(rec->n_accept, (int64_t)cfg->Lmax * cfg->RmaxRec, 0, s)) ||
      (st = fill_i64(reinterpret_cast<int64_t *>(dm.acc.pending), 1, 0, s)) ||
      (st = smc_init_from_prior(m, pop, cfg->rng, s)))
    return st;
  CycleDyn init{};
  init.seed = cfg->rng.seed;
  init.run = cfg->rng.run;
  init.T = m->dev.T;
  init.P = P;
  init.check_every = cfg->check_every;
  init.force_every = cfg->force_every;
  init.burn_in = cfg->burn_in;
  init.cap = cap;
  init.D2 = cfg->D2;
  init.Rbar = cfg->Rbar;
  init.kR = kR;
  init.Lmax = cfg->Lmax;
  init.rec_stride = cfg->RmaxRec;
  init.m_slots = cfg->Rbar;
  init.J = pop->J;
  __atomic_store_n(prog, 0u, __ATOMIC_RELEASE);
  if ((st = launch_cycle_init(cyc, init, s))) return st;

  // Steps in flight: at most kAhead beyond the last one seen to finish.  The
  // stream is polled every millisecond while the word stands still; once all
  // its work has completed, the word gets 10 more ms before the run fails.
  // Every step but the last few advances the committed date or runs M
  // iterations, so a run takes at most T chunks and kappa steps of M slots
  // per cycle: more launches than that mean the run is not progressing.
  constexpr uint32_t kAhead = 3;
  const int64_t max_steps = m->dev.T + (int64_t)cfg->Lmax * cfg->kappa + kAhead + 1;
  uint32_t launched = 0, word = 0;
  using clock = std::chrono::steady_clock;
  for (;;) {
    word = __atomic_load_n(prog, __ATOMIC_ACQUIRE);
    if (word & 3u) break;
    if (launched - (word >> 2) < kAhead) {
      if ((int64_t)launched >= max_steps) {
        (void)hipStreamSynchronize(s);
        return set_error(SMC_E_DEVICE, "the device-driven run did not end in %lld steps",
                         (long long)max_steps);
      }
      if (hipGraphLaunch(exec, s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "launching a step failed");
      ++launched;
      continue;
    }
    auto next_poll = clock::now() + std::chrono::milliseconds(1);
    clock::time_point idle_since{};
    bool idle = false;
    const uint32_t seen = word;
    while ((word = __atomic_load_n(prog, __ATOMIC_ACQUIRE)) == seen) {
      const auto now = clock::now();
      if (now < next_poll) continue;
      next_poll = now + std::chrono::milliseconds(1);
      if (!idle) {
        const hipError_t q = hipStreamQuery(s);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return set_error(SMC_E_DEVICE, "a step failed: %s",
                                              hipGetErrorString(q));
        idle = true;
        idle_since = now;
      } else if (now - idle_since > std::chrono::milliseconds(10)) {
        return set_error(SMC_E_DEVICE, "the device-driven run stopped reporting progress");
      }
    }
  }
  CycleDyn fin{};
  if (hipMemcpyAsync(&fin, cyc, sizeof fin, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "reading the run's state failed");
  const int32_t Ln = fin.l;
  if (Ln > 0 &&
      (hipMemcpyAsync(rec->t_end, t_end_d, Ln * sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
           hipSuccess ||
       hipMemcpyAsync(rec->R, r_d, Ln * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipMemcpyAsync(rec->rss, rss_d, Ln * sizeof(double), hipMemcpyDeviceToHost, s) !=
           hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    return set_error(SMC_E_DEVICE, "reading the record failed");
  rec->L = Ln;
  rec->evals = fin.evals;
  rec->mh_steps = fin.steps;
  if (fin.err == 2) return set_error(SMC_E_NUMERIC, "numerical flags 0x%x in cycle %d", fin.flags, Ln);
  if (fin.err) return set_error(SMC_E_INVALID_ARG, "record holds only %d cycles", cfg->Lmax);
  if ((st = smc_log_ml(Ln, pop->J, rec->group_logwbar, rec->log_ml, s))) return st;
  if (rec->log_score && cfg->burn_in > 0 &&
      (st = smc_log_score(Ln, pop->J, rec->group_logwbar, rec->t_end, cfg->burn_in,
                          rec->log_score, s)))
    return st;
  return SMC_OK;
}

extern "C" {

smc_status smc_hybrid_report(const smc_run_record *rec1, const smc_run_record *rec2,
                             double *out, void *stream) {
  if (!rec1 || !rec2 || !out || !rec1->log_ml || !rec2->log_ml)
    return set_error(SMC_E_INVALID_ARG, "NULL record, estimate or output");
  hipStream_t s = as_stream(stream);
  const bool scores = rec1->log_score && rec2->log_score;
  double v[4][3] = {};
  if (hipMemcpyAsync(v[0], rec1->log_ml, 3 * sizeof(double), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(v[1], rec2->log_ml, 3 * sizeof(double), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      (scores &&
       (hipMemcpyAsync(v[2], rec1->log_score, 3 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(v[3], rec2->log_score, 3 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess)) ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "reading the estimates failed");
  const auto z = [](const double *a, const double *b) {
    return fabs(a[0] - b[0]) / hypot(a[1], b[1]);
  };
  out[0] = z(v[0], v[1]);
  out[1] = scores ? z(v[2], v[3]) : NAN;
  return SMC_OK;
}

smc_status smc_run_hybrid(const smc_model *m, smc_particles *pop, const smc_run_config *cfg,
                          uint64_t seed2, smc_run_record *rec1, smc_run_record *rec2,
                          double *seconds, void *stream) {
  smc_status st;
  if ((st = check_model(m))) return st;
  if (!cfg || !rec1 || !rec2) return set_error(SMC_E_INVALID_ARG, "NULL config or record");
  if (cfg->replay) return set_error(SMC_E_INVALID_ARG, "step 1 of the hybrid method adapts");
  if (!rec2->t_end || !rec2->R || !rec2->hchol || !rec1->hchol)
    return set_error(SMC_E_INVALID_ARG, "a record array is NULL");
  hipStream_t s = as_stream(stream);
  const int32_t d = m->dev.d;
  using clock = std::chrono::steady_clock;
  auto t0 = clock::now();
  if ((st = smc_run(m, pop, cfg, rec1, stream))) return st;
  if (hipStreamSynchronize(s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "hybrid: synchronising after step 1 failed");
  auto t1 = clock::now();
  // retain the design of step 1 and replay it with the new key
  const int32_t L = rec1->L;
  for (int32_t l = 0; l < L; ++l) {
    rec2->t_end[l] = rec1->t_end[l];
    rec2->R[l] = rec1->R[l];
  }
  if (hipMemcpyAsync(rec2->hchol, rec1->hchol,
                     (size_t)L * cfg->RmaxRec * d * d * sizeof(double), hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "hybrid: copying the design failed");
  if (cfg->kernel == SMC_KERNEL_INDEPENDENT &&
      (!rec1->mean || !rec2->mean ||
       hipMemcpyAsync(rec2->mean, rec1->mean, (size_t)L * cfg->RmaxRec * d * sizeof(double),
                      hipMemcpyDeviceToDevice, s) != hipSuccess))
    return set_error(SMC_E_DEVICE, "hybrid: copying the sampler's means failed");
  smc_run_config c2 = *cfg;
  c2.replay = 1;
  c2.rng.seed = seed2;
  if ((st = smc_run(m, pop, &c2, rec2, stream))) return st;
  if (hipStreamSynchronize(s) != hipSuccess)
    return set_error(SMC_E_DEVICE, "hybrid: synchronising after step 2 failed");
  auto t2 = clock::now();
  if (seconds) {
    seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    seconds[1] = std::chrono::duration<double>(t2 - t1).count();
  }
  return SMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ batched runs --
#include "batch.h"

extern "C" {

size_t smc_batch_ws_bytes(int32_t n_runs) {
  if (n_runs < 1 || n_runs > kMaxBatch) return 0;
  return align256((size_t)n_runs * sizeof(BatchStatic)) + 256;
}

smc_status smc_run_batch(int32_t n, const smc_model *const *models, smc_particles *const *pops,
                         const smc_run_config *cfgs, smc_run_record *recs, void *bws,
                         size_t bws_bytes, int32_t waves, smc_batch_timing *timing,
                         void *stream) {
  smc_status st;
  if (timing) {
    timing->launches = 0;
    if (timing->capacity < 0 || (timing->capacity > 0 && (!timing->ms || !timing->evals)))
      return set_error(SMC_E_INVALID_ARG, "batch timing arrays");
  }
  if (n < 1 || n > kMaxBatch)
    return set_error(SMC_E_INVALID_ARG, "a batch holds 1..%d runs", kMaxBatch);
  if (!models || !pops || !cfgs || !recs || !bws)
    return set_error(SMC_E_INVALID_ARG, "NULL batch argument");
  if (bws_bytes < smc_batch_ws_bytes(n) || (reinterpret_cast<uintptr_t>(bws) & 255))
    return set_error(SMC_E_WORKSPACE, "batch workspace too small or misaligned");
  hipStream_t s = as_stream(stream);
  const bool replay = cfgs[0].replay != 0;
  const int32_t kernel = cfgs[0].kernel;
  const bool mala = kernel == SMC_KERNEL_MALA;
  int32_t family = -1;
  for (int i = 0; i < n; ++i) {
    const smc_model *m = models[i];
    if ((st = check_model(m)) || (st = check_pop(m, pops[i]))) return st;
    const smc_run_config &c = cfgs[i];
    const smc_run_record &r = recs[i];
    if (c.J != pops[i]->J || c.N != pops[i]->N)
      return set_error(SMC_E_INVALID_ARG, "run %d: config and population shapes differ", i);
    if (!r.t_end || !r.R || !r.rss || !r.n_accept || !r.hchol || !r.group_logwbar || !r.log_ml)
      return set_error(SMC_E_INVALID_ARG, "run %d: a record array is NULL", i);
    if (c.Lmax < 1 || c.RmaxRec < 1 || c.check_every < 1 || c.force_every < 0)
      return set_error(SMC_E_INVALID_ARG, "run %d: bad record capacity", i);
    if ((c.kernel != SMC_KERNEL_RW && c.kernel != SMC_KERNEL_MALA) || c.stop_rule != 0)
      return set_error(SMC_E_UNSUPPORTED,
                       "batched runs use the random walk or the Langevin step and fixed R_l");
    if (c.kernel != kernel)
      return set_error(SMC_E_INVALID_ARG, "the runs of a batch share one Metropolis kernel");
    if (mala) {
      if (!pops[i]->grad)
        return set_error(SMC_E_INVALID_ARG, "run %d: the Langevin kernel needs pop->grad", i);
      const WsLayout L = ws_layout(m->dev, pops[i]->J, pops[i]->N);
      const size_t need =
          L.wcols + adjoint_ckpt_bytes(m->dev, (int64_t)pops[i]->J * pops[i]->N, m->dev.T);
      if (pops[i]->ws_bytes < need)
        return set_error(SMC_E_WORKSPACE, "run %d: the Langevin kernel needs %zu workspace bytes",
                         i, need);
    }
    if (c.burn_in != 0 || r.moments || r.log_score || c.graph != 0)
      return set_error(SMC_E_UNSUPPORTED, "batched runs: no burn-in, moment reports or log score");
    if ((c.replay != 0) != replay)
      return set_error(SMC_E_INVALID_ARG, "all runs of a batch adapt, or all replay");
    const DevModel &dm = m->dev;
    const bool ok_model = dm.kind == SMC_MODEL_EGARCH &&
                          ((dm.K == 1 && dm.shock == SMC_SHOCK_GAUSS) ||
                           (dm.K == 2 && dm.shock == SMC_SHOCK_STUDENT_T));
    if (!ok_model)
      return set_error(SMC_E_UNSUPPORTED, "batched runs: EGARCH(1) Gaussian or EGARCH(2)-t");
    const int32_t fam = dm.prec == SMC_FP32 ? kFamilyFp32 : kFamilyFp64;
    if (family >= 0 && fam != family)
      return set_error(SMC_E_UNSUPPORTED, "batched runs share one precision");
    family = fam;
  }
  // FP32 random-walk batches take their first model's launch shape; the item
  // (a block of particles of one run) is that many particles
  const bool shaped = family == kFamilyFp32 && !mala;
  const int32_t bshape = shaped ? models[0]->dev.block : 0;
  const int32_t ushape = shaped ? models[0]->dev.unroll : 0;
  const int64_t item = bshape ? bshape : 64;
  BatchStatic *table = reinterpret_cast<BatchStatic *>(bws);
  unsigned int *queue = reinterpret_cast<unsigned int *>(reinterpret_cast<char *>(bws) +
                                                         align256((size_t)n * sizeof(BatchStatic)));
  // Static table, written by a kernel from its arguments.
  BatchStaticArgs sa{};
  sa.dst = table;
  sa.n = n;
  for (int i = 0; i < n; ++i) {
    const DevModel &dm = models[i]->dev;
    const WsLayout L = ws_layout(dm, pops[i]->J, pops[i]->N);
    BatchStatic &b = sa.src[i];
    b.theta = pops[i]->theta;
    b.logprior = pops[i]->logprior;
    b.loglik = pops[i]->loglik;
    b.state = pops[i]->state;
    b.part = ws_at<double>(pops[i], L.mpart);
    b.mh = ws_at<int32_t>(pops[i], L.small + kSmallMh);
    b.flags = ws_at<int32_t>(pops[i], L.small + kSmallFlags);
    b.y = dm.prec == SMC_FP32 ? static_cast<const void *>(dm.y32) : static_cast<const void *>(dm.y);
    b.grad = mala ? pops[i]->grad : nullptr;
    b.ckpt = mala ? static_cast<void *>(ws_at<char>(pops[i], L.wcols)) : nullptr;
    b.seed = cfgs[i].rng.seed;
    b.run = cfgs[i].rng.run;
    b.P = (int64_t)pops[i]->J * pops[i]->N;
    b.tag = dm.K == 1 ? 0 : 1;
    b.d = dm.d;
  }
  if ((st = launch_batch_static(sa, s))) return st;

  enum Phase { kCStart, kCNext, kCPend, kM, kDone };
  struct Run {
    Phase ph = kCStart;
    int64_t t = 0;        // start of the current cycle
    int64_t tc = 0;       // C-phase position
    int64_t t_stop = 0;   // this C phase's last possible date
    int64_t t_new = 0;    // end of the C phase
    int64_t chunk = 16, last_len = 0;
    bool zero_first = true;
    std::vector<int64_t> dates;
    int32_t l = 0, r = 0, R = 0;
    double rss = NAN;
    int64_t evals = 0, steps = 0;
  };
  std::vector<Run> run(n);
  for (int i = 0; i < n; ++i) {
    const WsLayout L = ws_layout(models[i]->dev, pops[i]->J, pops[i]->N);
    if ((st = fill_i32(ws_at<int32_t>(pops[i], L.small + kSmallFlags), 1, 0, s)) ||
        (st = fill_i64(recs[i].n_accept, (int64_t)cfgs[i].Lmax * cfgs[i].RmaxRec, 0, s)) ||
        (st = smc_init_from_prior(models[i], pops[i], cfgs[i].rng, stream)))
      return st;
  }
  // Pinned readback area of the adaptive C phases: per run, the RSS of the
  // chunk's checked dates followed by the run's flags word (a replay reads nothing back, so
  // it can be captured).  One area per host thread, grown on demand and kept.
  constexpr size_t kRow = kMaxChunk + 1;  // doubles per run
  double *host_rss = nullptr;
  if (!replay && !(host_rss = batch_readback((size_t)n * kRow)))
    return set_error(SMC_E_DEVICE, "pinned host buffer for the batch failed");
  auto flags_of = [&](int i) -> int32_t * {
    return reinterpret_cast<int32_t *>(host_rss + (size_t)i * kRow + kMaxChunk);
  };
  // per-launch timing of the persistent M step
  struct Timed {
    hipEvent_t a = nullptr, b = nullptr;
  };
  std::vector<Timed> timed;

  auto end_c_phase = [&](int i) -> smc_status {
    Run &u = run[i];
    const smc_model *m = models[i];
    smc_particles *pop = pops[i];
    const smc_run_config &c = cfgs[i];
    smc_status e;
    if ((e = launch_group_logwbar(pop->logw, pop->J, pop->N,
                                  recs[i].group_logwbar + (int64_t)u.l * c.J, s)))
      return e;
    if ((e = smc_resample(m, pop, c.scheme, c.rng, u.l + 1, stream))) return e;
    // the Langevin drift needs the posterior gradient at the new date
    if (mala && (e = smc_posterior_grad(m, pop, u.tc, stream))) return e;
    u.t_new = u.tc;
    u.last_len = u.t_new - u.t;
    u.R = c.replay ? recs[i].R[u.l] : (u.rss < c.D2 ? c.kappa * c.Rbar : c.Rbar);
    if (u.R < 1 || u.R > c.RmaxRec)
      return set_error(SMC_E_INVALID_ARG, "run %d: R_l out of the record's range", i);
    u.r = 0;
    u.ph = kM;
    return SMC_OK;
  };

  for (;;) {
    bool all_done = true;
    for (int i = 0; i < n; ++i) all_done = all_done && run[i].ph == kDone;
    if (all_done) break;
    std::vector<int> pend;
    // (a) C phases: start or continue a chunk
    for (int i = 0; i < n; ++i) {
      Run &u = run[i];
      const smc_run_config &c = cfgs[i];
      const smc_model *m = models[i];
      smc_particles *pop = pops[i];
      const int64_t P = (int64_t)pop->J * pop->N;
      const int64_t T = m->dev.T;
      if (u.ph == kCStart) {
        if (u.l >= c.Lmax) return set_error(SMC_E_INVALID_ARG, "run %d: record full", i);
        u.t_stop = T;
        if (c.force_every > 0)
          u.t_stop = std::min(u.t_stop, (u.t / c.force_every + 1) * c.force_every);
        if (c.replay) {
          u.t_stop = recs[i].t_end[u.l];
          if (u.t_stop <= u.t || u.t_stop > T)
            return set_error(SMC_E_INVALID_ARG, "run %d: replayed date out of order", i);
        }
        u.tc = u.t;
        u.zero_first = true;
        if (c.replay) {
          if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik,
                                   u.t, u.t_stop, true, s)))
            return st;
          u.evals += P * (u.t_stop - u.t);
          u.tc = u.t_stop;
          if ((st = end_c_phase(i))) return st;
          continue;
        }
        const int64_t cap = chunk_capacity(m, pop);
        if (cap < 1) return set_error(SMC_E_WORKSPACE, "run %d: no room for C-phase chunks", i);
        u.chunk = std::min<int64_t>(cap, std::max<int64_t>(16, 2 * u.last_len + 16));
        u.ph = kCNext;
      }
      if (u.ph == kCNext) {
        const int64_t t1 = std::min(u.tc + u.chunk, u.t_stop);
        u.dates.clear();
        for (int64_t q = u.tc + 1; q <= t1; ++q)
          if (q % c.check_every == 0 || q == u.t_stop) u.dates.push_back(q);
        const WsLayout L = ws_layout(m->dev, pop->J, pop->N);
        if (u.dates.empty()) {
          if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik,
                                   u.tc, t1, u.zero_first, s)))
            return st;
          u.evals += P * (t1 - u.tc);
          u.zero_first = false;
          u.tc = t1;
          continue;
        }
        if ((st = launch_cscan(m->dev, P, pop->theta, pop->state, pop->logw, u.tc, t1,
                               c.check_every, u.t_stop, u.zero_first, ws_at<double>(pop, L.wcols),
                               s)) ||
            (st = launch_rss_scan(ws_at<double>(pop, L.wcols), P, (int64_t)u.dates.size(),
                                  ws_at<double>(pop, L.rsscols), s)))
          return st;
        if (hipMemcpyAsync(host_rss + (size_t)i * kRow, ws_at<double>(pop, L.rsscols),
                           u.dates.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipMemcpyAsync(flags_of(i), ws_at<int32_t>(pop, L.small + kSmallFlags),
                           sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
          return set_error(SMC_E_DEVICE, "run %d: RSS readback failed", i);
        u.ph = kCPend;
        pend.push_back(i);
      }
    }
    // (b) one M iteration of every run in its M phase
    std::vector<int> act;
    for (int i = 0; i < n; ++i)
      if (run[i].ph == kM) act.push_back(i);
    if (!act.empty()) {
      std::stable_sort(act.begin(), act.end(),
                       [&](int a, int b) { return run[a].t_new > run[b].t_new; });
      BatchArgs ba{};
      ba.runs = table;
      ba.queue = queue;
      ba.n_active = (int32_t)act.size();
      ba.target_permille = mala ? 574 : 250;
      ba.kernel = kernel;
      int32_t mut = 0, mom = 0;
      for (size_t q = 0; q < act.size(); ++q) {
        const int i = act[q];
        Run &u = run[i];
        const smc_run_config &c = cfgs[i];
        const int64_t P = (int64_t)pops[i]->J * pops[i]->N;
        const int32_t d = models[i]->dev.d;
        BatchDyn &dy = ba.dyn[q];
        const int64_t slot = (int64_t)u.l * c.RmaxRec + u.r;
        dy.hchol = recs[i].hchol + slot * d * d;
        dy.n_accept = reinterpret_cast<unsigned long long *>(recs[i].n_accept + slot);
        dy.prev_nacc = u.r == 0 ? nullptr : recs[i].n_accept + slot - 1;
        dy.t = u.t_new;
        dy.idx = i;
        dy.cycle = u.l + 1;
        dy.iter = u.r + 1;
        dy.mh_reset = u.r == 0 ? 5 : 0;
        dy.mut_begin = mut;
        mut += (int32_t)((P + item - 1) / item);
        int64_t ch = 0, nb = 0;
        moment_partition(P, d, ch, nb);
        dy.mom_begin = mom;
        dy.mom_nb = (int32_t)nb;
        dy.mom_chunk = (int32_t)ch;
        mom += (int32_t)nb;
        u.evals += P * u.t_new;
        u.steps += 1;
      }
      ba.n_mut_items = mut;
      ba.n_mom_items = mom;
      KernelTimer kt{};
      const bool timed_launch = timing && timing->launches < timing->capacity;
      if (timed_launch) {
        const int32_t k = timing->launches;
        timed.emplace_back();
        if ((st = timing_event(2 * (size_t)k, &timed.back().a)) ||
            (st = timing_event(2 * (size_t)k + 1, &timed.back().b)))
          return st;
        kt = KernelTimer{timed.back().a, timed.back().b};
        int64_t e1 = 0, e2 = 0;
        for (int i : act) {
          const int64_t ev = (int64_t)pops[i]->J * pops[i]->N * run[i].t_new;
          if (models[i]->dev.K == 1) e1 += ev;
          else e2 += ev;
        }
        timing->evals[2 * k] = e1;
        timing->evals[2 * k + 1] = e2;
        timing->launches = k + 1;
      }
      if ((st = launch_batch_m(ba, !replay, family, waves > 0 ? waves : 2048, s,
                               timed_launch ? &kt : nullptr, bshape, ushape)))
        return st;
      for (int i : act) {
        Run &u = run[i];
        if (++u.r >= u.R) {
          if (!cfgs[i].replay) {
            recs[i].t_end[u.l] = u.t_new;
            recs[i].R[u.l] = u.R;
          }
          recs[i].rss[u.l] = u.rss;
          u.t = u.t_new;
          ++u.l;
          u.ph = u.t < models[i]->dev.T ? kCStart : kDone;
        }
      }
    }
    // (c) one synchronisation for every pending C-phase chunk
    if (!pend.empty()) {
      if (hipStreamSynchronize(s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "batch synchronisation failed");
      for (int i : pend) {
        Run &u = run[i];
        const smc_run_config &c = cfgs[i];
        const smc_model *m = models[i];
        smc_particles *pop = pops[i];
        const int64_t P = (int64_t)pop->J * pop->N;
        const double *hr = host_rss + (size_t)i * kRow;
        // a run whose S or M phase raised a numerical flag stops the batch
        // at its next C-phase readback, as smc_run stops
        if (*flags_of(i)) {
          recs[i].L = u.l;
          return set_error(SMC_E_NUMERIC, "run %d: numerical flags 0x%x in cycle %d", i,
                           *flags_of(i), u.l);
        }
        const int64_t nc = (int64_t)u.dates.size();
        int64_t stop_col = -1;
        for (int64_t q = 0; q < nc; ++q)
          if (hr[q] < c.D1) {
            stop_col = q;
            break;
          }
        const int64_t t1 = u.dates.back() < u.t_stop ? std::min(u.tc + u.chunk, u.t_stop)
                                                      : u.t_stop;
        const int64_t t_commit = stop_col >= 0 ? u.dates[stop_col] : t1;
        if ((st = launch_ccommit(m->dev, P, pop->theta, pop->state, pop->logw, pop->loglik,
                                 u.tc, t_commit, u.zero_first, s)))
          return st;
        u.evals += P * (t_commit - u.tc);
        u.zero_first = false;
        u.rss = stop_col >= 0 ? hr[stop_col] : hr[nc - 1];
        u.tc = t_commit;
        if (stop_col >= 0 || u.tc >= u.t_stop) {
          if ((st = end_c_phase(i))) return st;
        } else {
          u.chunk = std::min(2 * u.chunk, chunk_capacity(m, pop));
          u.ph = kCNext;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    recs[i].L = run[i].l;
    recs[i].evals = run[i].evals;
    recs[i].mh_steps = run[i].steps;
    if ((st = smc_log_ml(run[i].l, pops[i]->J, recs[i].group_logwbar, recs[i].log_ml, stream)))
      return st;
  }
  if (!timed.empty()) {
    if (hipStreamSynchronize(s) != hipSuccess)
      return set_error(SMC_E_DEVICE, "synchronising for the batch timings failed");
    for (size_t k = 0; k < timed.size(); ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, timed[k].a, timed[k].b) != hipSuccess)
        return set_error(SMC_E_DEVICE, "reading a batch timing failed");
      timing->ms[k] = ms;
    }
  }
  if (!replay) {
    // numerical flags of every run (adaptive batches synchronise anyway)
    for (int i = 0; i < n; ++i) {
      int32_t fl = 0;
      const WsLayout L = ws_layout(models[i]->dev, pops[i]->J, pops[i]->N);
      if (hipMemcpyAsync(&fl, ws_at<int32_t>(pops[i], L.small + kSmallFlags), sizeof fl,
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return set_error(SMC_E_DEVICE, "reading flags failed");
      if (fl) return set_error(SMC_E_NUMERIC, "run %d: numerical flags 0x%x", i, fl);
    }
  }
  return SMC_OK;
}

}  // extern "C"
