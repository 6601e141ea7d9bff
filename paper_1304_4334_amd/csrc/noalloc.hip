// The particle moments (pooled mean, variance and the scaled Cholesky factor
// of the random-walk proposal) for callers that cannot allocate device
// memory: the same kernels as smc_particle_moments, with their scratch (the
// moment partials and the flags word) in a file-scope device array instead
// of the caller's workspace.
//
// Every GPU the library runs on holds its own copy of the array until the
// process ends.  Its device address is looked up once per device, with that
// device current, at the entry point's first call there; host code uses only
// that address (the array's name is a host-side stand-in).  Calls on one GPU
// share the array: overlapping calls race, and each call clears the flags
// word it uses before its kernels run.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"
#include "launch.h"
#include "smc.h"

namespace smc {

namespace {

// Partials: at most kMomBlocks matrices of 32 x 32 doubles plus their sum
// (the 32-wide path), then the flags word.
constexpr size_t kPartBytes = (size_t)(kMomBlocks + 1) * 32 * 32 * sizeof(double);
constexpr size_t kFlagsOff = kPartBytes;
static_assert(kPartBytes + 256 == SMC_MOMENTS_SCRATCH_BYTES, "header constant");

static __device__ __align__(256) char scratch[SMC_MOMENTS_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
char *g_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of the array, or NULL (error
// recorded).
char *scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(SMC_E_DEVICE, "no current device (or device index %d beyond %d)", dev,
              kMaxDevices - 1);
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(SMC_E_DEVICE, "looking up the static scratch on device %d: %s", dev,
                hipGetErrorString(e));
      return nullptr;
    }
    g_ptr[dev] = static_cast<char *>(p);
  }
  return g_ptr[dev];
}

}  // namespace

}  // namespace smc

using namespace smc;

extern "C" smc_status smc_particle_moments_noalloc(const smc_model *m, const smc_particles *pop,
                                                   const int32_t *mh, double *mean, double *cov,
                                                   double *hchol, void *stream) {
  if (!m) return set_error(SMC_E_INVALID_ARG, "model handle is NULL");
  if (!pop || !pop->theta) return set_error(SMC_E_INVALID_ARG, "particles or theta is NULL");
  if (pop->J < 2 || pop->N < 2) return set_error(SMC_E_INVALID_ARG, "need J >= 2 and N >= 2");
  if ((int64_t)pop->J * pop->N > (int64_t)1 << 30)
    return set_error(SMC_E_UNSUPPORTED, "more than 2^30 particles");
  if (!mh || !hchol) return set_error(SMC_E_INVALID_ARG, "mh and hchol are required");
  const int64_t P = (int64_t)pop->J * pop->N;
  const int32_t d = m->dev.d;
  if (d + 1 > kDMax) return set_error(SMC_E_UNSUPPORTED, "moments need d < %d", kDMax);
  int64_t chunk = 0, nb = 0;
  moment_partition(P, d, chunk, nb);
  const size_t W = d + 1 <= 16 ? 16 : 32;
  const size_t need = (size_t)(nb + 1) * W * W * sizeof(double);
  if (nb > kMomBlocks || need > kPartBytes)
    return set_error(SMC_E_WORKSPACE, "moments of %lld particles need %zu scratch bytes > %zu",
                     (long long)P, need, kPartBytes);
  char *base = scratch_for_current_device();
  if (!base) return SMC_E_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t *flags = reinterpret_cast<int32_t *>(base + kFlagsOff);
  smc_status st;
  if ((st = fill_i32(flags, 1, 0, s))) return st;
  MomArgs a{};
  a.theta = pop->theta;
  a.P = P;
  a.d = d;
  a.part = reinterpret_cast<double *>(base);
  a.mh = const_cast<int32_t *>(mh);
  a.mean_out = mean;
  a.cov_out = cov;
  a.hchol = hchol;
  a.flags = flags;
  return launch_moments(a, s);
}
