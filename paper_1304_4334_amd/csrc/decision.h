// The C-phase stopping decision as the device hands it to the host thread
// that waits for it (plain C++, shared by the device kernel that writes it
// and the host code that reads it).
#pragma once

#include <stdint.h>
#include <string.h>

namespace smc {

// A C-phase chunk's outcome, decided on the device: the date the weights are
// committed to (the first checked date whose RSS fell below the threshold, or
// the chunk's end), the RSS there, whether it fell below, and whether the
// phase ends with this chunk (it fell below, or the chunk reached the
// phase's last date).
struct StopInfo {
  int64_t t_commit;
  double rss;
  int32_t below;
  int32_t ends;
};

// The same decision, with the workspace's flags word, in page-locked
// coherent host memory.  Six 32-bit payload words, each paired with the
// call's sequence number in one naturally aligned 8-byte word, so the host
// never relies on a store wider than 8 bytes landing whole: it accepts the
// slot only when all six pairs carry its sequence number.  The device writes
// the 48 bytes as three 16-byte stores.
//   payload 0, 1: t_commit (low, high); 2, 3: rss bits (low, high);
//   4: flags; 5: bit 0 the phase ends, bit 1 the RSS fell below.
struct alignas(16) DecisionSlot {
  uint32_t w[12];  // w[2i] = sequence number, w[2i + 1] = payload i
};

// Reads the slot once: true when every pair carries `seq`, two consecutive
// reads agree, and the decision is consistent with the chunk (t, t1] that
// was evaluated (t < t_commit <= t1, 0 <= rss <= 1 up to rounding, "fell
// below" only with "ends").  Anything else is a slot still being written,
// or not yet written, for this call.
inline bool read_decision(const volatile DecisionSlot *slot, uint32_t seq, int64_t t, int64_t t1,
                          StopInfo *out, int32_t *flags) {
  uint32_t a[12], b[12];
  for (int i = 0; i < 12; ++i) a[i] = slot->w[i];
  for (int i = 0; i < 12; ++i) b[i] = slot->w[i];
  for (int i = 0; i < 12; ++i)
    if (a[i] != b[i] || ((i & 1) == 0 && a[i] != seq)) return false;
  const int64_t tc = (int64_t)(((uint64_t)a[3] << 32) | a[1]);
  const uint64_t rb = ((uint64_t)a[7] << 32) | a[5];
  double rss;
  memcpy(&rss, &rb, sizeof rss);
  const uint32_t eb = a[11];
  if (!(tc > t && tc <= t1)) return false;
  if (!(rss >= 0.0 && rss <= 1.0 + 1e-12)) return false;  // NaN fails too
  if (eb > 3u || ((eb & 2u) && !(eb & 1u))) return false;
  out->t_commit = tc;
  out->rss = rss;
  out->ends = (int32_t)(eb & 1u);
  out->below = (int32_t)((eb >> 1) & 1u);
  if (flags) *flags = (int32_t)a[9];
  return true;
}

}  // namespace smc
