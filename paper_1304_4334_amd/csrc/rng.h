// Counter-based random numbers on the device: Philox4x64-10 (Salmon, Moraes,
// Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
//
// Every draw is addressed by (key = (seed, run), counter = (index, cycle,
// iteration, purpose | block << 8)), so a particle's draws do not depend on
// how particles are spread over waves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

struct U64x4 {
  uint64_t x0, x1, x2, x3;
};

// The 128-bit product a b as (hi, lo) from four 32 x 32 -> 64-bit
// multiply-adds: with a = a1 2^32 + a0 and b likewise, t = a0 b1 + hi(a0 b0)
// and u = a1 b0 + lo(t) cannot overflow, lo = lo(u) 2^32 + lo(a0 b0) and
// hi = a1 b1 + hi(t) + hi(u).
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;
  hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
  lo = (u << 32) | (uint32_t)p00;
}

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul_wide(kM0, c.x0, hi0, lo0);
    mul_wide(kM1, c.x2, hi1, lo1);
    c = U64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ U64x4 draw4(uint64_t seed, uint64_t run, uint64_t c0, uint64_t c1,
                                       uint64_t c2, uint64_t c3) {
  return philox4x64_10(U64x4{c0, c1, c2, c3}, seed, run);
}

// Top 53 bits as a double in [0,1), (0,1] and (0,1).
__device__ __forceinline__ double u01_co(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double u01_oc(uint64_t x) {
  return ((double)(x >> 11) + 1.0) * 0x1.0p-53;
}
__device__ __forceinline__ double u01_oo(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

// Box-Muller pair from two words: r = sqrt(-2 log u1) with u1 in (0,1],
// angle 2 pi u2 with u2 in [0,1).
__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double &z0, double &z1) {
  const double r = sqrt(-2.0 * log(u01_oc(a)));
  double s, c;
  sincospi(2.0 * u01_co(b), &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// n standard normals: block q (counter word 3 = purpose | q << 8) yields
// z[4q..4q+3] from its words (x0,x1) and (x2,x3).
template <int N>
__device__ __forceinline__ void normals(uint64_t seed, uint64_t run, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t purpose, double (&z)[N], int n) {
#pragma unroll
  for (int q = 0; 4 * q < N; ++q) {
    if (4 * q < n) {
      const U64x4 w = draw4(seed, run, c0, c1, c2, purpose | ((uint64_t)q << 8));
      double a, b, c, d;
      box_muller(w.x0, w.x1, a, b);
      box_muller(w.x2, w.x3, c, d);
      z[4 * q] = a;
      if (4 * q + 1 < N) z[4 * q + 1] = b;
      if (4 * q + 2 < N) z[4 * q + 2] = c;
      if (4 * q + 3 < N) z[4 * q + 3] = d;
    }
  }
}

}  // namespace smc
