// Deterministic reductions and scans (fixed combination order; no
// floating-point atomics): within a wave through DPP lane moves, and over a
// block of kBlock = 256 threads (4 waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "common.h"

namespace smc {

template <typename T>
struct OpSum {
  __device__ static T apply(T a, T b) { return a + b; }
};
template <typename T>
struct OpMax {
  __device__ static T apply(T a, T b) { return a > b ? a : b; }
};

// Lane moves within a wave through DPP (no LDS traffic).  A 64-bit value moves
// as two 32-bit halves under the same control; lanes whose source lies outside
// the row, or whose row is not in kRowMask, receive 0.  Controls used here:
// 0xB1 / 0x4E quad_perm [1,0,3,2] / [2,3,0,1], 0x111.. row_shr:n,
// 0x121.. row_ror:n, 0x142 / 0x143 row_bcast:15 / row_bcast:31.  Every lane
// of the wave must be active.
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ uint32_t dpp_b32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, kRowMask, 0xF, true);
}
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t x = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp_b32<kCtrl, kRowMask>((uint32_t)x);
  const uint64_t hi = dpp_b32<kCtrl, kRowMask>((uint32_t)(x >> 32));
  return __builtin_bit_cast(double, (hi << 32) | lo);
}
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ int32_t dpp_i32(int32_t v) {
  return (int32_t)dpp_b32<kCtrl, kRowMask>((uint32_t)v);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t x = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return __builtin_bit_cast(double, (hi << 32) | lo);
}

// Reduces v over the wave; every lane gets the result.  Quads first (lanes
// ^1, then ^2), then rows of 16 (rotations by 4 and 8), then the four row
// values in the fixed order (r0 op r1) op (r2 op r3), read from lanes 0, 16,
// 32 and 48.
template <class Op>
__device__ __forceinline__ double wave_reduce(double v) {
  v = Op::apply(v, dpp_f64<0xB1>(v));
  v = Op::apply(v, dpp_f64<0x4E>(v));
  v = Op::apply(v, dpp_f64<0x124>(v));
  v = Op::apply(v, dpp_f64<0x128>(v));
  return Op::apply(Op::apply(readlane_f64(v, 0), readlane_f64(v, 16)),
                   Op::apply(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Inclusive scan over the wave: shifted adds within each row of 16 lanes,
// then row 0's total into row 1 and row 2's into row 3, then lanes 0..31's
// total into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  static_assert(std::is_same<T, double>::value || std::is_same<T, int32_t>::value,
                "double or int32 scans");
  if constexpr (std::is_same<T, double>::value) {
    v += dpp_f64<0x111>(v);
    v += dpp_f64<0x112>(v);
    v += dpp_f64<0x114>(v);
    v += dpp_f64<0x118>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
  } else {
    v += dpp_i32<0x111>(v);
    v += dpp_i32<0x112>(v);
    v += dpp_i32<0x114>(v);
    v += dpp_i32<0x118>(v);
    v += dpp_i32<0x142, 0xA>(v);
    v += dpp_i32<0x143, 0xC>(v);
  }
  return v;
}

// Reduces v over a 256-thread block; every thread gets the result.
template <class Op>
__device__ double block_reduce(double v, double *lds /* >= 4 */) {
  v = wave_reduce<Op>(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  return Op::apply(Op::apply(lds[0], lds[1]), Op::apply(lds[2], lds[3]));
}

}  // namespace smc
