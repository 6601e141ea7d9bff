// Deterministic block reductions and scans (fixed combination order; no
// floating-point atomics), for blocks of kBlock = 256 threads (4 waves).
#pragma once

#include <hip/hip_runtime.h>

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

template <class Op, typename T>
__device__ __forceinline__ T wave_reduce(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = Op::apply(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduces v over a 256-thread block; every thread gets the result.
template <class Op, typename T>
__device__ T block_reduce(T v, T *lds /* >= 4 */) {
  v = wave_reduce<Op>(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  T r = Op::apply(Op::apply(lds[0], lds[1]), Op::apply(lds[2], lds[3]));
  return r;
}

// Inclusive scan over a 256-thread block (Hillis-Steele in LDS); `total`
// receives the block sum.
template <typename T>
__device__ T block_inclusive_scan(T v, T *lds /* >= 256 */, T &total) {
  __syncthreads();
  lds[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int off = 1; off < kBlock; off <<= 1) {
    T add = (threadIdx.x >= (unsigned)off) ? lds[threadIdx.x - off] : T(0);
    __syncthreads();
    lds[threadIdx.x] += add;
    __syncthreads();
  }
  T r = lds[threadIdx.x];
  total = lds[kBlock - 1];
  __syncthreads();
  return r;
}

}  // namespace smc
