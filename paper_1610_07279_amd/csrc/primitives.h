// Wave64 / workgroup building blocks for gfx950 (device inline helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gothic {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of m strictly below this lane
__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ unsigned wave_incl_sum(unsigned v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned t = __shfl_up(v, d, 64);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
  return v;
}

// Exclusive prefix sum over a workgroup of NT threads (NT multiple of 64,
// NT <= 1024).  `sh` must hold NT/64 + 1 unsigned.  Returns the exclusive
// prefix; *total receives the workgroup sum.  Contains barriers.
template <int NT>
__device__ __forceinline__ unsigned block_excl_sum(unsigned v, unsigned *sh, unsigned *total) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, l = lane_id();
  unsigned inc = wave_incl_sum(v);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x < 64) {
    unsigned t = (l < NW) ? sh[l] : 0u;
    unsigned ti = wave_incl_sum(t);
    if (l < NW) sh[l] = ti - t;
    if (l == NW - 1) sh[NW] = ti;
  }
  __syncthreads();
  unsigned r = sh[w] + inc - v;
  *total = sh[NW];
  __syncthreads();
  return r;
}

}  // namespace gothic
