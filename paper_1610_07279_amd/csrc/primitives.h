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

// DPP move (gfx9 encodings): lanes without a source lane read 0
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_or_zero(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// inclusive prefix sum over the 64 lanes (all lanes active): shifts by 1, 2,
// 4, 8 inside each row of 16 lanes, then row_bcast:15 adds row r's total to
// rows 1 and 3 and row_bcast:31 adds row 1's total to rows 2 and 3
__device__ __forceinline__ unsigned wave_incl_sum(unsigned v) {
  v += dpp_or_zero<0x111, 0xf>(v);
  v += dpp_or_zero<0x112, 0xf>(v);
  v += dpp_or_zero<0x114, 0xf>(v);
  v += dpp_or_zero<0x118, 0xf>(v);
  v += dpp_or_zero<0x142, 0xa>(v);
  v += dpp_or_zero<0x143, 0xc>(v);
  return v;
}

// inclusive prefix maximum over the 64 lanes (all lanes active), the steps
// of wave_incl_sum
__device__ __forceinline__ unsigned wave_incl_max(unsigned v) {
  v = max(v, dpp_or_zero<0x111, 0xf>(v));
  v = max(v, dpp_or_zero<0x112, 0xf>(v));
  v = max(v, dpp_or_zero<0x114, 0xf>(v));
  v = max(v, dpp_or_zero<0x118, 0xf>(v));
  v = max(v, dpp_or_zero<0x142, 0xa>(v));
  v = max(v, dpp_or_zero<0x143, 0xc>(v));
  return v;
}

// the value of lane 63
__device__ __forceinline__ unsigned wave_last(unsigned v) {
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
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
