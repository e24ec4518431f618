// Device-wide exclusive prefix sum of uint32 with a device-resident length.
//
// Used for the child numbering of the breadth-first tree (Section 2.1 of the
// paper numbers new cells by prefix sums), for active-particle compaction and
// for the radix-sort offsets.  Three launches over a fixed grid so the length
// may live on the device (no host read-back, capturable in a graph), or one
// workgroup when the host's bound on the length is small:
//   1. each block sums its contiguous chunk,
//   2. one block scans the chunk sums and writes the total,
//   3. each block scans its chunk again, offset by its chunk prefix.
// Memory is read and written in 16-byte vectors; the arrays must start on
// 16-byte boundaries.
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr int kScanBlocks = 1024;
constexpr int kScanThreads = 256;
// A block takes its chunk in rounds of kRound elements: thread t holds the
// four uint4 at offsets 4 t + 1024 q (q = 0..3) of the round, so every load
// instruction of a wave covers 1 KB of contiguous memory and four of them are
// in flight at once.  Chunks are whole rounds, so every vector access is
// aligned (the arrays start on 256-byte boundaries).
constexpr int kSub = 4 * kScanThreads;  // elements of one sub-round (one uint4 per thread)
constexpr int kRound = 4 * kSub;

int scan_blocks() { return kScanBlocks; }

__device__ __forceinline__ int64_t scan_len(int64_t n_host, const unsigned *n_dev,
                                            const unsigned *lo_dev) {
  if (!n_dev) return n_host;
  int64_t hi = *n_dev;
  int64_t lo = lo_dev ? (int64_t)*lo_dev : 0;
  return hi > lo ? hi - lo : 0;
}

// the chunk [s, e) of this block: ceil(n / blocks) rounded up to whole rounds
__device__ __forceinline__ void scan_chunk(int64_t n, int64_t *s, int64_t *e) {
  int64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  chunk = (chunk + kRound - 1) / kRound * kRound;
  *s = (int64_t)blockIdx.x * chunk;
  *e = *s + chunk < n ? *s + chunk : n;
  if (*s > n) *s = n;
}

// four elements from i (a multiple of 4); those at or past e read as 0
__device__ __forceinline__ uint4 load4(const uint32_t *in, int64_t i, int64_t e) {
  if (i + 4 <= e) return *reinterpret_cast<const uint4 *>(in + i);
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (i < e) v.x = in[i];
  if (i + 1 < e) v.y = in[i + 1];
  if (i + 2 < e) v.z = in[i + 2];
  return v;
}

__device__ __forceinline__ void store4(uint32_t *out, int64_t i, int64_t e, uint4 v) {
  if (i + 4 <= e) {
    *reinterpret_cast<uint4 *>(out + i) = v;
    return;
  }
  if (i < e) out[i] = v.x;
  if (i + 1 < e) out[i + 1] = v.y;
  if (i + 2 < e) out[i + 2] = v.z;
}

__global__ void __launch_bounds__(kScanThreads)
scan_reduce_k(const uint32_t *in, int64_t n_host, const unsigned *n_dev, const unsigned *lo_dev,
              int64_t n_max, uint32_t *part) {
  __shared__ unsigned sh[kScanThreads / 64 + 1];
  int64_t n = scan_len(n_host, n_dev, lo_dev);
  if (n > n_max) n = n_max;
  int64_t s, e;
  scan_chunk(n, &s, &e);
  unsigned acc = 0;
  for (int64_t base = s; base < e; base += kRound) {
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = load4(in, base + q * kSub + 4 * threadIdx.x, e);
#pragma unroll
    for (int q = 0; q < 4; ++q) acc += v[q].x + v[q].y + v[q].z + v[q].w;
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += sh[w];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kScanBlocks)
scan_partials_k(uint32_t *part, unsigned *total_dev) {
  __shared__ unsigned sh[kScanBlocks / 64 + 1];
  unsigned v = part[threadIdx.x];
  unsigned tot;
  unsigned ex = block_excl_sum<kScanBlocks>(v, sh, &tot);
  part[threadIdx.x] = ex;
  if (threadIdx.x == 0 && total_dev) *total_dev = tot;
}

// in and out may be the same array (each thread rewrites what it read)
__global__ void __launch_bounds__(kScanThreads)
scan_apply_k(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
             const unsigned *lo_dev, int64_t n_max, const uint32_t *part) {
  constexpr int NW = kScanThreads / 64;
  __shared__ unsigned sh[4][NW];
  int64_t n = scan_len(n_host, n_dev, lo_dev);
  if (n > n_max) n = n_max;
  int64_t s, e;
  scan_chunk(n, &s, &e);
  const int w = threadIdx.x >> 6, lane = lane_id();
  unsigned run = part[blockIdx.x];
  for (int64_t base = s; base < e; base += kRound) {
    uint4 v[4];
    unsigned inc[4], own[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = load4(in, base + q * kSub + 4 * threadIdx.x, e);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      own[q] = v[q].x + v[q].y + v[q].z + v[q].w;
      inc[q] = wave_incl_sum(own[q]);
      if (lane == 63) sh[q][w] = inc[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned before = 0, total = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const unsigned t = sh[q][k];
        before += k < w ? t : 0u;
        total += t;
      }
      const unsigned x = run + before + inc[q] - own[q];
      uint4 o;
      o.x = x;
      o.y = x + v[q].x;
      o.z = o.y + v[q].y;
      o.w = o.z + v[q].z;
      store4(out, base + q * kSub + 4 * threadIdx.x, e, o);
      run += total;
    }
    __syncthreads();
  }
}

// At most kSmallScan elements (a bound the host knows): one workgroup scans
// them in rounds of four per thread, carrying the running total, in one
// launch instead of three (small systems, upper tree levels, short sort
// histograms: the three launches' latency is most of their cost).
constexpr int kSmallThreads = 1024;
constexpr int64_t kSmallScan = 2 * 4 * kSmallThreads;

__global__ void __launch_bounds__(kSmallThreads)
scan_small_k(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
             const unsigned *lo_dev, int64_t n_max, unsigned *total_dev) {
  __shared__ unsigned sh[kSmallThreads / 64 + 1];
  int64_t n = scan_len(n_host, n_dev, lo_dev);
  if (n > n_max) n = n_max;
  unsigned run = 0;
  for (int64_t base = 0; base < n; base += 4 * kSmallThreads) {  // block-uniform
    const int64_t i = base + 4 * (int64_t)threadIdx.x;
    const uint4 v = load4(in, i, n);
    unsigned tot;
    const unsigned ex = block_excl_sum<kSmallThreads>(v.x + v.y + v.z + v.w, sh, &tot);
    uint4 o;
    o.x = run + ex;
    o.y = o.x + v.x;
    o.z = o.y + v.y;
    o.w = o.z + v.z;
    store4(out, i, n, o);
    run += tot;
  }
  if (threadIdx.x == 0 && total_dev) *total_dev = run;
}

void scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
                    const unsigned *lo_dev, int64_t n_max, unsigned *total_dev, uint32_t *part,
                    hipStream_t s) {
  if (n_max <= kSmallScan) {
    hipLaunchKernelGGL(scan_small_k, dim3(1), dim3(kSmallThreads), 0, s, in, out, n_host, n_dev,
                       lo_dev, n_max, total_dev);
    return;
  }
  hipLaunchKernelGGL(scan_reduce_k, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, n_host,
                     n_dev, lo_dev, n_max, part);
  hipLaunchKernelGGL(scan_partials_k, dim3(1), dim3(kScanBlocks), 0, s, part, total_dev);
  hipLaunchKernelGGL(scan_apply_k, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, out, n_host,
                     n_dev, lo_dev, n_max, part);
}

}  // namespace gothic
