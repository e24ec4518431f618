// Device-wide exclusive prefix sum of uint32 with a device-resident length.
//
// Used for the child numbering of the breadth-first tree (Section 2.1 of the
// paper numbers new cells by prefix sums), for active-particle compaction and
// for the radix-sort offsets.  Three launches over a fixed grid so the length
// may live on the device (no host read-back, capturable in a graph):
//   1. each block sums its contiguous chunk,
//   2. one block scans the chunk sums and writes the total,
//   3. each block scans its chunk again, offset by its chunk prefix.
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr int kScanBlocks = 512;
constexpr int kScanThreads = 256;

int scan_blocks() { return kScanBlocks; }

__device__ __forceinline__ int64_t scan_len(int64_t n_host, const unsigned *n_dev,
                                            const unsigned *lo_dev) {
  if (!n_dev) return n_host;
  int64_t hi = *n_dev;
  int64_t lo = lo_dev ? (int64_t)*lo_dev : 0;
  return hi > lo ? hi - lo : 0;
}

__global__ void __launch_bounds__(kScanThreads)
scan_reduce_k(const uint32_t *in, int64_t n_host, const unsigned *n_dev, const unsigned *lo_dev,
              int64_t n_max, uint32_t *part) {
  __shared__ unsigned sh[kScanThreads / 64 + 1];
  int64_t n = scan_len(n_host, n_dev, lo_dev);
  if (n > n_max) n = n_max;
  const int64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  const int64_t s = (int64_t)blockIdx.x * chunk;
  const int64_t e = s + chunk < n ? s + chunk : n;
  unsigned acc = 0;
  for (int64_t i = s + threadIdx.x; i < e; i += kScanThreads) acc += in[i];
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

__global__ void __launch_bounds__(kScanThreads)
scan_apply_k(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
             const unsigned *lo_dev, int64_t n_max, const uint32_t *part) {
  __shared__ unsigned sh[kScanThreads / 64 + 1];
  int64_t n = scan_len(n_host, n_dev, lo_dev);
  if (n > n_max) n = n_max;
  const int64_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
  const int64_t s = (int64_t)blockIdx.x * chunk;
  const int64_t e = s + chunk < n ? s + chunk : n;
  unsigned run = part[blockIdx.x];
  for (int64_t base = s; base < e; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    unsigned v = i < e ? in[i] : 0u;
    unsigned tot;
    unsigned ex = block_excl_sum<kScanThreads>(v, sh, &tot);
    if (i < e) out[i] = run + ex;
    run += tot;
  }
}

void scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
                    const unsigned *lo_dev, int64_t n_max, unsigned *total_dev, uint32_t *part,
                    hipStream_t s) {
  hipLaunchKernelGGL(scan_reduce_k, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, n_host,
                     n_dev, lo_dev, n_max, part);
  hipLaunchKernelGGL(scan_partials_k, dim3(1), dim3(kScanBlocks), 0, s, part, total_dev);
  hipLaunchKernelGGL(scan_apply_k, dim3(kScanBlocks), dim3(kScanThreads), 0, s, in, out, n_host,
                     n_dev, lo_dev, n_max, part);
}

}  // namespace gothic
