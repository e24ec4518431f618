// Stable least-significant-digit radix sort of (63-bit key, 32-bit index)
// pairs: the key sort of Section 2.1 (the paper uses a library radix sort;
// this one is written for wave64).  Eight passes of 8-bit digits.  Per pass:
//   hist:    per-tile digit counts, stored digit-major,
//   scan:    exclusive scan of the digit-major table = global start of every
//            (digit, tile) bucket,
//   scatter: each tile ranks its elements stably (tile order, then wave
//            order, then lane order) with ballot-based digit matching,
//            places them in LDS in digit order and writes each digit's run
//            to its bucket with neighbouring threads on neighbouring
//            addresses.
// Equal keys keep the order of their indices, so the result is the
// lexicographic (key, original index) order.  With several systems the key
// passes are followed by passes on the digits of the system id (derived from
// the index), which makes the order (system, key, index): each system's
// particles stay in their own index range, sorted as if alone.
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
// up to kSmallSortN elements the tiles hold 2 items per thread: four times
// the workgroups, each with a quarter of the rounds (small systems are bound
// by the latency of each pass, not by its bytes)
constexpr int kSmallSortItems = 2;
constexpr int64_t kSmallSortN = 65536;

static int sort_tile(int64_t n) {
  return kSortThreads * (n <= kSmallSortN ? kSmallSortItems : kSortItems);
}
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kPasses = 8;

// passes over the digits of the system id (0 for one system)
static int sys_passes(int nsys) {
  int bits = 0;
  while (nsys > 1 && (1 << bits) < nsys) ++bits;
  return (bits + kRadixBits - 1) / kRadixBits;
}

bool keys_to_B(int nsys) { return ((kPasses + sys_passes(nsys)) & 1) != 0; }

// radix digit of an element: of the key, or (sys_shift >= 0) of its system id
__device__ __forceinline__ unsigned digit_of(uint64_t key, uint32_t id, int shift, int sys_shift,
                                             const uint32_t *__restrict__ soff, unsigned nsys) {
  if (sys_shift < 0) return (unsigned)(key >> shift) & (kRadix - 1);
  return (sys_of(soff, nsys, id) >> sys_shift) & (kRadix - 1);
}

// table entries for any length up to n: the small tiles' count for lengths up
// to kSmallSortN, the large tiles' beyond
int64_t radix_hist_entries(int64_t n) {
  const int64_t small_n = n < kSmallSortN ? n : kSmallSortN;
  const int small_tile = kSortThreads * kSmallSortItems, tile = kSortThreads * kSortItems;
  int64_t tiles = (small_n + small_tile - 1) / small_tile;
  const int64_t large = (n + tile - 1) / tile;
  if (large > tiles) tiles = large;
  return (tiles < 1 ? 1 : tiles) * kRadix;
}

template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
radix_hist_k(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ids, int64_t n,
             int shift, int sys_shift, const uint32_t *__restrict__ soff, unsigned nsys,
             int64_t ntiles, uint32_t *__restrict__ hist) {
  __shared__ unsigned cnt[kRadix];
  for (int t = threadIdx.x; t < kRadix; t += kSortThreads) cnt[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortThreads * ITEMS;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t e = base + r * kSortThreads + threadIdx.x;
    if (e < n) {
      const unsigned d = sys_shift < 0 ? (unsigned)(keys[e] >> shift) & (kRadix - 1)
                                       : digit_of(0, ids[e], 0, sys_shift, soff, nsys);
      atomicAdd(&cnt[d], 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kRadix; t += kSortThreads)
    hist[(int64_t)t * ntiles + blockIdx.x] = cnt[t];
}

template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_k(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ iin,
                uint64_t *__restrict__ kout, uint32_t *__restrict__ iout, int64_t n, int shift,
                int sys_shift, const uint32_t *__restrict__ soff, unsigned nsys, int64_t ntiles,
                const uint32_t *__restrict__ hist, const uint32_t *__restrict__ ofs) {
  constexpr int NW = kSortThreads / 64;
  constexpr int TILE = kSortThreads * ITEMS;
  static_assert(kSortThreads == kRadix, "one digit per thread in the local scan");
  __shared__ unsigned gofs[kRadix];    // global start of (digit, this tile)
  __shared__ unsigned lstart[kRadix];  // start of the digit inside the tile
  __shared__ unsigned run[kRadix];
  __shared__ unsigned wcnt[NW][kRadix];
  __shared__ unsigned scan_sh[NW + 1];
  __shared__ uint64_t sk[TILE];   // the tile in digit order
  __shared__ uint32_t si[TILE];
  const int t0 = threadIdx.x;
  gofs[t0] = ofs[(int64_t)t0 * ntiles + blockIdx.x];
  run[t0] = 0;
  unsigned total;
  lstart[t0] = block_excl_sum<kSortThreads>(hist[(int64_t)t0 * ntiles + blockIdx.x], scan_sh,
                                            &total);
  const int w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * TILE;
  // rank stably inside the tile (item round, then wave, then lane) and
  // place each element at its digit's run in LDS
  for (int r = 0; r < ITEMS; ++r) {
    for (int t = threadIdx.x; t < NW * kRadix; t += kSortThreads) (&wcnt[0][0])[t] = 0;
    __syncthreads();
    const int64_t e = base + r * kSortThreads + threadIdx.x;
    const bool valid = e < n;
    uint64_t key = valid ? kin[e] : 0;
    uint32_t id = valid ? iin[e] : 0;
    const unsigned d = digit_of(key, id, shift, sys_shift, soff, nsys);
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const unsigned below = lanes_below(m);
    const unsigned cnt = (unsigned)__popcll(m);
    if (valid && below == cnt - 1) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      unsigned pos = lstart[d] + run[d] + below;
      for (int v = 0; v < w; ++v) pos += wcnt[v][d];
      if (pos < (unsigned)TILE) {
        sk[pos] = key;
        si[pos] = id;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kRadix; t += kSortThreads) {
      unsigned s = 0;
      for (int v = 0; v < NW; ++v) s += wcnt[v][t];
      run[t] += s;
    }
    __syncthreads();
  }
  // write the tile out in digit order: neighbouring threads write
  // neighbouring addresses inside each digit's bucket
  const int64_t m_tile = n - base < TILE ? n - base : TILE;
  for (int j = threadIdx.x; j < m_tile; j += kSortThreads) {
    const uint64_t key = sk[j];
    const uint32_t id = si[j];
    const unsigned d = digit_of(key, id, shift, sys_shift, soff, nsys);
    const unsigned pos = gofs[d] + ((unsigned)j - lstart[d]);
    if (pos < n) {
      kout[pos] = key;
      iout[pos] = id;
    }
  }
}

void launch_radix_sort(gothic_ctx *c, int64_t n, int nsys, hipStream_t s) {
  const int passes = kPasses + sys_passes(nsys);
  // the key kernel wrote to B when the pass count is odd: the result always
  // ends in keyA / idxA
  uint64_t *ka = c->b.keyA, *kb = c->b.keyB;
  uint32_t *ia = c->b.idxA, *ib = c->b.idxB;
  if (passes & 1) {
    ka = c->b.keyB; kb = c->b.keyA;
    ia = c->b.idxB; ib = c->b.idxA;
  }
  if (n <= 1) return;  // then nsys <= 1 (systems are never empty): an even count, in A
  const bool small = n <= kSmallSortN;
  const int tile = sort_tile(n);
  const int64_t ntiles = (n + tile - 1) / tile;
  uint32_t *hist = c->b.hist;
  uint32_t *ofs = c->b.hist + ntiles * kRadix;
  for (int p = 0; p < passes; ++p) {
    const int shift = p < kPasses ? p * kRadixBits : 0;
    const int sys_shift = p < kPasses ? -1 : (p - kPasses) * kRadixBits;
    hipLaunchKernelGGL(small ? radix_hist_k<kSmallSortItems> : radix_hist_k<kSortItems>,
                       dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, ka, ia, n, shift,
                       sys_shift, c->b.soff, (unsigned)nsys, ntiles, hist);
    scan_exclusive(hist, ofs, ntiles * kRadix, nullptr, nullptr, ntiles * kRadix,
                   &c->b.ctl->scan_total, c->b.part, s);
    hipLaunchKernelGGL(small ? radix_scatter_k<kSmallSortItems> : radix_scatter_k<kSortItems>,
                       dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, ka, ia, kb, ib, n, shift,
                       sys_shift, c->b.soff, (unsigned)nsys, ntiles, hist, ofs);
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *ti = ia; ia = ib; ib = ti;
  }
}

}  // namespace gothic
