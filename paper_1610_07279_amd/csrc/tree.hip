// Permutation to key order and the breadth-first octree (Section 2.1).
//
// A cell at level l is a run of sorted keys sharing their top 3l bits, and
// splitting it into eight sub-cubes is cutting the run where the next 3-bit
// digit changes.  The tree is built one level at a time, breadth first, with
// every count on the device:
//   count: each level-l node holding more than n_leaf particles (and above
//          level 21) finds its child boundaries by searching for the seven
//          digit changes (nine-way steps over long runs, then bisection) and
//          counts its non-empty children;
//          other nodes become leaves;
//   scan:  exclusive prefix sum of the child counts = serial numbers of the
//          level-(l+1) nodes (the prefix sums of Section 2.1);
//   write: split nodes write their children (parent order, then digit
//          order), which is the breadth-first numbering.
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr int kBuildThreads = 256;
constexpr unsigned kNone = 0xffffffffu;

// Key order: positions and masses, active flags and (acceleration MAC) the
// magnitudes of the previous accelerations.  sign_active: the flag is the
// sign bit of the mass (set by the block-step predictor), which is cleared.
__global__ void __launch_bounds__(256)
permute_k(const float4 *__restrict__ xyzm, const uint8_t *__restrict__ active, int sign_active,
          const float4 *__restrict__ acc_old, int64_t n, const uint32_t *__restrict__ perm,
          float4 *__restrict__ pos, uint32_t *__restrict__ flag, float *__restrict__ amag,
          Ctl *ctl) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    uint32_t i = perm[k];
    if (i >= n) {
      atomicOr(&ctl->flags, kFlagBadIndex);
      i = 0;
    }
    float4 p = xyzm[i];
    if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w)))
      atomicOr(&ctl->flags, kFlagNonFinite);  // (a reused tree skips the key pass)
    unsigned f = 1u;
    if (sign_active) {
      f = signbit(p.w) ? 1u : 0u;
      p.w = fabsf(p.w);
    } else if (active) {
      f = active[i] != 0 ? 1u : 0u;
    }
    pos[k] = p;
    flag[k] = f;
    if (acc_old) {
      const float4 a = acc_old[i];
      amag[k] = sqrtf(a.x * a.x + a.y * a.y + a.z * a.z);
    }
  }
}

void launch_permute(gothic_ctx *c, const float4 *xyzm, const uint8_t *active, bool sign_active,
                    const float4 *acc_old, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(permute_k, dim3(g), dim3(256), 0, s, xyzm, active, sign_active ? 1 : 0,
                     acc_old, n, c->b.idxA,
                     c->b.pos, c->b.flag, c->b.amag, c->b.ctl);
}

__global__ void __launch_bounds__(256)
build_init_k(Ctl *ctl, int nsys, const uint32_t *__restrict__ soff, uint32_t *first,
             uint32_t *count, uint32_t *parent, uint8_t *level) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nsys; r += gridDim.x * blockDim.x) {
    first[r] = soff[r];
    count[r] = soff[r + 1] - soff[r];
    parent[r] = kNone;
    level[r] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->lvl_start[0] = 0;
    for (int l = 1; l < kMaxLevels + 2; ++l) ctl->lvl_start[l] = (unsigned)nsys;
    ctl->n_nodes = (unsigned)nsys;
    ctl->nsys = (unsigned)nsys;
  }
}

__device__ __forceinline__ unsigned digit_at(uint64_t key, int shift) {
  return (unsigned)(key >> shift) & 7u;
}

// The children of node k of level l (particles [f, f + c) in key order):
// records the 7 inner boundaries in bnd8[1..7] and returns how many of the 8
// digit runs are non-empty (0 for a leaf).  KS is a global or an LDS key
// array.
template <class KS>
__device__ __forceinline__ unsigned count_children(int l, int n_leaf, int64_t n, KS ks,
                                                   uint32_t f, uint32_t c, Ctl *ctl,
                                                   uint32_t *bnd8) {
  const int shift = 3 * (kNlev - 1 - l);
  unsigned nc = 0;
  if ((int64_t)f + c > n) {
    atomicOr(&ctl->flags, kFlagBadIndex);
  } else if (c > (uint32_t)n_leaf && l < kNlev) {
    // the first index with digit >= d, for d = 1..7: each lies in [a[d], b[d]]
    // (indices below a[d] have a smaller digit, those from b[d] on one at
    // least d).  Runs of more than 2^16 (the few nodes of the top levels,
    // where the search latency is not hidden by other nodes) are narrowed
    // by eight probes per digit and round (every load of a round in
    // flight at once); then bisection, all digits in lock step.
    uint32_t a[8], b[8];
#pragma unroll
    for (int d = 1; d < 8; ++d) { a[d] = f; b[d] = f + c; }
    for (uint32_t len = c; len > 64 && c > 65536u; len = (len + 8) / 9) {
#pragma unroll
      for (int d = 1; d < 8; ++d) {
        const uint32_t span = b[d] - a[d];
        if (span <= 8) continue;
        uint32_t q[8];
        bool g[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          q[j] = a[d] + (uint32_t)(((uint64_t)span * (uint64_t)(j + 1)) / 9u);
          g[j] = digit_at(ks[q[j]], shift) >= (unsigned)d;
        }
        uint32_t na = a[d], nb = b[d];
#pragma unroll
        for (int j = 7; j >= 0; --j)
          if (g[j]) nb = q[j];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (!g[j]) na = q[j] + 1;
        a[d] = na;
        b[d] = nb;
      }
    }
    for (uint32_t len = c > 65536u ? 64u : c; len > 0; len >>= 1) {
#pragma unroll
      for (int d = 1; d < 8; ++d) {
        if (a[d] < b[d]) {
          const uint32_t mid = a[d] + ((b[d] - a[d]) >> 1);
          if (digit_at(ks[mid], shift) >= (unsigned)d) b[d] = mid; else a[d] = mid + 1;
        }
      }
    }
    // one more pass guarantees convergence for any length
#pragma unroll
    for (int d = 1; d < 8; ++d) {
      while (a[d] < b[d]) {
        const uint32_t mid = a[d] + ((b[d] - a[d]) >> 1);
        if (digit_at(ks[mid], shift) >= (unsigned)d) b[d] = mid; else a[d] = mid + 1;
      }
    }
    uint32_t prev = f;
#pragma unroll
    for (int d = 1; d < 8; ++d) {
      bnd8[d] = a[d];
      nc += (a[d] > prev) ? 1u : 0u;
      prev = a[d];
    }
    nc += (f + c > prev) ? 1u : 0u;
  }
  return nc;
}

// The children of node k of level l, numbered from base (the next level's
// start plus the node's exclusive prefix of child counts): written from the
// boundaries the count pass stored.
__device__ __forceinline__ void write_children(int l, int n_leaf, int64_t n, int64_t cap_nodes,
                                               int64_t k, uint32_t f, uint32_t c, int64_t base,
                                               const uint32_t *bnd8, uint32_t *child_first,
                                               uint8_t *n_child, uint32_t *cfirst,
                                               uint32_t *ccount, uint32_t *cparent,
                                               uint8_t *clevel) {
  // only nodes the count pass split have boundaries stored
  if (c <= (uint32_t)n_leaf || (int64_t)f + c > n) return;
  // recover the non-empty children from the stored boundaries
  int made = 0;
  {
    uint32_t s = f;
#pragma unroll
    for (int d = 1; d <= 8; ++d) {
      const uint32_t e = (d < 8) ? bnd8[d] : f + c;
      if (e > s) { ++made; s = e; }
    }
  }
  if (made == 0) return;
  if (base + made > cap_nodes) {
    // out of node capacity: keep the tree consistent by leaving this node a
    // leaf (flagged; the host grows the arrays and repeats the evaluation)
    child_first[k] = 0;
    n_child[k] = 0;
    return;
  }
  uint32_t s = f;
  int j = 0;
#pragma unroll
  for (int d = 1; d <= 8; ++d) {
    const uint32_t e = (d < 8) ? bnd8[d] : f + c;
    if (e > s) {
      cfirst[base + j] = s;
      ccount[base + j] = e - s;
      cparent[base + j] = (uint32_t)k;
      clevel[base + j] = (uint8_t)(l + 1);
      ++j;
      s = e;
    }
  }
  child_first[k] = (uint32_t)base;
  n_child[k] = (uint8_t)made;
}

// Count children of every level-l node; record the 7 inner boundaries.
__global__ void __launch_bounds__(kBuildThreads)
build_count_k(int l, int n_leaf, int64_t n, int64_t cap_nodes, int64_t cap_level, Ctl *ctl,
              const uint64_t *__restrict__ ks, const uint32_t *__restrict__ first,
              const uint32_t *__restrict__ count, uint32_t *__restrict__ child_first,
              uint8_t *__restrict__ n_child, uint32_t *__restrict__ nch,
              uint32_t *__restrict__ bnd) {
  if (ctl->flags & kFlagNodeOverflow) return;  // tree abandoned; the host repeats
  const int64_t lo = ctl->lvl_start[l];
  int64_t hi = ctl->lvl_start[l + 1];
  if (hi > cap_nodes) hi = cap_nodes;
  if (hi - lo > cap_level) hi = lo + cap_level;
  for (int64_t k = lo + (int64_t)blockIdx.x * kBuildThreads + threadIdx.x; k < hi;
       k += (int64_t)gridDim.x * kBuildThreads) {
    const unsigned nc = count_children(l, n_leaf, n, ks, first[k], count[k], ctl,
                                       bnd + (k - lo) * 8);
    nch[k - lo] = nc;
    if (nc == 0) {
      child_first[k] = 0;
      n_child[k] = 0;
    }
  }
}

__global__ void __launch_bounds__(kBuildThreads)
build_write_k(int l, int n_leaf, int64_t n, int64_t cap_nodes, int64_t cap_level, Ctl *ctl,
              const uint32_t *__restrict__ first,
              const uint32_t *__restrict__ count, const uint32_t *__restrict__ ofs,
              const uint32_t *__restrict__ bnd, uint32_t *__restrict__ child_first,
              uint8_t *__restrict__ n_child, uint32_t *__restrict__ cfirst,
              uint32_t *__restrict__ ccount, uint32_t *__restrict__ cparent,
              uint8_t *__restrict__ clevel) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const int64_t lo = ctl->lvl_start[l];
  int64_t hi = ctl->lvl_start[l + 1];
  const int64_t nxt = ctl->lvl_start[l + 1];
  const int64_t total = ctl->scan_total;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t end = nxt + total;
    ctl->lvl_start[l + 2] = (unsigned)(end > 0xffffffffll ? 0xffffffffll : end);
    if (end > cap_nodes) atomicOr(&ctl->flags, kFlagNodeOverflow);
  }
  if (hi > cap_nodes) hi = cap_nodes;
  if (hi - lo > cap_level) hi = lo + cap_level;
  for (int64_t k = lo + (int64_t)blockIdx.x * kBuildThreads + threadIdx.x; k < hi;
       k += (int64_t)gridDim.x * kBuildThreads)
    write_children(l, n_leaf, n, cap_nodes, k, first[k], count[k], nxt + ofs[k - lo],
                   bnd + (k - lo) * 8, child_first, n_child, cfirst, ccount, cparent, clevel);
}

// Small systems (n <= kSmallBuild particles, a bound the host knows): the
// whole level loop (count, prefix sum of the child counts, write) in one
// workgroup, with the sorted keys in LDS and a barrier between the phases,
// instead of three to five launches per level.  Same arithmetic and outputs
// as build_count_k / scan / build_write_k.
constexpr int kSmallBuild = 8192;
constexpr int kSmallBuildThreads = 1024;

__global__ void __launch_bounds__(kSmallBuildThreads)
build_small_k(int n_leaf, int64_t n, int64_t cap_nodes, int64_t cap_level, Ctl *ctl,
              const uint64_t *__restrict__ ks_g, uint32_t *first, uint32_t *count,
              uint32_t *child_first, uint8_t *n_child, uint32_t *parent, uint8_t *level,
              uint32_t *nch, uint32_t *bnd) {
  __shared__ uint64_t ks[kSmallBuild];
  __shared__ unsigned sh[kSmallBuildThreads / 64 + 1];
  const int t = threadIdx.x;
  for (int64_t i = t; i < n; i += kSmallBuildThreads) ks[i] = ks_g[i];
  __syncthreads();
  for (int l = 0; l <= kNlev; ++l) {
    if (ctl->flags & kFlagNodeOverflow) break;  // block-uniform (read after a barrier)
    const int64_t lo = ctl->lvl_start[l];
    int64_t hi = ctl->lvl_start[l + 1];
    if (lo >= hi) {
      // an empty level: so are all deeper ones, which end where it does
      // (what the remaining count / scan / write passes would record)
      if (t == 0)
        for (int j = l + 2; j <= kNlev + 1; ++j) ctl->lvl_start[j] = (unsigned)hi;
      break;
    }
    if (hi > cap_nodes) hi = cap_nodes;
    if (hi - lo > cap_level) hi = lo + cap_level;
    for (int64_t k = lo + t; k < hi; k += kSmallBuildThreads) {
      const unsigned nc = count_children(l, n_leaf, n, ks, first[k], count[k], ctl,
                                         bnd + (k - lo) * 8);
      nch[k - lo] = nc;
      if (nc == 0) {
        child_first[k] = 0;
        n_child[k] = 0;
      }
    }
    __syncthreads();
    if (l == kNlev) break;
    // exclusive prefix sum of the child counts over the level (in place),
    // in rounds of one count per thread
    const int64_t m = hi > lo ? hi - lo : 0;
    unsigned run = 0;
    for (int64_t b0 = 0; b0 < m; b0 += kSmallBuildThreads) {  // block-uniform
      const int64_t i = b0 + t;
      const unsigned v = i < m ? nch[i] : 0u;
      unsigned tot;
      const unsigned ex = block_excl_sum<kSmallBuildThreads>(v, sh, &tot);
      if (i < m) nch[i] = run + ex;
      run += tot;
    }
    const int64_t nxt = ctl->lvl_start[l + 1];
    __syncthreads();
    if (t == 0) {
      const int64_t end = nxt + run;
      ctl->lvl_start[l + 2] = (unsigned)(end > 0xffffffffll ? 0xffffffffll : end);
      if (end > cap_nodes) atomicOr(&ctl->flags, kFlagNodeOverflow);
    }
    // (with the level past the node capacity the write still runs, as
    // build_write_k does: nodes whose children do not fit stay leaves)
    for (int64_t k = lo + t; k < hi; k += kSmallBuildThreads)
      write_children(l, n_leaf, n, cap_nodes, k, first[k], count[k], nxt + nch[k - lo],
                     bnd + (k - lo) * 8, child_first, n_child, first, count, parent, level);
    __syncthreads();
  }
}

// n_nodes = end of the deepest level
__global__ void build_final_k(Ctl *ctl, int64_t cap_nodes) {
  if (threadIdx.x == 0) {
    int64_t e = ctl->lvl_start[kMaxLevels];
    ctl->n_nodes = (unsigned)(e > cap_nodes ? cap_nodes : e);
    ctl->tree_ok = (ctl->flags & kFlagNodeOverflow) ? 0u : 1u;
  }
}

void launch_build(gothic_ctx *c, int64_t n, int nsys, hipStream_t s) {
  Buffers &B = c->b;
  const int ib = (nsys + 255) / 256;
  hipLaunchKernelGGL(build_init_k, dim3(ib > 1024 ? 1024 : ib), dim3(256), 0, s, B.ctl, nsys,
                     B.soff, B.first, B.count, B.parent, B.level);
  const int64_t cap = c->cap_nodes;
  if (n <= kSmallBuild) {
    hipLaunchKernelGGL(build_small_k, dim3(1), dim3(kSmallBuildThreads), 0, s, c->prm.n_leaf, n,
                       cap, c->cap_n, B.ctl, B.keyA, B.first, B.count, B.child_first, B.n_child,
                       B.parent, B.level, B.nch, B.bnd);
    hipLaunchKernelGGL(build_final_k, dim3(1), dim3(64), 0, s, B.ctl, cap);
    return;
  }
  // grid large enough for the widest level (at most min(cap, nsys 8^l) nodes)
  for (int l = 0; l <= kNlev; ++l) {
    int64_t widest = nsys;
    for (int q = 0; q < l && widest < cap; ++q) widest *= 8;
    if (widest > cap) widest = cap;
    int64_t nb = (widest + kBuildThreads - 1) / kBuildThreads;
    const int g = (int)(nb > 4096 ? 4096 : (nb < 1 ? 1 : nb));
    hipLaunchKernelGGL(build_count_k, dim3(g), dim3(kBuildThreads), 0, s, l, c->prm.n_leaf, n, cap,
                       c->cap_n, B.ctl, B.keyA, B.first, B.count, B.child_first, B.n_child,
                       B.nch, B.bnd);
    if (l == kNlev) break;
    // the nodes of level l: at most nsys 8^l (and at most cap_n)
    int64_t lvl_max = nsys;
    for (int q = 0; q < l && lvl_max < c->cap_n; ++q) lvl_max *= 8;
    if (lvl_max > c->cap_n) lvl_max = c->cap_n;
    scan_exclusive(B.nch, B.nch, 0, &B.ctl->lvl_start[l + 1], &B.ctl->lvl_start[l], lvl_max,
                   &B.ctl->scan_total, B.part, s);
    hipLaunchKernelGGL(build_write_k, dim3(g), dim3(kBuildThreads), 0, s, l, c->prm.n_leaf, n, cap,
                       c->cap_n, B.ctl,
                       B.first, B.count, B.nch, B.bnd, B.child_first, B.n_child, B.first,
                       B.count, B.parent, B.level);
  }
  hipLaunchKernelGGL(build_final_k, dim3(1), dim3(64), 0, s, B.ctl, cap);
}

}  // namespace gothic
