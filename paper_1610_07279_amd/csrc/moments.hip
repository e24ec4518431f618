// Pseudo j-particles (Section 2.1): for every node the total mass M_J, the
// centre of mass r_J and the radius b_J of the smallest sphere about r_J that
// holds all member particles; with multipole = 2 also the second moments
// S_ab = sum m (r - r_J)_a (r - r_J)_b.  Recomputed on every call, in FP32.
//   leaves:    straight from the member particles (centre of mass taken
//              relative to the first member, so a one-particle leaf has
//              r_J = r exactly and b_J = 0);
//   internal:  bottom-up one level at a time from the children (masses and
//              centres add; second moments by the parallel-axis rule);
//   b_J:       particle-parallel: each particle walks up its ancestor chain
//              one level per step; lanes of a wave that share an ancestor
//              (always a contiguous run in key order) max-reduce their
//              distances and one lane per run issues an atomic max.
// The node record read by the walk is written here: (x, y, z, M) and
// (b_J, first|child_first, count|n_child, is_leaf).
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr unsigned kNone = 0xffffffffu;

__device__ __forceinline__ float u2f(unsigned u) { return __uint_as_float(u); }

__global__ void __launch_bounds__(256)
leaf_moments_k(Ctl *__restrict__ ctl, int64_t n, const uint32_t *__restrict__ first,
               const uint32_t *__restrict__ count, const uint8_t *__restrict__ n_child,
               const float4 *__restrict__ pos, uint32_t *__restrict__ leaf_of,
               float4 *__restrict__ nrec, float4 *__restrict__ quad, int want_quad) {
  if (ctl->flags & kFlagNodeOverflow) return;  // incomplete tree: nothing to do
  const int64_t nn = ctl->n_nodes;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (n_child[k] != 0) continue;
    const uint32_t f = first[k], c = count[k];
    if (c == 0 || (int64_t)f + c > n) {
      atomicOr(&ctl->flags, kFlagBadIndex);
      continue;
    }
    const float4 p0 = pos[f];
    float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
    for (uint32_t j = f; j < f + c; ++j) {
      const float4 p = pos[j];
      M += p.w;
      sx += p.w * (p.x - p0.x);
      sy += p.w * (p.y - p0.y);
      sz += p.w * (p.z - p0.z);
      leaf_of[j] = (uint32_t)k;
    }
    float cx = p0.x, cy = p0.y, cz = p0.z;
    if (M > 0.f) {
      cx = p0.x + sx / M;
      cy = p0.y + sy / M;
      cz = p0.z + sz / M;
    }
    float b2 = 0.f, xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
    for (uint32_t j = f; j < f + c; ++j) {
      const float4 p = pos[j];
      const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
      b2 = fmaxf(b2, dx * dx + dy * dy + dz * dz);
      if (want_quad) {
        xx += p.w * dx * dx; yy += p.w * dy * dy; zz += p.w * dz * dz;
        xy += p.w * dx * dy; xz += p.w * dx * dz; yz += p.w * dy * dz;
      }
    }
    const float b = (M > 0.f) ? sqrtf(b2) : 0.f;
    nrec[2 * k] = make_float4(cx, cy, cz, M);
    nrec[2 * k + 1] = make_float4(b, u2f(f), u2f(c), u2f(1u));
    quad[2 * k] = make_float4(xx, yy, zz, xy);
    quad[2 * k + 1] = make_float4(xz, yz, xx + yy + zz, 0.f);
  }
}

__global__ void __launch_bounds__(256)
internal_moments_k(int l, Ctl *__restrict__ ctl, const uint32_t *__restrict__ child_first,
                   const uint8_t *__restrict__ n_child, float4 *__restrict__ nrec,
                   float4 *__restrict__ quad, int want_quad) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const int64_t hi_all = ctl->n_nodes;
  const int64_t lo = ctl->lvl_start[l];
  int64_t hi = ctl->lvl_start[l + 1];
  if (hi > hi_all) hi = hi_all;
  for (int64_t k = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < hi;
       k += (int64_t)gridDim.x * blockDim.x) {
    const unsigned nc = n_child[k];
    if (nc == 0) continue;
    const uint32_t cf = child_first[k];
    if (cf <= k || (int64_t)cf + nc > hi_all) {
      atomicOr(&ctl->flags, kFlagBadIndex);
      continue;
    }
    const float4 r0 = nrec[2 * (size_t)cf];
    float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
    for (unsigned q = 0; q < nc; ++q) {
      const float4 r = nrec[2 * (cf + q)];
      M += r.w;
      sx += r.w * (r.x - r0.x);
      sy += r.w * (r.y - r0.y);
      sz += r.w * (r.z - r0.z);
    }
    float cx = r0.x, cy = r0.y, cz = r0.z;
    if (M > 0.f) {
      cx = r0.x + sx / M;
      cy = r0.y + sy / M;
      cz = r0.z + sz / M;
    }
    float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
    if (want_quad) {
      for (unsigned q = 0; q < nc; ++q) {
        const float4 r = nrec[2 * (cf + q)];
        const float4 s0 = quad[2 * (cf + q)], s1 = quad[2 * (cf + q) + 1];
        const float dx = r.x - cx, dy = r.y - cy, dz = r.z - cz;
        xx += s0.x + r.w * dx * dx; yy += s0.y + r.w * dy * dy; zz += s0.z + r.w * dz * dz;
        xy += s0.w + r.w * dx * dy; xz += s1.x + r.w * dx * dz; yz += s1.y + r.w * dy * dz;
      }
    }
    nrec[2 * k] = make_float4(cx, cy, cz, M);
    nrec[2 * k + 1] = make_float4(0.f, u2f(cf), u2f(nc), u2f(0u));
    quad[2 * k] = make_float4(xx, yy, zz, xy);
    quad[2 * k + 1] = make_float4(xz, yz, xx + yy + zz, 0.f);
  }
}

__global__ void __launch_bounds__(256)
radius_k(Ctl *__restrict__ ctl, int64_t n, const float4 *__restrict__ pos,
         const uint32_t *__restrict__ leaf_of, const uint32_t *__restrict__ parent,
         const uint8_t *__restrict__ level, float4 *__restrict__ nrec) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const unsigned nn = ctl->n_nodes;
  // Loop control is wave-uniform (readfirstlane) and the per-lane steps are
  // predicated rather than branched, so every lane takes part in each shuffle.
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool inr = i < n;
    const int64_t ic = inr ? i : n - 1;
    const float4 p = pos[ic];
    const unsigned lf = leaf_of[ic];
    const unsigned par = lf < nn ? parent[lf] : kNone;
    unsigned node = (inr && (par < nn)) ? par : kNone;
    int lv = (node != kNone) ? (int)level[node != kNone ? node : 0] : -1;
    int top = lv;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) top = max(top, __shfl_xor(top, d, 64));
    top = __builtin_amdgcn_readfirstlane(top);
    for (int l = top; l >= 0; --l) {
      const bool part = (node != kNone) && (lv == l);
      const unsigned key = part ? node : kNone;
      const unsigned ns = part ? node : 0u;
      const float4 r = nrec[2 * (size_t)ns];
      const float dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
      float dist = (part && r.w > 0.f) ? sqrtf(dx * dx + dy * dy + dz * dz) : 0.f;
      // segmented max over contiguous runs of equal key
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const float od = __shfl_down(dist, d, 64);
        const unsigned ok = __shfl_down(key, d, 64);
        dist = (lane + d < 64 && ok == key) ? fmaxf(dist, od) : dist;
      }
      const unsigned prev = __shfl_up(key, 1, 64);
      if (part && (lane == 0 || prev != key))
        atomicMax(reinterpret_cast<unsigned *>(&nrec[2 * (size_t)node + 1].x),
                  __float_as_uint(dist));
      const unsigned up0 = parent[ns];
      const unsigned up = up0 < nn ? up0 : kNone;  // the root's parent is kNone
      const int uplv = (up != kNone) ? (int)level[up != kNone ? up : 0] : -1;
      node = part ? up : node;
      lv = part ? uplv : lv;
    }
  }
}

void launch_moments(gothic_ctx *c, int64_t n, hipStream_t s) {
  Buffers &B = c->b;
  const int wq = c->prm.multipole == 2 ? 1 : 0;
  int64_t nb = (c->cap_nodes + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(leaf_moments_k, dim3(g), dim3(256), 0, s, B.ctl, n, B.first, B.count,
                     B.n_child, B.pos, B.leaf_of, B.nrec, B.quad, wq);
  for (int l = kNlev - 1; l >= 0; --l) {
    int64_t widest = 1;
    for (int q = 0; q < l && widest < c->cap_nodes; ++q) widest *= 8;
    if (widest > c->cap_nodes) widest = c->cap_nodes;
    int64_t lb = (widest + 255) / 256;
    int gl = (int)(lb > 4096 ? 4096 : (lb < 1 ? 1 : lb));
    hipLaunchKernelGGL(internal_moments_k, dim3(gl), dim3(256), 0, s, l, B.ctl, B.child_first,
                       B.n_child, B.nrec, B.quad, wq);
  }
  int64_t pb = (n + 255) / 256;
  int gp = (int)(pb > 8192 ? 8192 : (pb < 1 ? 1 : pb));
  hipLaunchKernelGGL(radius_k, dim3(gp), dim3(256), 0, s, B.ctl, n, B.pos, B.leaf_of, B.parent,
                     B.level, B.nrec);
}

}  // namespace gothic
