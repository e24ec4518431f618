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

// Each wave takes a contiguous chunk of key-ordered particles, in tiles of
// 64.  A node's particles are contiguous, so at every level the ancestors of
// a tile form runs; runs that end inside the tile are complete and issue one
// atomic max each, the last run of a tile is carried to the next tile as a
// per-level running (node, max) in LDS.  Upper-level nodes thus receive one
// atomic per wave chunk instead of one per 64 particles.
constexpr int kRadiusWaves = 4;  // waves per workgroup

__device__ __forceinline__ void flush_b(float4 *nrec, unsigned node, float v) {
  // every lane passes the same (node, v): the atomic is combined per wave
  atomicMax(reinterpret_cast<unsigned *>(&nrec[2 * (size_t)node + 1].x), __float_as_uint(v));
}

__global__ void __launch_bounds__(256)
radius_k(Ctl *__restrict__ ctl, int64_t n, const float4 *__restrict__ pos,
         const uint32_t *__restrict__ leaf_of, const uint32_t *__restrict__ parent,
         const uint8_t *__restrict__ level, float4 *__restrict__ nrec) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const unsigned nn = ctl->n_nodes;
  __shared__ unsigned s_node[kRadiusWaves][kMaxLevels];
  __shared__ float s_max[kRadiusWaves][kMaxLevels];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  if (lane < kMaxLevels) {
    s_node[w][lane] = kNone;
    s_max[w][lane] = 0.f;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int64_t nw = (int64_t)gridDim.x * kRadiusWaves;
  const int64_t wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kRadiusWaves + w));
  const int64_t chunk = ((n + nw - 1) / nw + 63) / 64 * 64;
  const int64_t c0 = wid * chunk;
  const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
  for (int64_t base = c0; base < c1; base += 64) {
    const int64_t i = base + lane;
    const bool inr = i < c1;
    const int64_t ic = inr ? i : c1 - 1;
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
      // a parent is one level up (breadth-first levels): only the parent
      // index is needed for the next level, loaded together with the record
      const unsigned up0 = parent[ns];
      const float dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
      float dist = (part && r.w > 0.f) ? sqrtf(dx * dx + dy * dy + dz * dz) : 0.f;
      // segmented max over contiguous runs of equal key: the first lane of
      // each run ends up with the run's maximum
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const float od = __shfl_down(dist, d, 64);
        const unsigned ok = __shfl_down(key, d, 64);
        dist = (lane + d < 64 && ok == key) ? fmaxf(dist, od) : dist;
      }
      const unsigned prev = __shfl_up(key, 1, 64);
      const bool lead = part && (lane == 0 || prev != key);
      const unsigned long long lm = __ballot(lead);
      if (lm) {
        const int fl = __builtin_amdgcn_readfirstlane(__ffsll((long long)lm) - 1);
        const int ll = __builtin_amdgcn_readfirstlane(63 - __clzll((long long)lm));
        const unsigned fnode = __builtin_amdgcn_readfirstlane(__shfl(key, fl, 64));
        const unsigned lnode = __builtin_amdgcn_readfirstlane(__shfl(key, ll, 64));
        const float fmx = __shfl(dist, fl, 64);
        const float lmx = __shfl(dist, ll, 64);
        unsigned rn = __builtin_amdgcn_readfirstlane(s_node[w][l]);
        float rm = s_max[w][l];
        // runs strictly inside the tile are complete
        if (lead && lane != fl && lane != ll) flush_b(nrec, node, dist);
        if (fl == ll) {
          if (fnode == rn) {
            rm = fmaxf(rm, fmx);
          } else {
            if (rn != kNone) flush_b(nrec, rn, rm);
            rn = fnode;
            rm = fmx;
          }
        } else {
          if (fnode == rn) {
            flush_b(nrec, rn, fmaxf(rm, fmx));
          } else {
            if (rn != kNone) flush_b(nrec, rn, rm);
            flush_b(nrec, fnode, fmx);
          }
          rn = lnode;
          rm = lmx;
        }
        s_node[w][l] = rn;  // same value from every lane
        s_max[w][l] = rm;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      const unsigned up = up0 < nn ? up0 : kNone;  // the root's parent is kNone
      node = part ? up : node;
      lv = part ? (up != kNone ? lv - 1 : -1) : lv;
    }
  }
  // carried runs of the last tile
  for (int l = 0; l < kMaxLevels; ++l) {
    const unsigned rn = __builtin_amdgcn_readfirstlane(s_node[w][l]);
    if (rn != kNone) flush_b(nrec, rn, s_max[w][l]);
  }
}

// Critical distance of the multipole MAC of Warren & Salmon (Section 2.2) for
// every node: b_J/2 + sqrt(b_J^2/4 + sqrt(3 B2 / delta)), B2 = trace of the
// second moments (sum m |r - r_J|^2), once b_J is final.
__global__ void __launch_bounds__(256)
mac_crit_k(const Ctl *__restrict__ ctl, float delta, const float4 *__restrict__ nrec,
           const float4 *__restrict__ quad, float *__restrict__ mcrit) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const int64_t nn = ctl->n_nodes;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const float b = nrec[2 * k + 1].x;
    const float B2 = quad[2 * k + 1].z;
    mcrit[k] = 0.5f * b + sqrtf(0.25f * b * b + sqrtf(3.0f * B2 / delta));
  }
}

void launch_moments(gothic_ctx *c, int64_t n, int nsys, hipStream_t s) {
  Buffers &B = c->b;
  // second moments for quadrupole terms and for the B2 of the multipole MAC
  const int wq = (c->prm.multipole == 2 || c->prm.mac == 2) ? 1 : 0;
  int64_t nb = (c->cap_nodes + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(leaf_moments_k, dim3(g), dim3(256), 0, s, B.ctl, n, B.first, B.count,
                     B.n_child, B.pos, B.leaf_of, B.nrec, B.quad, wq);
  for (int l = kNlev - 1; l >= 0; --l) {
    int64_t widest = nsys;
    for (int q = 0; q < l && widest < c->cap_nodes; ++q) widest *= 8;
    if (widest > c->cap_nodes) widest = c->cap_nodes;
    int64_t lb = (widest + 255) / 256;
    int gl = (int)(lb > 4096 ? 4096 : (lb < 1 ? 1 : lb));
    hipLaunchKernelGGL(internal_moments_k, dim3(gl), dim3(256), 0, s, l, B.ctl, B.child_first,
                       B.n_child, B.nrec, B.quad, wq);
  }
  // about 1024 particles per wave chunk (more waves only for small n)
  int64_t pb = (n + 4095) / 4096;
  int gp = (int)(pb > 16384 ? 16384 : (pb < 1 ? 1 : pb));
  hipLaunchKernelGGL(radius_k, dim3(gp), dim3(256), 0, s, B.ctl, n, B.pos, B.leaf_of, B.parent,
                     B.level, B.nrec);
  if (c->prm.mac == 2)
    hipLaunchKernelGGL(mac_crit_k, dim3(g), dim3(256), 0, s, B.ctl, c->prm.mac_delta, B.nrec,
                       B.quad, B.mcrit);
}

}  // namespace gothic
