// Pseudo j-particles (Section 2.1): for every node the total mass M_J, the
// centre of mass r_J and the radius b_J of the smallest sphere about r_J that
// holds all member particles; with multipole = 2 also the second moments
// S_ab = sum m (r - r_J)_a (r - r_J)_b.  Recomputed on every call, in FP32.
//   leaves:    straight from the member particles (centre of mass taken
//              relative to the first member, so a one-particle leaf has
//              r_J = r exactly and b_J = 0);
//   internal:  bottom-up one level at a time from the children (masses and
//              centres add; second moments by the parallel-axis rule);
//   b_J:       particle-parallel over the ancestor table written with the
//              tree: lanes of a wave that share an ancestor (always a
//              contiguous run in key order) max-reduce their distances; whole
//              nodes are stored, nodes shared between waves take an atomic max.
// The node record read by the walk is written here: (x, y, z, M) and
// (b_J, first|child_first, count|n_child, is_leaf).
#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr unsigned kNone = 0xffffffffu;

__device__ __forceinline__ float u2f(unsigned u) { return __uint_as_float(u); }

// a float moved between lanes of a row of 16 by a DPP control that gives
// every lane a source (row rotations, quad permutations)
template <int CTRL>
__device__ __forceinline__ float row_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// sum / max over aligned groups of L lanes (L = 4 or 16), in every lane:
// for L = 16 rotate by 8 and 4 within the row first; then swap lane pairs
// of each quad (quad_perm [2,3,0,1] and [1,0,3,2])
template <int L>
__device__ __forceinline__ float grp_sum(float v) {
  if (L == 16) {
    v += row_dpp<0x128>(v);  // row_ror:8
    v += row_dpp<0x124>(v);  // row_ror:4
  }
  v += row_dpp<0x4e>(v);
  v += row_dpp<0xb1>(v);
  return v;
}
template <int L>
__device__ __forceinline__ float grp_max(float v) {
  if (L == 16) {
    v = fmaxf(v, row_dpp<0x128>(v));
    v = fmaxf(v, row_dpp<0x124>(v));
  }
  v = fmaxf(v, row_dpp<0x4e>(v));
  v = fmaxf(v, row_dpp<0xb1>(v));
  return v;
}

// Leaves: L lanes per node (4 when leaves hold at most 16 particles, else
// 16), each lane taking members lane, lane + L, ... (coalesced loads, the
// first 4 L held in registers for both passes), sums and maxima reduced
// across the L lanes.  Groups whose node is internal take no part but run the
// same shuffles.
template <int L>
__global__ void __launch_bounds__(256)
leaf_moments_k(Ctl *__restrict__ ctl, int64_t n, const uint32_t *__restrict__ first,
               const uint32_t *__restrict__ count, const uint8_t *__restrict__ n_child,
               const float4 *__restrict__ pos, float4 *__restrict__ nrec,
               float4 *__restrict__ quad, int want_quad) {
  if (ctl->flags & kFlagNodeOverflow) return;  // incomplete tree: nothing to do
  constexpr int NPW = 64 / L;                  // nodes per wave pass
  const int64_t nn = ctl->n_nodes;
  const int lane = lane_id();
  const int rl = lane & (L - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t k0 = wave * NPW; k0 < nn; k0 += nwaves * NPW) {  // wave-uniform
    const int64_t k = k0 + lane / L;
    bool leaf = k < nn && n_child[k] == 0;
    const uint32_t f = leaf ? first[k] : 0u, c = leaf ? count[k] : 0u;
    if (leaf && (c == 0 || (int64_t)f + c > n)) {
      if (rl == 0) atomicOr(&ctl->flags, kFlagBadIndex);
      leaf = false;
    }
    const uint32_t cnt = leaf ? c : 0u;
    const float4 p0 = pos[leaf ? f : 0u];
    // the first 4 L members (all of them unless particles share a level-21
    // cell): up to four per lane, kept in registers for the second pass
    float4 m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t t = (uint32_t)rl + (uint32_t)L * u;
      m[u] = t < cnt ? pos[f + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      M += m[u].w;
      sx += m[u].w * (m[u].x - p0.x);
      sy += m[u].w * (m[u].y - p0.y);
      sz += m[u].w * (m[u].z - p0.z);
    }
    for (uint32_t t = (uint32_t)rl + 4u * L; t < cnt; t += L) {  // members past 4 L
      const float4 p = pos[f + t];
      M += p.w;
      sx += p.w * (p.x - p0.x);
      sy += p.w * (p.y - p0.y);
      sz += p.w * (p.z - p0.z);
    }
    M = grp_sum<L>(M);
    sx = grp_sum<L>(sx);
    sy = grp_sum<L>(sy);
    sz = grp_sum<L>(sz);
    float cx = p0.x, cy = p0.y, cz = p0.z;
    if (M > 0.f) {
      cx = p0.x + sx / M;
      cy = p0.y + sy / M;
      cz = p0.z + sz / M;
    }
    float b2 = 0.f, xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if ((uint32_t)rl + (uint32_t)L * u >= cnt) continue;
      const float4 p = m[u];
      const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
      b2 = fmaxf(b2, dx * dx + dy * dy + dz * dz);
      xx += p.w * dx * dx; yy += p.w * dy * dy; zz += p.w * dz * dz;
      xy += p.w * dx * dy; xz += p.w * dx * dz; yz += p.w * dy * dz;
    }
    for (uint32_t t = (uint32_t)rl + 4u * L; t < cnt; t += L) {
      const float4 p = pos[f + t];
      const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
      b2 = fmaxf(b2, dx * dx + dy * dy + dz * dz);
      xx += p.w * dx * dx; yy += p.w * dy * dy; zz += p.w * dz * dz;
      xy += p.w * dx * dy; xz += p.w * dx * dz; yz += p.w * dy * dz;
    }
    b2 = grp_max<L>(b2);
    if (want_quad) {
      xx = grp_sum<L>(xx); yy = grp_sum<L>(yy); zz = grp_sum<L>(zz);
      xy = grp_sum<L>(xy); xz = grp_sum<L>(xz); yz = grp_sum<L>(yz);
    } else {
      xx = yy = zz = xy = xz = yz = 0.f;
    }
    if (leaf && rl == 0) {
      const float b = (M > 0.f) ? sqrtf(b2) : 0.f;
      nrec[2 * k] = make_float4(cx, cy, cz, M);
      nrec[2 * k + 1] = make_float4(b, u2f(f), u2f(c), u2f(1u));
      quad[2 * k] = make_float4(xx, yy, zz, xy);
      quad[2 * k + 1] = make_float4(xz, yz, xx + yy + zz, 0.f);
    }
  }
}

// sum over the 8 lanes of a segment (lanes 8s .. 8s+7)
__device__ __forceinline__ float seg_sum8(float v) {
#pragma unroll
  for (int d = 4; d >= 1; d >>= 1) v += __shfl_xor(v, d, 8);
  return v;
}

// Internal nodes of level l from their children: 8 lanes per node, lane q
// reading child q (all children's records in flight at once), sums reduced
// across the 8 lanes; second moments about the new centre by the
// parallel-axis rule.
__device__ __forceinline__ void internal_level(int l, Ctl *ctl, const uint32_t *child_first,
                                               const uint8_t *n_child, float4 *nrec,
                                               float4 *quad, int want_quad, int64_t wave,
                                               int64_t nwaves) {
  const int64_t hi_all = ctl->n_nodes;
  const int64_t lo = ctl->lvl_start[l];
  int64_t hi = ctl->lvl_start[l + 1];
  if (hi > hi_all) hi = hi_all;
  const int lane = lane_id();
  const unsigned q = (unsigned)(lane & 7);
  for (int64_t k0 = lo + wave * 8; k0 < hi; k0 += nwaves * 8) {  // wave-uniform
    const int64_t k = k0 + (lane >> 3);
    const unsigned nc = k < hi ? n_child[k] : 0u;
    const uint32_t cf = nc ? child_first[k] : 0u;
    bool inner = nc != 0;
    if (inner && (cf <= k || (int64_t)cf + nc > hi_all)) {
      if (q == 0) atomicOr(&ctl->flags, kFlagBadIndex);
      inner = false;
    }
    const bool mine = inner && q < nc;  // this lane reads child q
    // Lanes without a child read record 0, the root, which this pass writes
    // last: it may hold anything (NaN included), so those lanes contribute
    // through selects, never through a product with a zero weight.
    const float4 r0 = nrec[2 * (size_t)(inner ? cf : 0u)];
    const float4 r = nrec[2 * (size_t)(mine ? cf + q : 0u)];
    const float w = mine ? r.w : 0.f;
    const float M = seg_sum8(w);
    const float sx = seg_sum8(mine ? w * (r.x - r0.x) : 0.f);
    const float sy = seg_sum8(mine ? w * (r.y - r0.y) : 0.f);
    const float sz = seg_sum8(mine ? w * (r.z - r0.z) : 0.f);
    float cx = r0.x, cy = r0.y, cz = r0.z;
    if (M > 0.f) {
      cx = r0.x + sx / M;
      cy = r0.y + sy / M;
      cz = r0.z + sz / M;
    }
    float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
    if (want_quad) {
      const size_t cq = 2 * (size_t)(mine ? cf + q : 0u);
      const float4 s0 = quad[cq], s1 = quad[cq + 1];
      const float dx = r.x - cx, dy = r.y - cy, dz = r.z - cz;
      xx = seg_sum8(mine ? s0.x + w * dx * dx : 0.f);
      yy = seg_sum8(mine ? s0.y + w * dy * dy : 0.f);
      zz = seg_sum8(mine ? s0.z + w * dz * dz : 0.f);
      xy = seg_sum8(mine ? s0.w + w * dx * dy : 0.f);
      xz = seg_sum8(mine ? s1.x + w * dx * dz : 0.f);
      yz = seg_sum8(mine ? s1.y + w * dy * dz : 0.f);
    }
    if (inner && q == 0) {
      nrec[2 * k] = make_float4(cx, cy, cz, M);
      nrec[2 * k + 1] = make_float4(0.f, u2f(cf), u2f(nc), u2f(0u));
      quad[2 * k] = make_float4(xx, yy, zz, xy);
      quad[2 * k + 1] = make_float4(xz, yz, xx + yy + zz, 0.f);
    }
  }
}


__global__ void __launch_bounds__(256)
internal_moments_k(int l, Ctl *__restrict__ ctl, const uint32_t *__restrict__ child_first,
                   const uint8_t *__restrict__ n_child, float4 *__restrict__ nrec,
                   float4 *__restrict__ quad, int want_quad) {
  if (ctl->flags & kFlagNodeOverflow) return;
  internal_level(l, ctl, child_first, n_child, nrec, quad, want_quad,
                 ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6,
                 ((int64_t)gridDim.x * blockDim.x) >> 6);
}

// Small trees (systems of at most kSmallMoments particles, a bound the host
// knows): every level in one workgroup, deepest first, a barrier between
// levels, instead of one launch per level.
constexpr int kSmallMoments = 8192;

__global__ void __launch_bounds__(1024)
internal_moments_small_k(Ctl *__restrict__ ctl, const uint32_t *__restrict__ child_first,
                         const uint8_t *__restrict__ n_child, float4 *nrec, float4 *quad,
                         int want_quad) {
  if (ctl->flags & kFlagNodeOverflow) return;
  for (int l = kNlev - 1; l >= 0; --l) {
    internal_level(l, ctl, child_first, n_child, nrec, quad, want_quad, threadIdx.x >> 6,
                   blockDim.x >> 6);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- b_J
// Every particle's ancestors are written once per tree into a level-major
// table (anc[l * n + k] = the level-l ancestor of key-ordered particle k, for
// l below its leaf's level).  The radius pass then works on contiguous chunks
// of particles, one wave per chunk, in tiles of 64: a node's particles are
// contiguous, so at every level the ancestors of a tile form runs.  A run
// that starts and ends inside the wave's chunk is a whole node and its
// maximum is stored; runs that may reach past either end of the chunk are
// combined across waves with an atomic max.  The last run of every level is
// carried from tile to tile in LDS.
__global__ void __launch_bounds__(256)
leaf_map_k(const Ctl *__restrict__ ctl, int64_t n, const uint32_t *__restrict__ first,
           const uint32_t *__restrict__ count, const uint8_t *__restrict__ n_child,
           uint32_t *__restrict__ leaf_of) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const int64_t nn = ctl->n_nodes;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (n_child[k] != 0) continue;
    const uint32_t f = first[k], c = count[k];
    if ((int64_t)f + c > n) continue;
    for (uint32_t j = f; j < f + c; ++j) leaf_of[j] = (uint32_t)k;
  }
}

__global__ void __launch_bounds__(256)
ancestors_k(Ctl *__restrict__ ctl, int64_t n, const uint32_t *__restrict__ leaf_of,
            const uint32_t *__restrict__ parent, const uint8_t *__restrict__ level,
            uint32_t *__restrict__ anc, uint8_t *__restrict__ leaflev) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const unsigned nn = ctl->n_nodes;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    uint32_t node = leaf_of[k];
    if (node >= nn) {
      atomicOr(&ctl->flags, kFlagBadIndex);
      leaflev[k] = 0;
      continue;
    }
    const int L = level[node];
    leaflev[k] = (uint8_t)L;
    for (int l = L - 1; l >= 0; --l) {
      const uint32_t up = parent[node];
      node = up < nn ? up : 0u;
      anc[(int64_t)l * n + k] = node;
    }
  }
}

constexpr int kRadiusWaves = 4;  // waves per workgroup

// per wave and level: the run carried from tile to tile
struct RadiusCarry {
  unsigned node[kRadiusWaves][kMaxLevels];
  float max[kRadiusWaves][kMaxLevels];
  unsigned open[kRadiusWaves][kMaxLevels];  // the run may hold particles before the chunk
};

// the radius of a node seen by one wave: stored if the wave saw all of the
// node's particles, else an atomic max (radii are >= 0, so their bit
// patterns order like the values); one lane writes
__device__ __forceinline__ void put_b(float4 *nrec, unsigned node, float v, bool shared_node) {
  if (lane_id() == 0) {
    float *dst = &nrec[2 * (size_t)node + 1].x;
    if (shared_node) atomicMax(reinterpret_cast<unsigned *>(dst), __float_as_uint(v));
    else *dst = v;
  }
}

// DPP lane moves within the wave (gfx9 encodings): row_shr:1,2,4,8 shift
// inside each row of 16 lanes, row_bcast:15 / row_bcast:31 carry the last
// lane of a row into the next row(s), wave_shr:1 shifts the whole wave by
// one lane.  Lanes without a source read `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_move(unsigned v, unsigned old) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}

// inclusive max scan from lane 0 upward, restarted at lanes with head set:
// the last lane of each run of lanes ends up with the run's maximum.
// Values are non-negative floats, whose bit patterns order like the values.
__device__ __forceinline__ unsigned seg_max_scan(unsigned v, unsigned head) {
#define GOTHIC_SEG_STEP(ctrl, rows)                   \
  {                                                   \
    const unsigned ov = dpp_move<ctrl, rows>(v, 0u);  \
    const unsigned oh = dpp_move<ctrl, rows>(head, 0u); \
    v = head ? v : max(v, ov);                        \
    head |= oh;                                       \
  }
  GOTHIC_SEG_STEP(0x111, 0xf)
  GOTHIC_SEG_STEP(0x112, 0xf)
  GOTHIC_SEG_STEP(0x114, 0xf)
  GOTHIC_SEG_STEP(0x118, 0xf)
  GOTHIC_SEG_STEP(0x142, 0xa)
  GOTHIC_SEG_STEP(0x143, 0xc)
#undef GOTHIC_SEG_STEP
  return v;
}

// one level of one tile: lane holds (key = node or kNone, dist); at_start:
// the tile is the first of the chunk
__device__ __forceinline__ void radius_level(float4 *nrec, RadiusCarry &rc, int w, int l,
                                             unsigned key, float dist, bool at_start) {
  const int lane = lane_id();
  // one node under the whole tile (the tiles of the upper levels): keys are
  // contiguous runs, so equal first and last keys mean a single run, whose
  // maximum is a plain scan over the wave
  const unsigned k0 = (unsigned)__builtin_amdgcn_readfirstlane((int)key);
  const unsigned k63 = (unsigned)__builtin_amdgcn_readlane((int)key, 63);
  if (k0 == k63 && k0 != kNone) {
    const float mx = __uint_as_float(wave_last(wave_incl_max(__float_as_uint(dist))));
    unsigned rn = __builtin_amdgcn_readfirstlane(rc.node[w][l]);
    float rm = rc.max[w][l];
    bool ropen = __builtin_amdgcn_readfirstlane(rc.open[w][l]) != 0u;
    if (k0 == rn) {
      rm = fmaxf(rm, mx);
    } else {
      if (rn != kNone) put_b(nrec, rn, rm, ropen);
      rn = k0;
      rm = mx;
      ropen = at_start;
    }
    rc.node[w][l] = rn;  // same value from every lane
    rc.max[w][l] = rm;
    rc.open[w][l] = ropen ? 1u : 0u;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return;
  }
  const bool part = key != kNone;
  // runs of equal key: heads from the previous lane's key, the run maximum
  // at each run's last lane
  const unsigned prev = dpp_move<0x138, 0xf>(key, ~key);
  const unsigned next = __shfl_down(key, 1, 64);
  const unsigned head = (lane == 0 || prev != key) ? 1u : 0u;
  const float run_max = __uint_as_float(seg_max_scan(__float_as_uint(dist), head));
  const bool tail = part && (lane == 63 || next != key);
  const unsigned long long tm = __ballot(tail);
  if (!tm) return;
  const int fl = __builtin_amdgcn_readfirstlane(__ffsll((long long)tm) - 1);
  const int ll = __builtin_amdgcn_readfirstlane(63 - __clzll((long long)tm));
  const unsigned fnode = (unsigned)__builtin_amdgcn_readlane((int)key, fl);
  const unsigned lnode = (unsigned)__builtin_amdgcn_readlane((int)key, ll);
  const float fmx = __uint_as_float((unsigned)__builtin_amdgcn_readlane(
      (int)__float_as_uint(run_max), fl));
  const float lmx = __uint_as_float((unsigned)__builtin_amdgcn_readlane(
      (int)__float_as_uint(run_max), ll));
  // the first run reaches back to lane 0 iff lane 0 holds a particle of it
  const bool first_open =
      at_start && (unsigned)__builtin_amdgcn_readfirstlane((int)key) == fnode;
  unsigned rn = __builtin_amdgcn_readfirstlane(rc.node[w][l]);
  float rm = rc.max[w][l];
  bool ropen = __builtin_amdgcn_readfirstlane(rc.open[w][l]) != 0u;
  // runs strictly inside the tile are whole nodes
  if (tail && lane != fl && lane != ll) nrec[2 * (size_t)key + 1].x = run_max;
  if (fl == ll) {
    if (fnode == rn) {
      rm = fmaxf(rm, fmx);
    } else {
      if (rn != kNone) put_b(nrec, rn, rm, ropen);
      rn = fnode;
      rm = fmx;
      ropen = first_open;
    }
  } else {
    if (fnode == rn) {
      put_b(nrec, rn, fmaxf(rm, fmx), ropen);
    } else {
      if (rn != kNone) put_b(nrec, rn, rm, ropen);
      put_b(nrec, fnode, fmx, first_open);
    }
    rn = lnode;
    rm = lmx;
    ropen = false;
  }
  rc.node[w][l] = rn;  // same value from every lane
  rc.max[w][l] = rm;
  rc.open[w][l] = ropen ? 1u : 0u;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(256)
radius_k(Ctl *__restrict__ ctl, int64_t n, const float4 *__restrict__ pos,
         const uint32_t *__restrict__ anc, const uint8_t *__restrict__ leaflev,
         float4 *__restrict__ nrec) {
  if (ctl->flags & kFlagNodeOverflow) return;
  const unsigned nn = ctl->n_nodes;
  __shared__ RadiusCarry rc;
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  if (lane < kMaxLevels) {
    rc.node[w][lane] = kNone;
    rc.max[w][lane] = 0.f;
    rc.open[w][lane] = 0u;
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
    const int L = inr ? (int)leaflev[ic] : 0;  // ancestors at levels 0 .. L-1
    int top = L - 1;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) top = max(top, __shfl_xor(top, d, 64));
    top = __builtin_amdgcn_readfirstlane(top);
    // the nodes of four levels are loaded before they are reduced
    for (int l0 = top; l0 >= 0; l0 -= 4) {
      unsigned nd[4];
      float4 rr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int l = l0 - u;
        const bool part = l >= 0 && l < L;
        const unsigned a = part ? anc[(int64_t)l * n + ic] : kNone;
        nd[u] = (part && a < nn) ? a : kNone;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) rr[u] = nrec[2 * (size_t)(nd[u] != kNone ? nd[u] : 0u)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int l = l0 - u;
        if (l < 0) break;  // uniform
        const float4 r = rr[u];
        const float dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
        const float dist = (nd[u] != kNone && r.w > 0.f) ? sqrtf(dx * dx + dy * dy + dz * dz) : 0.f;
        radius_level(nrec, rc, w, l, nd[u], dist, base == c0);
      }
    }
  }
  // The carried runs may continue in the next chunk: one lane per level
  // combines them with an atomic max.  Near the root every wave's run is the
  // same node, so the atomic is skipped when the stored radius is already
  // at least as large (radii only grow during the pass, so a stale read can
  // only lead to an unneeded atomic, never to a missed one).
  if (lane < kMaxLevels) {
    const unsigned rn = rc.node[w][lane];
    if (rn != kNone) {
      unsigned *dst = reinterpret_cast<unsigned *>(&nrec[2 * (size_t)rn + 1].x);
      const unsigned v = __float_as_uint(rc.max[w][lane]);
      if (v > *dst) atomicMax(dst, v);
    }
  }
}

void launch_ancestors(gothic_ctx *c, int64_t n, hipStream_t s) {
  Buffers &B = c->b;
  int64_t nb = (c->cap_nodes + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(leaf_map_k, dim3(g), dim3(256), 0, s, B.ctl, n, B.first, B.count, B.n_child,
                     B.leaf_of);
  int64_t pb = (n + 255) / 256;
  int gp = (int)(pb > 8192 ? 8192 : (pb < 1 ? 1 : pb));
  hipLaunchKernelGGL(ancestors_k, dim3(gp), dim3(256), 0, s, B.ctl, n, B.leaf_of, B.parent,
                     B.level, B.anc, B.leaflev);
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
  int64_t nb = (c->cap_nodes + 15) / 16;  // 16 nodes per workgroup pass
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  if (c->prm.n_leaf <= 16) {
    int64_t nb4 = (c->cap_nodes + 63) / 64;  // 64 nodes per workgroup pass
    int g4 = (int)(nb4 > 8192 ? 8192 : (nb4 < 1 ? 1 : nb4));
    hipLaunchKernelGGL(leaf_moments_k<4>, dim3(g4), dim3(256), 0, s, B.ctl, n, B.first, B.count,
                       B.n_child, B.pos, B.nrec, B.quad, wq);
  } else {
    hipLaunchKernelGGL(leaf_moments_k<16>, dim3(g), dim3(256), 0, s, B.ctl, n, B.first, B.count,
                       B.n_child, B.pos, B.nrec, B.quad, wq);
  }
  if (n <= kSmallMoments) {
    hipLaunchKernelGGL(internal_moments_small_k, dim3(1), dim3(1024), 0, s, B.ctl, B.child_first,
                       B.n_child, B.nrec, B.quad, wq);
  } else {
    for (int l = kNlev - 1; l >= 0; --l) {
      int64_t widest = nsys;
      for (int q = 0; q < l && widest < c->cap_nodes; ++q) widest *= 8;
      if (widest > c->cap_nodes) widest = c->cap_nodes;
      int64_t lb = (widest + 31) / 32;  // 32 nodes per workgroup pass
      int gl = (int)(lb > 4096 ? 4096 : (lb < 1 ? 1 : lb));
      hipLaunchKernelGGL(internal_moments_k, dim3(gl), dim3(256), 0, s, l, B.ctl,
                         B.child_first, B.n_child, B.nrec, B.quad, wq);
    }
  }
  // about 1024 particles per wave chunk; small systems take chunks of down
  // to one tile of 64 so that at least 256 workgroups share the levels' work
  int64_t pb = (n + 4095) / 4096;
  if (pb < 256) {
    const int64_t small = (n + 255) / 256;
    pb = small < 256 ? small : 256;
  }
  int gp = (int)(pb > 16384 ? 16384 : (pb < 1 ? 1 : pb));
  hipLaunchKernelGGL(radius_k, dim3(gp), dim3(256), 0, s, B.ctl, n, B.pos, B.anc, B.leaflev,
                     B.nrec);
  if (c->prm.mac == 2)
    hipLaunchKernelGGL(mac_crit_k, dim3(g), dim3(256), 0, s, B.ctl, c->prm.mac_delta, B.nrec,
                       B.quad, B.mcrit);
}

}  // namespace gothic
