// Tree walk and force (Sections 2.2, 2.3 and 2.5 of the paper).
//
// One wave64 walks the tree for one group of G i-particles at a time
// (persistent waves claim groups from a device counter).  In a batched
// evaluation every group belongs to one system and starts at that system's
// root with that system's softening and opening angle, so one launch walks
// all systems.  The group is
// represented by its pseudo i-particle (r_I, b_I); a candidate pseudo
// j-particle J is at distance d = lambda r_JI with lambda = 1 - b_I / r_JI
// (0 when b_I >= r_JI), and is accepted when b_J <= theta d (the opening-angle
// MAC of Barnes & Hut written without the division), or by the acceleration
// or multipole MAC of Section 2.2 (params.mac).  Up to 64 pending
// nodes are tested at once, one per lane, and ballot/prefix-sum compaction
// routes
//   accepted nodes        -> the LDS interaction list (pseudo particles),
//   rejected internal     -> their children onto the pending stack,
//   rejected leaves       -> their member particles to the LDS list.
// The pending nodes form a last-in-first-out stack whose top lives in LDS
// and whose older part spills to a per-wave global stack.  Taking the
// newest 64 nodes first keeps the stack near depth x 512 entries, where a
// first-in-first-out frontier would grow to a whole tree level for groups
// spread over the system (sparse block-step groups).  The set of interactions
// does not depend on the order in which pending nodes are tested.
// When the list is full it is flushed: every lane accumulates the softened
// force and potential of its i-particle from the list entries (broadcast LDS
// reads, FP32 with the hardware reciprocal square root).  A group of gc <= G
// particles is laid out on the fewest power-of-two slots that hold it, and the
// S = 64 / slots lanes sharing an i-particle take every S-th entry
// (ij-parallelisation) and are summed at the end.  Each flush's partial sums
// are added to the running totals with Neumaier compensation (or plainly).
//
// Pair terms with d = r_J - r_i, R^2 = |d|^2 + eps^2:
//   monopole    a += M d / R^3,  phi -= M / R
//   quadrupole  a += d (7.5 q / R^7 - 1.5 tr S / R^5) - 3 S d / R^5,
//               phi -= 1.5 q / R^5 - 0.5 tr S / R^3,   q = d.S.d
// (evaluated in the factored form given at flush()).
// (second-order Taylor term of the softened kernel about the centre of mass).
// The self pair adds no force and m_i/eps to -phi, which is removed.
#include "common.h"
#include "primitives.h"

namespace gothic {

// LDS part of the pending stack per wave: room for the children of 64 opened
// nodes (8 each), so one batch's pushes always fit once older entries spill
constexpr int kQueueCap = 512;
constexpr int kQueueSlack = 8;   // above the LDS stack: the child writes run up to 7 past it
constexpr int kXcds = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kSpillChunk = 256;  // entries moved to the global stack at a time

struct WalkArgs {
  Ctl *ctl;
  int64_t n;
  const float4 *nrec;
  const float4 *quad;
  const float4 *pos;
  const uint32_t *alist;
  const uint32_t *gfirst;
  const float4 *ball;
  const uint32_t *perm;
  float4 *out;
  uint32_t *gent;
  uint32_t *spill;
  int64_t spill_cap;
  const SysRec *sys;
  const uint32_t *soff;
  const float *gamin;   // acceleration MAC: smallest |a_old| per group
  const float *mcrit;   // multipole MAC: critical distance per node
  float mac_delta;
  int mac;              // 0 opening angle, 1 acceleration, 2 multipole (Warren-Salmon)
  int G, logG, D, DQ;
  int wave_bytes;       // LDS of a wave
  int seg_bytes;        // LDS of one walk of a wave (W < 64: 64 / W walks per wave)
  int compensated;
  // list read-back: the groups gsel[0 .. ngsel) are walked (each by the waves
  // in turn, no claim counters) and every accepted node J is recorded as J,
  // every opened leaf J as J | kRecLeaf, in rec[k * rec_cap ...] for the k-th
  // listed group, with its node and leaf counts in rec_n[2k], rec_n[2k + 1]
  const uint32_t *gsel;
  unsigned ngsel;
  uint32_t *rec, *rec_n;
  int64_t rec_cap;
};

constexpr uint32_t kRecLeaf = 0x80000000u;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void neumaier(float &sum, float &c, float x) {
  const float t = sum + x;
  c += (fabsf(sum) >= fabsf(x)) ? ((sum - t) + x) : ((x - t) + sum);
  sum = t;
}

struct Acc {
  float x, y, z, p;     // running sums (p = sum of m/R, i.e. -phi)
  float cx, cy, cz, cp; // compensation terms
};

// Lanes per i-particle S = 2^LOGS; LOGS < 0 reads it at run time.  A
// compile-time S lets the unrolled list reads use immediate LDS offsets.
template <int LOGS>
__device__ __forceinline__ int lanes_per_i(int S) {
  return LOGS >= 0 ? (1 << LOGS) : S;
}

// Quadrupole list entries hold three float4 (one LDS array, 48 bytes each):
//   (x, y, z, M), (3Sxx, 3Syy, 3Szz, 3Sxy), (3Sxz, 3Syz, -tr/2, -3tr/2)
// so that with d = r_J - r_i, ri = 1/R, u = ri^2, s = 3 S d, w = 1.5 u d.S.d:
//   a   += d ri^3 (M + u (5 w - 1.5 tr)) - u ri^3 s
//   phi -= ri (M + u (w - 0.5 tr))

// one monopole list entry j on the i-particle at pi
__device__ __forceinline__ void mono_term(const float4 j, const float4 pi, float eps2, float &fx,
                                          float &fy, float &fz, float &fp) {
  const float dx = j.x - pi.x, dy = j.y - pi.y, dz = j.z - pi.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float mr = j.w * ri;
  const float mr3 = mr * ri * ri;
  fp += mr;
  fx = fmaf(mr3, dx, fx);
  fy = fmaf(mr3, dy, fy);
  fz = fmaf(mr3, dz, fz);
}

// one quadrupole list entry (q0, q1, q2) on the i-particle at pi; with
// v = u d.(3S).d = 2w the two uses of w become fused multiply-adds
__device__ __forceinline__ void quad_term(const float4 q0, const float4 q1, const float4 q2,
                                          const float4 pi, float eps2, float &fx, float &fy,
                                          float &fz, float &fp) {
  const float dx = q0.x - pi.x, dy = q0.y - pi.y, dz = q0.z - pi.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float u = ri * ri;
  const float ri3 = ri * u;
  // s = 3 S d   (q1 = 3(xx yy zz xy), q2 = 3(xz yz) | -tr/2, -3tr/2)
  const float sx = fmaf(q1.x, dx, fmaf(q1.w, dy, q2.x * dz));
  const float sy = fmaf(q1.w, dx, fmaf(q1.y, dy, q2.y * dz));
  const float sz = fmaf(q2.x, dx, fmaf(q2.y, dy, q1.z * dz));
  const float v = u * fmaf(dx, sx, fmaf(dy, sy, dz * sz));  // 3 u d.S.d = 2w
  const float coef = ri3 * fmaf(u, fmaf(2.5f, v, q2.w), q0.w);
  const float r5 = ri3 * u;
  fx = fmaf(-r5, sx, fmaf(coef, dx, fx));
  fy = fmaf(-r5, sy, fmaf(coef, dy, fy));
  fz = fmaf(-r5, sz, fmaf(coef, dz, fz));
  fp = fmaf(ri, fmaf(u, fmaf(0.5f, v, q2.z), q0.w), fp);
}

// The list is split into rounds of S entries, lane sub of an i-particle
// taking entry round * S + sub.  Full rounds run under wave-uniform loop
// control (scalar compare, immediate LDS offsets in the unrolled body); the
// last partial round, if any, under per-lane control.  LISTS selects the
// lists evaluated (bit 0 particles, bit 1 quadrupole nodes): a full list is
// flushed alone, both at the end of the walk.
template <int MULTI, int LOGS, int LISTS = 3>
__device__ __forceinline__ void flush(const WalkArgs &a, const float4 *pl, const float4 *ql,
                                      int np, int nq, float4 pi, float eps2, int sub, int S_rt,
                                      Acc &acc) {
  wave_sync();
  const int S = lanes_per_i<LOGS>(S_rt);
  float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
  if (LISTS & 1) {
    constexpr int U = 4;
    const float4 *pj = pl + sub;
    int k0 = 0;
    for (; k0 + U * S <= np; k0 += U * S) {
#pragma unroll
      for (int u = 0; u < U; ++u) mono_term(pj[k0 + u * S], pi, eps2, fx, fy, fz, fp);
    }
    for (int k = k0 + sub; k < np; k += S) mono_term(pl[k], pi, eps2, fx, fy, fz, fp);
  }
  if (MULTI == 2 && (LISTS & 2)) {
    constexpr int U = 2;
    const float4 *qj = ql + 3 * sub;
    int k0 = 0;
    for (; k0 + U * S <= nq; k0 += U * S) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float4 *q = qj + 3 * (k0 + u * S);
        quad_term(q[0], q[1], q[2], pi, eps2, fx, fy, fz, fp);
      }
    }
    for (int k = k0 + sub; k < nq; k += S)
      quad_term(ql[3 * k], ql[3 * k + 1], ql[3 * k + 2], pi, eps2, fx, fy, fz, fp);
  }
  if (a.compensated) {
    neumaier(acc.x, acc.cx, fx);
    neumaier(acc.y, acc.cy, fy);
    neumaier(acc.z, acc.cz, fz);
    neumaier(acc.p, acc.cp, fp);
  } else {
    acc.x += fx; acc.y += fy; acc.z += fz; acc.p += fp;
  }
  wave_sync();
}

// The flush for a group's lane shape: shape 0 is the kernel's own (G
// i-particles, S = 64 / G lanes each), shape 1 half as many i-particles with
// twice the lanes (both with compile-time S), shape 2 fewer still (run-time S).
template <int MULTI, int LOGS, int LISTS = 3>
__device__ __forceinline__ void flush_shape(int shape, const WalkArgs &a, const float4 *pl,
                                            const float4 *ql, int np, int nq, float4 pi,
                                            float eps2, int sub, int S, Acc &acc) {
  constexpr int LOGS1 = LOGS >= 0 && LOGS < 6 ? LOGS + 1 : -1;
  if (shape == 0) flush<MULTI, LOGS, LISTS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
  else if (shape == 1) flush<MULTI, LOGS1, LISTS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
  else flush<MULTI, -1, LISTS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
}

template <int MULTI, int LOGS, bool REC>
__global__ void __launch_bounds__(256) walk_k(WalkArgs a) {
  extern __shared__ float4 smem[];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  char *wbase = reinterpret_cast<char *>(smem) + (size_t)w * a.wave_bytes;
  float4 *pl = reinterpret_cast<float4 *>(wbase);
  float4 *ql = pl + a.D;  // quadrupole entries, three float4 each
  uint32_t *queue = reinterpret_cast<uint32_t *>(ql + (MULTI == 2 ? 3 * a.DQ : 0));
  uint32_t *tpre = queue + kQueueCap + kQueueSlack;
  uint32_t *tsrc = tpre + 64;

  const int64_t slot = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
  // Every value that steers a loop below is wave-uniform and kept in scalar
  // registers (readfirstlane / ballot), and no lane-dependent branch encloses
  // a cross-lane operation inside a loop: the compiler may otherwise split the
  // loops by lane and leave a shuffle reading an inactive lane.
  uint32_t *spill = a.spill + slot * a.spill_cap;
  const int G = a.G;
  Ctl *ctl = a.ctl;
  if (ctl->flags & kFlagNodeOverflow) return;  // no valid tree: the host repeats
  const unsigned ng = ctl->n_groups, nn = ctl->n_nodes, nsys = ctl->nsys;
  const unsigned nwork = REC ? a.ngsel : ng;
  const int D = a.D, DQ = a.DQ;
  // with fewer groups than waves the surplus waves have nothing to claim:
  // they leave before touching the shared counters
  if (slot >= (int64_t)nwork) return;

  unsigned long long t_node = 0, t_part = 0, t_int = 0, t_nint = 0, t_mac = 0;
  // XCD-aware work distribution: the groups (key order, hence spatially
  // ordered) are cut into kXcds contiguous ranges; the waves of a workgroup
  // on XCD x (blockIdx % kXcds under round-robin dispatch) drain range x
  // first, so neighbouring groups share that XCD's L2, then help elsewhere.
  unsigned xr = blockIdx.x % kXcds;
  int tried = 0;
  int64_t rec_item = slot;
  const int64_t nslots = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (;;) {
    unsigned g = ng;
    unsigned rk = 0;  // REC: position of g in the work list
    if (REC) {
      if (rec_item < (int64_t)nwork) {
        rk = (unsigned)rec_item;
        g = a.gsel[rk];
        if (g >= ng) g = ng;
        rec_item += nslots;
      }
      tried = kXcds;
    }
    while (tried < kXcds) {
      const unsigned lo = (unsigned)(((unsigned long long)xr * ng) / kXcds);
      const unsigned hi = (unsigned)(((unsigned long long)(xr + 1) * ng) / kXcds);
      const unsigned cl =
          __builtin_amdgcn_readfirstlane(atomicAdd(&ctl->xwork[kXworkStride * xr], lane == 0 ? 1u : 0u));
      if (lo + cl < hi) {
        g = lo + cl;
        break;
      }
      ++tried;
      xr = (xr + 1) % kXcds;
    }
    if (g >= ng) break;
    const unsigned gs = a.gfirst[g];
    const unsigned ge = a.gfirst[g + 1];
    const int gc0 = (int)(ge > gs ? ge - gs : 0u);
    const int gc = gc0 < G ? gc0 : G;
    const float4 bl = a.ball[g];
    // The group's gc particles take the fewest of 2^lgx <= G slots that hold
    // them, each slot S = 64 / 2^lgx lanes: a group split short by r_crit
    // (sparse regions, few active particles) keeps every lane of the flush.
    int lgx = a.logG;
    while (lgx > 0 && (1 << (lgx - 1)) >= gc) --lgx;  // wave-uniform
    const int shape = lgx == a.logG ? 0 : (lgx == a.logG - 1 ? 1 : 2);
    const int Gx = 1 << lgx, S = 64 >> lgx;
    const int il = lane & (Gx - 1), sub = lane >> lgx;
    const bool vi = il < gc;
    const uint32_t ki0 = a.alist[gs + (vi ? il : 0)];
    const uint32_t ki = ki0 < a.n ? ki0 : 0u;
    const float4 pi = a.pos[ki];
    // the group's system (groups never span two): its root is node sys
    const uint32_t k_first = __builtin_amdgcn_readfirstlane(a.alist[gs]);
    const unsigned sy = __builtin_amdgcn_readfirstlane(
        sys_of(a.soff, nsys, k_first < a.n ? k_first : 0u));
    const float eps2 = a.sys[sy].eps2, theta = a.sys[sy].theta, inv_eps = a.sys[sy].inv_eps;
    // acceleration MAC: accept when m b^2 <= (delta |a_old|_min) d^4
    const float dfac = a.mac == 1 ? a.mac_delta * a.gamin[g] : 0.f;
    Acc acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int np = 0, nq = 0;
    // the LDS stack holds the newest entries [0, qt), the global stack the
    // older entries [0, stop)
    unsigned qt = 1;
    int64_t stop = 0;
    unsigned long long e_node = 0, e_part = 0, n_mac = 0;
    int64_t rec_len = 0, rec_leaves = 0;
    if (lane == 0) queue[0] = sy;
    wave_sync();

    // a valid walk pops every node at most once; the bound only guards
    // against a corrupted tree
    unsigned long long pops = 0;
    while ((qt > 0 || stop > 0) && pops <= (unsigned long long)nn) {
      if (qt == 0) {  // LDS part empty: bring back the newest spilled entries
        // the spill entries were written by other lanes of this wave
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        const int64_t m = stop < kQueueCap / 2 ? stop : kQueueCap / 2;
        for (int64_t t = lane; t < m; t += 64) queue[t] = spill[stop - m + t];
        stop -= m;
        qt = (unsigned)m;
        wave_sync();
      }
      const unsigned nb = qt < 64u ? qt : 64u;
      const bool has = (unsigned)lane < nb;
      // below max(qt, 64) <= kQueueCap for every lane
      const unsigned qv = queue[qt - nb + lane];
      // lanes without a node read the root; an entry past the node count
      // (never produced by a valid tree) is dropped the same way
      const unsigned node = (has && qv < nn) ? qv : 0u;
      qt -= nb;  // pop the newest nb entries
      n_mac += nb;
      pops += nb;
      const float4 r0 = a.nrec[2 * (size_t)node];
      const float4 r1 = a.nrec[2 * (size_t)node + 1];
      // the second moments are read with the record, before the MAC decides
      // whether they are needed, so the two loads share one wait
      float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
      if (MULTI == 2) {
        s0 = a.quad[2 * (size_t)node];
        s1 = a.quad[2 * (size_t)node + 1];
      }
      const float dx = r0.x - bl.x, dy = r0.y - bl.y, dz = r0.z - bl.z;
      // the hardware square root (within 1 ulp): the MAC decision it feeds
      // is only sensitive far beyond that
      const float rji = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
      const float dist = fmaxf(rji - bl.w, 0.f);
      // multipole acceptance (Section 2.2); with the acceleration and
      // multipole MACs a node of positive size that may hold a member of the
      // group (b_J >= d) is never accepted
      bool mac_ok;
      if (a.mac == 0) {
        mac_ok = r1.x <= theta * dist;
      } else {
        const bool outside = !(r1.x > 0.f && r1.x >= dist);
        if (a.mac == 1) {
          const float d2 = dist * dist;
          mac_ok = outside && (r0.w * r1.x * r1.x <= dfac * (d2 * d2));
        } else {
          mac_ok = outside && (a.mcrit[node] <= dist);
        }
      }
      const bool accept = has && qv < nn && mac_ok;
      const bool leaf = __float_as_uint(r1.w) != 0u;
      const bool open_leaf = has && qv < nn && !accept && leaf;
      const bool open_int = has && qv < nn && !accept && !leaf;
      if (REC) {
        const unsigned long long rm = __ballot(accept || open_leaf);
        const int64_t at = rec_len + (int64_t)lanes_below(rm);
        if ((accept || open_leaf) && at < a.rec_cap)
          a.rec[(int64_t)rk * a.rec_cap + at] = node | (open_leaf ? kRecLeaf : 0u);
        rec_len += __popcll(rm);
        rec_leaves += __popcll(__ballot(open_leaf));
      }

      // (1) accepted pseudo j-particles
      const unsigned long long am = __ballot(accept);
      const int nacc = __popcll(am);
      if (nacc) {
        if (MULTI == 1) {
          if (np + nacc > D) {
            flush_shape<MULTI, LOGS>(shape, a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            np = 0; nq = 0;
          }
          if (accept) pl[np + lanes_below(am)] = r0;
          np += nacc;
        } else {
          if (nq + nacc > DQ) {
            flush_shape<MULTI, LOGS, 2>(shape, a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            nq = 0;
          }
          if (accept) {
            const int q = nq + (int)lanes_below(am);
            ql[3 * q] = r0;
            ql[3 * q + 1] = make_float4(3.f * s0.x, 3.f * s0.y, 3.f * s0.z, 3.f * s0.w);
            ql[3 * q + 2] = make_float4(3.f * s1.x, 3.f * s1.y, -0.5f * s1.z, -1.5f * s1.z);
          }
          nq += nacc;
        }
        e_node += (unsigned)nacc;
      }

      // (2) children of rejected internal nodes -> pending stack
      const unsigned nc0 = open_int ? __float_as_uint(r1.z) : 0u;
      const unsigned nc = nc0 < 8u ? nc0 : 8u;  // an octree node has at most eight
      const unsigned cf = __float_as_uint(r1.y);
      unsigned cinc = wave_incl_sum(nc);
      const unsigned C = wave_last(cinc);
      if (C) {
        // keeps the compiler from rebuilding cinc - nc out of the scan's terms
        asm volatile("" : "+v"(cinc));
        const unsigned pre = cinc - nc;
        if (qt + C > (unsigned)kQueueCap) {
          // move the oldest LDS entries to the global stack to make room
          unsigned k = qt + C - (unsigned)kQueueCap;
          k = (k + kSpillChunk - 1) / kSpillChunk * kSpillChunk;
          if (k > qt) k = qt;
          if (stop + k <= a.spill_cap) {
            for (unsigned t = lane; t < k; t += 64) spill[stop + t] = queue[t];
            stop += k;
            // shift the remaining entries to the bottom, 64 at a time from
            // the bottom up: each round reads above what it writes
            const unsigned rest = qt - k;
            for (unsigned t0 = 0; t0 < rest; t0 += 64) {
              const unsigned t = t0 + lane;
              const uint32_t v = t < rest ? queue[k + t] : 0u;
              wave_sync();
              if (t < rest) queue[t] = v;
              wave_sync();
            }
            qt = rest;
          } else {
            atomicOr(&ctl->flags, kFlagSpillOverflow);  // all lanes, same bit
          }
          wave_sync();
        }
        if (qt + C <= (unsigned)kQueueCap) {
          if (nc) {
            // all eight slots from the node's first child on are written,
            // the highest first: a slot past this node's children belongs to
            // a later lane, which writes it at a lower child index, hence
            // later; slots past the last child land in the slack above
            uint32_t *dst = queue + qt + pre;
#pragma unroll
            for (int q = 7; q >= 0; --q) {
              dst[q] = cf + (unsigned)q;
              __atomic_signal_fence(__ATOMIC_SEQ_CST);  // keeps the stores in this order
            }
          }
          qt += C;
        }
        wave_sync();
      }

      // (3) member particles of rejected leaves -> list
      const unsigned pc = open_leaf ? __float_as_uint(r1.z) : 0u;
      const unsigned pf = __float_as_uint(r1.y);
      const unsigned pinc = wave_incl_sum(pc);
      const unsigned P = wave_last(pinc);
      if (P) {
        tpre[lane] = pinc - pc;
        tsrc[lane] = pf;
        wave_sync();
        for (unsigned t0 = 0; t0 < P; t0 += 64) {
          if (np + 64 > D) {
            flush_shape<MULTI, LOGS, 1>(shape, a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            np = 0;
          }
          const unsigned t = t0 + lane;
          if (t < P) {
            int o = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
              if (tpre[o + step] <= t) o += step;
            const uint32_t src = tsrc[o] + (t - tpre[o]);
            pl[np + lane] = a.pos[src < a.n ? src : 0u];
          }
          np += (int)((P - t0) < 64u ? (P - t0) : 64u);
        }
        e_part += P;
        wave_sync();
      }
    }
    if (pops > (unsigned long long)nn) atomicOr(&ctl->flags, kFlagBadIndex);
    flush_shape<MULTI, LOGS>(shape, a, pl, ql, np, nq, pi, eps2, sub, S, acc);

    float ax = acc.x + acc.cx, ay = acc.y + acc.cy, az = acc.z + acc.cz, ap = acc.p + acc.cp;
    for (int m = Gx; m < 64; m <<= 1) {
      ax += __shfl_xor(ax, m, 64);
      ay += __shfl_xor(ay, m, 64);
      az += __shfl_xor(az, m, 64);
      ap += __shfl_xor(ap, m, 64);
    }
    const uint32_t dst = a.perm[ki];
    if (sub == 0 && vi && ki0 < a.n && dst < a.n)
      a.out[dst] = make_float4(ax, ay, az, -ap + pi.w * inv_eps);
    // same value from every lane
    a.gent[2 * (size_t)g] = (uint32_t)e_node;
    a.gent[2 * (size_t)g + 1] = (uint32_t)e_part;
    if (REC && lane == 0) {
      a.rec_n[2 * (size_t)rk] = (uint32_t)(rec_len - rec_leaves);
      a.rec_n[2 * (size_t)rk + 1] = (uint32_t)rec_leaves;
    }
    t_node += e_node;
    t_part += e_part;
    t_int += (unsigned long long)gc * (e_node + e_part);
    t_nint += (unsigned long long)gc * e_node;
    t_mac += n_mac;
  }
  if (!REC && lane == 0 && t_mac) {
    atomicAdd(&ctl->node_entries, t_node);
    atomicAdd(&ctl->part_entries, t_part);
    atomicAdd(&ctl->interactions, t_int);
    atomicAdd(&ctl->node_interactions, t_nint);
    atomicAdd(&ctl->mac_tests, t_mac);
  }
}

// ---------------------------------------------------------------------------
// Walk width W < 64.  The paper shares one traversal among the T_sub threads
// of a warp (Table 2); here a wave64 holds NSEG = 64 / W independent walks
// ("segments") of W lanes, each with its own group, pending stack (LDS ring of
// 8 W entries and a global spill region), interaction list and leaf-gather
// table, all carved from the wave's LDS.  A group has up to G i-particles with
// S = W / G lanes each.  Every count that steers a segment's loops is uniform
// over that segment's lanes, so segments diverge from each other but never
// inside themselves, and every ballot, prefix sum and broadcast below reads
// lanes of its own segment only.  A segment that finds no group left leaves
// the claim loop while the others go on.

// inclusive prefix sum inside each segment of W = 2^LOGW lanes (W >= 16):
// the row steps of wave_incl_sum, then row_bcast:15 for W = 32
template <int LOGW>
__device__ __forceinline__ unsigned seg_incl_sum(unsigned v) {
  v += dpp_or_zero<0x111, 0xf>(v);
  v += dpp_or_zero<0x112, 0xf>(v);
  v += dpp_or_zero<0x114, 0xf>(v);
  v += dpp_or_zero<0x118, 0xf>(v);
  if (LOGW >= 5) v += dpp_or_zero<0x142, 0xa>(v);
  if (LOGW >= 6) v += dpp_or_zero<0x143, 0xc>(v);
  return v;
}

template <int MULTI, int LOGS, int LOGW, bool REC>
__global__ void __launch_bounds__(256) walk_seg_k(WalkArgs a) {
  constexpr int W = 1 << LOGW;
  constexpr int NSEG = 64 >> LOGW;
  constexpr unsigned QC = 8u * W;  // the children of W rejected nodes always fit
  constexpr unsigned QM = QC - 1;
  constexpr unsigned CHUNK = QC / 2;
  extern __shared__ float4 smem[];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int seg = lane >> LOGW, sl = lane & (W - 1);
  const unsigned long long segm = (((1ull << (W - 1)) << 1) - 1ull) << (seg * W);
  char *sbase = reinterpret_cast<char *>(smem) + (size_t)w * a.wave_bytes +
                (size_t)seg * a.seg_bytes;
  float4 *pl = reinterpret_cast<float4 *>(sbase);
  float4 *ql = pl + a.D;
  uint32_t *queue = reinterpret_cast<uint32_t *>(ql + (MULTI == 2 ? 3 * a.DQ : 0));
  uint32_t *tpre = queue + QC;
  uint32_t *tsrc = tpre + W;

  const int64_t wslot = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
  const int64_t slot = wslot * NSEG + seg;
  uint32_t *spill = a.spill + slot * a.spill_cap;
  const int G = a.G;
  const int S = W >> a.logG;
  const int il = sl & (G - 1), sub = sl >> a.logG;
  Ctl *ctl = a.ctl;
  if (ctl->flags & kFlagNodeOverflow) return;  // no valid tree: the host repeats
  const unsigned ng = ctl->n_groups, nn = ctl->n_nodes, nsys = ctl->nsys;
  const unsigned nwork = REC ? a.ngsel : ng;
  const int D = a.D, DQ = a.DQ;
  if (wslot * NSEG >= (int64_t)nwork) return;  // the whole wave has nothing to claim

  unsigned long long t_node = 0, t_part = 0, t_int = 0, t_nint = 0, t_mac = 0;
  unsigned xr = blockIdx.x % kXcds;
  int tried = 0;
  int64_t rec_item = slot;
  const int64_t nslots = (int64_t)gridDim.x * (blockDim.x >> 6) * NSEG;
  for (;;) {
    unsigned g = ng;
    unsigned rk = 0;
    if (REC) {
      if (rec_item < (int64_t)nwork) {
        rk = (unsigned)rec_item;
        g = a.gsel[rk];
        if (g >= ng) g = ng;
        rec_item += nslots;
      }
      tried = kXcds;
    }
    while (tried < kXcds) {
      const unsigned lo = (unsigned)(((unsigned long long)xr * ng) / kXcds);
      const unsigned hi = (unsigned)(((unsigned long long)(xr + 1) * ng) / kXcds);
      unsigned cl = 0u;
      if (sl == 0) cl = atomicAdd(&ctl->xwork[kXworkStride * xr], 1u);
      cl = __shfl(cl, 0, W);
      if (lo + cl < hi) {
        g = lo + cl;
        break;
      }
      ++tried;
      xr = (xr + 1) % kXcds;
    }
    if (g >= ng) break;
    const unsigned gs = a.gfirst[g];
    const unsigned ge = a.gfirst[g + 1];
    const int gc0 = (int)(ge > gs ? ge - gs : 0u);
    const int gc = gc0 < G ? gc0 : G;
    const float4 bl = a.ball[g];
    const bool vi = il < gc;
    const uint32_t ki0 = a.alist[gs + (vi ? il : 0)];
    const uint32_t ki = ki0 < a.n ? ki0 : 0u;
    const float4 pi = a.pos[ki];
    const uint32_t k_first = a.alist[gs];
    const unsigned sy = sys_of(a.soff, nsys, k_first < a.n ? k_first : 0u);
    const float eps2 = a.sys[sy].eps2, theta = a.sys[sy].theta, inv_eps = a.sys[sy].inv_eps;
    const float dfac = a.mac == 1 ? a.mac_delta * a.gamin[g] : 0.f;
    Acc acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int np = 0, nq = 0;
    unsigned qb = 0, qt = 1;
    int64_t stop = 0;
    unsigned long long e_node = 0, e_part = 0, n_mac = 0;
    int64_t rec_len = 0, rec_leaves = 0;
    if (sl == 0) queue[0] = sy;
    wave_sync();

    unsigned long long pops = 0;
    while ((qt > qb || stop > 0) && pops <= (unsigned long long)nn) {
      if (qt == qb) {  // LDS part empty: bring back the newest spilled entries
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        const int64_t m = stop < (int64_t)CHUNK ? stop : (int64_t)CHUNK;
        for (int64_t t = sl; t < m; t += W) queue[(qb + t) & QM] = spill[stop - m + t];
        stop -= m;
        qt = qb + (unsigned)m;
        wave_sync();
      }
      const unsigned nb = (qt - qb) < (unsigned)W ? (qt - qb) : (unsigned)W;
      const bool has = (unsigned)sl < nb;
      const unsigned qv = queue[(qt - nb + sl) & QM];
      const unsigned node = (has && qv < nn) ? qv : 0u;
      qt -= nb;
      n_mac += nb;
      pops += nb;
      const float4 r0 = a.nrec[2 * (size_t)node];
      const float4 r1 = a.nrec[2 * (size_t)node + 1];
      float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
      if (MULTI == 2) {
        s0 = a.quad[2 * (size_t)node];
        s1 = a.quad[2 * (size_t)node + 1];
      }
      const float dx = r0.x - bl.x, dy = r0.y - bl.y, dz = r0.z - bl.z;
      const float rji = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
      const float dist = fmaxf(rji - bl.w, 0.f);
      bool mac_ok;
      if (a.mac == 0) {
        mac_ok = r1.x <= theta * dist;
      } else {
        const bool outside = !(r1.x > 0.f && r1.x >= dist);
        if (a.mac == 1) {
          const float d2 = dist * dist;
          mac_ok = outside && (r0.w * r1.x * r1.x <= dfac * (d2 * d2));
        } else {
          mac_ok = outside && (a.mcrit[node] <= dist);
        }
      }
      const bool accept = has && qv < nn && mac_ok;
      const bool leaf = __float_as_uint(r1.w) != 0u;
      const bool open_leaf = has && qv < nn && !accept && leaf;
      const bool open_int = has && qv < nn && !accept && !leaf;
      if (REC) {
        const unsigned long long rm = __ballot(accept || open_leaf) & segm;
        const int64_t at = rec_len + (int64_t)lanes_below(rm);
        if ((accept || open_leaf) && at < a.rec_cap)
          a.rec[(int64_t)rk * a.rec_cap + at] = node | (open_leaf ? kRecLeaf : 0u);
        rec_len += __popcll(rm);
        rec_leaves += __popcll(__ballot(open_leaf) & segm);
      }

      // (1) accepted pseudo j-particles
      const unsigned long long am = __ballot(accept) & segm;
      const int nacc = __popcll(am);
      if (nacc) {
        if (MULTI == 1) {
          if (np + nacc > D) {
            flush<MULTI, LOGS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            np = 0; nq = 0;
          }
          if (accept) pl[np + lanes_below(am)] = r0;
          np += nacc;
        } else {
          if (nq + nacc > DQ) {
            flush<MULTI, LOGS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            np = 0; nq = 0;
          }
          if (accept) {
            const int q = nq + (int)lanes_below(am);
            ql[3 * q] = r0;
            ql[3 * q + 1] = make_float4(3.f * s0.x, 3.f * s0.y, 3.f * s0.z, 3.f * s0.w);
            ql[3 * q + 2] = make_float4(3.f * s1.x, 3.f * s1.y, -0.5f * s1.z, -1.5f * s1.z);
          }
          nq += nacc;
        }
        e_node += (unsigned)nacc;
      }

      // (2) children of rejected internal nodes -> pending stack
      const unsigned nc = open_int ? __float_as_uint(r1.z) : 0u;
      const unsigned cf = __float_as_uint(r1.y);
      const unsigned cinc = seg_incl_sum<LOGW>(nc);
      const unsigned C = __shfl(cinc, W - 1, W);
      if (C) {
        const unsigned pre = cinc - nc;
        if ((qt - qb) + C > QC) {
          unsigned k = (qt - qb) + C - QC;
          k = (k + CHUNK - 1) / CHUNK * CHUNK;
          if (k > qt - qb) k = qt - qb;
          if (stop + k <= a.spill_cap) {
            for (unsigned t = sl; t < k; t += W) spill[stop + t] = queue[(qb + t) & QM];
            stop += k;
            qb += k;
          } else {
            atomicOr(&ctl->flags, kFlagSpillOverflow);
          }
          wave_sync();
        }
        if ((qt - qb) + C <= QC) {
          for (unsigned q = 0; q < nc; ++q) queue[(qt + pre + q) & QM] = cf + q;
          qt += C;
        }
        wave_sync();
      }

      // (3) member particles of rejected leaves -> list
      const unsigned pc = open_leaf ? __float_as_uint(r1.z) : 0u;
      const unsigned pf = __float_as_uint(r1.y);
      const unsigned pinc = seg_incl_sum<LOGW>(pc);
      const unsigned P = __shfl(pinc, W - 1, W);
      if (P) {
        tpre[sl] = pinc - pc;
        tsrc[sl] = pf;
        wave_sync();
        for (unsigned t0 = 0; t0 < P; t0 += W) {
          if (np + W > D) {
            flush<MULTI, LOGS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);
            np = 0; nq = 0;
          }
          const unsigned t = t0 + sl;
          if (t < P) {
            int o = 0;
#pragma unroll
            for (int step = W / 2; step >= 1; step >>= 1)
              if (tpre[o + step] <= t) o += step;
            const uint32_t src = tsrc[o] + (t - tpre[o]);
            pl[np + sl] = a.pos[src < a.n ? src : 0u];
          }
          np += (int)((P - t0) < (unsigned)W ? (P - t0) : (unsigned)W);
        }
        e_part += P;
        wave_sync();
      }
    }
    if (pops > (unsigned long long)nn) atomicOr(&ctl->flags, kFlagBadIndex);
    flush<MULTI, LOGS>(a, pl, ql, np, nq, pi, eps2, sub, S, acc);

    float ax = acc.x + acc.cx, ay = acc.y + acc.cy, az = acc.z + acc.cz, ap = acc.p + acc.cp;
    for (int m = G; m < W; m <<= 1) {
      ax += __shfl_xor(ax, m, W);
      ay += __shfl_xor(ay, m, W);
      az += __shfl_xor(az, m, W);
      ap += __shfl_xor(ap, m, W);
    }
    const uint32_t dst = a.perm[ki];
    if (sub == 0 && vi && ki0 < a.n && dst < a.n)
      a.out[dst] = make_float4(ax, ay, az, -ap + pi.w * inv_eps);
    a.gent[2 * (size_t)g] = (uint32_t)e_node;
    a.gent[2 * (size_t)g + 1] = (uint32_t)e_part;
    if (REC && sl == 0) {
      a.rec_n[2 * (size_t)rk] = (uint32_t)(rec_len - rec_leaves);
      a.rec_n[2 * (size_t)rk + 1] = (uint32_t)rec_leaves;
    }
    t_node += e_node;
    t_part += e_part;
    t_int += (unsigned long long)gc * (e_node + e_part);
    t_nint += (unsigned long long)gc * e_node;
    t_mac += n_mac;
  }
  if (!REC && sl == 0 && t_mac) {
    atomicAdd(&ctl->node_entries, t_node);
    atomicAdd(&ctl->part_entries, t_part);
    atomicAdd(&ctl->interactions, t_int);
    atomicAdd(&ctl->node_interactions, t_nint);
    atomicAdd(&ctl->mac_tests, t_mac);
  }
}

// LDS of one walk (a whole wave for W = 64, one segment otherwise): the
// particle list, the quadrupole node list, the pending stack (512 + 8 entries for
// W = 64, 8 W for a segment) and the leaf-gather table (W prefix sums and
// sources).
static int walk_bytes_for(int multi, int D, int DQ, int W) {
  const int ring = W == 64 ? kQueueCap + kQueueSlack : 8 * W;
  return D * 16 + (multi == 2 ? 3 * DQ * 16 : 0) + ring * 4 + 2 * W * 4;
}

// LDS list sizes (in float4 slots): list_depth is the budget of a wave, split
// evenly among its 64 / W walks.  Monopole entries take one slot; with
// quadrupole nodes half a walk's budget holds particle entries and half holds
// node entries of three slots each.  A walk's lists hold at least one batch
// (W entries), and for W = 64 at least 64 of each kind.  Small lists keep the
// LDS per wave near 8 KB so 16 waves fit on a CU and hide the walk's memory
// latency.
static void list_dims(int multi, int depth, int W, int *D, int *DQ) {
  const int per = depth / (64 / W);
  const int lo = W == 64 ? 64 : W;
  if (multi == 2) {
    *D = per / 2 < lo ? lo : per / 2;
    *DQ = per / 6 < lo ? lo : per / 6;
  } else {
    *D = per < lo ? lo : per;
    *DQ = 0;
  }
}

static int waves_per_block(int wb) {
  int w = 65536 / wb;
  return w >= 4 ? 4 : (w < 1 ? 1 : w);
}

static int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// The walk kernel for group size G and walk width W (S = W / G lanes per
// i-particle): compile-time S for the tuner's candidates, run-time S
// otherwise.
typedef void (*WalkFn)(WalkArgs);
template <int MULTI, int LOGW, bool REC>
static WalkFn walk_seg_fn(int S) {
  switch (S) {
    case 1: return walk_seg_k<MULTI, 0, LOGW, REC>;
    case 2: return walk_seg_k<MULTI, 1, LOGW, REC>;
    case 4: return walk_seg_k<MULTI, 2, LOGW, REC>;
    default: return walk_seg_k<MULTI, -1, LOGW, REC>;
  }
}

template <bool REC>
static WalkFn walk_fn(int multi, int G, int W) {
  const int S = W / G;
  if (W == 16) return multi == 2 ? walk_seg_fn<2, 4, REC>(S) : walk_seg_fn<1, 4, REC>(S);
  if (W == 32) return multi == 2 ? walk_seg_fn<2, 5, REC>(S) : walk_seg_fn<1, 5, REC>(S);
  if (multi == 2) {
    switch (S) {
      case 1: return walk_k<2, 0, REC>;
      case 2: return walk_k<2, 1, REC>;
      case 4: return walk_k<2, 2, REC>;
      case 8: return walk_k<2, 3, REC>;
      default: return walk_k<2, -1, REC>;
    }
  }
  switch (S) {
    case 1: return walk_k<1, 0, REC>;
    case 2: return walk_k<1, 1, REC>;
    case 4: return walk_k<1, 2, REC>;
    case 8: return walk_k<1, 3, REC>;
    default: return walk_k<1, -1, REC>;
  }
}

// resident walk waves of the kernel for each walk width W = 16 << lw and
// group size G = 2^lg <= W, kept per (multipole, list depth)
static void walk_occupancy(gothic_ctx *c) {
  const int multi = c->prm.multipole;
  const int depth = c->prm.list_depth;
  if (c->slots_multi == multi && c->slots_D == depth) return;
  for (int lw = 0; lw < kWalkWidths; ++lw) {
    const int W = 16 << lw;
    int D, DQ;
    list_dims(multi, depth, W, &D, &DQ);
    const int wb = (64 / W) * walk_bytes_for(multi, D, DQ, W);
    const int wpb = waves_per_block(wb);
    for (int lg = 0; lg < kGroupSizes; ++lg) {
      if ((1 << lg) > W) {
        c->slots_g[lw][lg] = 0;
        continue;
      }
      int per_cu = 0;
      const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, walk_fn<false>(multi, 1 << lg, W), wpb * 64, wpb * wb);
      if (e != hipSuccess || per_cu < 1) per_cu = 1;
      c->slots_g[lw][lg] = c->num_cus * per_cu * wpb;
    }
  }
  c->slots_multi = multi;
  c->slots_D = depth;
}

// the most persistent waves a walk of any shape launches (the spill stacks
// are sized for it)
int walk_slots(gothic_ctx *c) {
  walk_occupancy(c);
  int m = 0;
  for (int lw = 0; lw < kWalkWidths; ++lw)
    for (int lg = 0; lg < kGroupSizes; ++lg) m = c->slots_g[lw][lg] > m ? c->slots_g[lw][lg] : m;
  return m;
}

void launch_walk(gothic_ctx *c, int64_t n, float4 *acc_pot, hipStream_t s) {
  Buffers &B = c->b;
  WalkArgs a;
  const int multi = c->prm.multipole;
  const int W = c->cur_W;
  const int nseg = 64 / W;
  a.ctl = B.ctl;
  a.n = n;
  a.nrec = B.nrec;
  a.quad = B.quad;
  a.pos = B.pos;
  a.alist = B.alist;
  a.gfirst = B.gfirst;
  a.ball = B.ball;
  a.perm = B.idxA;
  a.out = acc_pot;
  a.gent = B.gent;
  a.spill = B.spill;
  a.spill_cap = c->spill_per_wave / nseg;  // a wave's region, split among its walks
  a.sys = B.sys;
  a.soff = B.soff;
  a.gamin = B.gamin;
  a.mcrit = B.mcrit;
  a.mac_delta = c->prm.mac_delta;
  a.mac = c->prm.mac;
  a.G = c->cur_G;
  const int lg = log2i(a.G);
  a.logG = lg;
  list_dims(multi, c->prm.list_depth, W, &a.D, &a.DQ);
  a.seg_bytes = walk_bytes_for(multi, a.D, a.DQ, W);
  a.wave_bytes = nseg * a.seg_bytes;
  a.compensated = c->prm.compensated;
  a.gsel = B.gsel;
  a.ngsel = B.ngsel;
  a.rec = B.rec;
  a.rec_n = B.rec_n;
  a.rec_cap = B.rec_cap;
  const bool rec = B.rec != nullptr;
  const int wpb = waves_per_block(a.wave_bytes);
  walk_occupancy(c);
  const int own = c->slots_g[log2i(W) - 4][lg];
  const int slots = own < c->walk_waves ? own : c->walk_waves;
  const int blocks = slots / wpb;
  hipLaunchKernelGGL(rec ? walk_fn<true>(multi, a.G, W) : walk_fn<false>(multi, a.G, W),
                     dim3(blocks), dim3(wpb * 64), wpb * a.wave_bytes, s, a);
}

}  // namespace gothic
