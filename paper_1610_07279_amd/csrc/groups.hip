// Active i-particles and their groups (Sections 2.3-2.4; block time steps,
// Section 2.7).  The active particles are compacted in key order.  Following
// Section 2.4, consecutive active particles farther apart than the critical
// separation r_crit (read from device memory, so a tuner can change it
// between replays of a captured step) start a new group (the squared gap is compared with
// r_crit^2 in float64 without fused operations, so the bounds are exact and
// reproducible); every run between such gaps is cut into groups of at most G.
// Each group gets its pseudo i-particle: the geometric centre r_I of the
// group's bounding box and the radius b_I of the sphere about r_I that holds
// every member (the GEO ball of Appendix B).  b_I is computed in FP32 and
// widened by a few ulp so the sphere provably holds the members.
#include "common.h"
#include "primitives.h"

namespace gothic {

__global__ void __launch_bounds__(256)
compact_k(int64_t n, int G, const uint32_t *__restrict__ flag, const uint32_t *__restrict__ ofs,
          uint32_t *__restrict__ alist, Ctl *ctl) {
  const unsigned na = ctl->scan_total;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->n_active = na;
  (void)G;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    if (flag[k]) {
      if (ofs[k] < na) alist[ofs[k]] = (uint32_t)k;
      else atomicOr(&ctl->flags, kFlagBadIndex);
    }
}

__device__ __forceinline__ double gap2(float4 p, float4 q) {
  const double dx = __dsub_rn((double)p.x, (double)q.x);
  const double dy = __dsub_rn((double)p.y, (double)q.y);
  const double dz = __dsub_rn((double)p.z, (double)q.z);
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// brk[a] = 1 where a new run starts (first active particle of a system, or a
// gap > r_crit; a negative r_crit is that fraction of the system's cube side)
__global__ void __launch_bounds__(256)
group_breaks_k(int64_t n, const float *__restrict__ rcrit, const Ctl *__restrict__ ctl,
               const uint32_t *__restrict__ soff, const SysRec *__restrict__ sys,
               const uint32_t *__restrict__ alist, const float4 *__restrict__ pos,
               uint32_t *__restrict__ brk) {
  const unsigned na = ctl->n_active, nsys = ctl->nsys;
  const float r_crit = *rcrit;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < na;
       a += (int64_t)gridDim.x * blockDim.x) {
    unsigned b = (a == 0);
    if (!b) {
      const uint32_t i = alist[a], j = alist[a - 1];
      if (i < n && j < n) {
        const unsigned si = sys_of(soff, nsys, i);
        if (si != sys_of(soff, nsys, j)) {
          b = 1u;
        } else {
          const double rc = r_crit < 0.f ? (double)(-r_crit) * sys[si].cube[3] : (double)r_crit;
          b = (rc > 0.0 && gap2(pos[i], pos[j]) > __dmul_rn(rc, rc)) ? 1u : 0u;
        }
      } else {
        b = 1u;
      }
    }
    brk[a] = b;
  }
}

// run starts: runpos[run id] = a
__global__ void __launch_bounds__(256)
group_runs_k(const Ctl *__restrict__ ctl, const uint32_t *__restrict__ brk,
             const uint32_t *__restrict__ runx, uint32_t *__restrict__ runpos) {
  const unsigned na = ctl->n_active;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < na;
       a += (int64_t)gridDim.x * blockDim.x)
    if (brk[a]) runpos[runx[a]] = (uint32_t)a;
}

// gflag[a] = 1 where a group starts: every G-th particle of its run
__global__ void __launch_bounds__(256)
group_starts_k(int G, Ctl *__restrict__ ctl, const uint32_t *__restrict__ brk,
               const uint32_t *__restrict__ runx, const uint32_t *__restrict__ runpos,
               uint32_t *__restrict__ gflag) {
  const unsigned na = ctl->n_active;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < na;
       a += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t run = runx[a] + brk[a] - 1u;  // inclusive count - 1
    const uint32_t rs = runpos[run];
    gflag[a] = (rs <= a && ((uint32_t)a - rs) % (uint32_t)G == 0u) ? 1u : 0u;
  }
}

__global__ void __launch_bounds__(256)
group_first_k(Ctl *__restrict__ ctl, const uint32_t *__restrict__ gflag,
              const uint32_t *__restrict__ gidx, uint32_t *__restrict__ gfirst) {
  const unsigned na = ctl->n_active, ng = ctl->scan_total;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->n_groups = ng;
    gfirst[ng] = na;
  }
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < na;
       a += (int64_t)gridDim.x * blockDim.x)
    if (gflag[a]) gfirst[gidx[a]] = (uint32_t)a;
}

// one wave per group; loop control is wave-uniform and the member load is
// predicated (lanes past the group's end re-read its first member)
__global__ void __launch_bounds__(256)
group_ball_k(int64_t n, const Ctl *__restrict__ ctl, const uint32_t *__restrict__ alist,
             const uint32_t *__restrict__ gfirst, const float4 *__restrict__ pos,
             float4 *__restrict__ ball, const float *__restrict__ amag,
             float *__restrict__ gamin) {
  const unsigned ng = ctl->n_groups, na = ctl->n_active;
  const int lane = lane_id();
  const int64_t wid = __builtin_amdgcn_readfirstlane(
      (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t g = wid; g < ng; g += nw) {
    const int64_t s = gfirst[g];
    const int64_t e = gfirst[g + 1];
    const int cnt = (int)(e - s < 64 ? (e > s ? e - s : 1) : 64);
    (void)na;
    const uint32_t ai = alist[s + (lane < cnt ? lane : 0)];
    const float4 p = pos[ai < n ? ai : 0];
    const float lx = wave_min(p.x), ly = wave_min(p.y), lz = wave_min(p.z);
    const float hx = wave_max(p.x), hy = wave_max(p.y), hz = wave_max(p.z);
    const float cx = 0.5f * (lx + hx), cy = 0.5f * (ly + hy), cz = 0.5f * (lz + hz);
    const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
    const float r = wave_max(sqrtf(dx * dx + dy * dy + dz * dz));
    ball[g] = make_float4(cx, cy, cz, r * (1.0f + 4.0f * 1.1920929e-7f));  // same from all lanes
    if (amag) {  // acceleration MAC: the group's smallest |a_old|
      const float am = wave_min(amag[ai < n ? ai : 0]);
      gamin[g] = am;
    }
  }
}

void launch_groups(gothic_ctx *c, int64_t n, hipStream_t s) {
  Buffers &B = c->b;
  const unsigned *na_dev = &B.ctl->n_active;
  scan_exclusive(B.flag, B.flag2, n, nullptr, nullptr, n, &B.ctl->scan_total, B.part, s);
  int64_t nb = (n + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(compact_k, dim3(g), dim3(256), 0, s, n, c->prm.group_size, B.flag, B.flag2,
                     B.alist, B.ctl);
  // runs between gaps > r_crit (flag: run breaks, flag2: run index, gA: run starts)
  hipLaunchKernelGGL(group_breaks_k, dim3(g), dim3(256), 0, s, n, B.rcrit, B.ctl, B.soff,
                     B.sys, B.alist, B.pos, B.flag);
  scan_exclusive(B.flag, B.flag2, 0, na_dev, nullptr, n, &B.ctl->scan_total, B.part, s);
  hipLaunchKernelGGL(group_runs_k, dim3(g), dim3(256), 0, s, B.ctl, B.flag, B.flag2, B.gA);
  // groups: every G-th particle of a run starts one (gB: starts, flag: group index)
  hipLaunchKernelGGL(group_starts_k, dim3(g), dim3(256), 0, s, c->prm.group_size, B.ctl, B.flag,
                     B.flag2, B.gA, B.gB);
  scan_exclusive(B.gB, B.flag, 0, na_dev, nullptr, n, &B.ctl->scan_total, B.part, s);
  hipLaunchKernelGGL(group_first_k, dim3(g), dim3(256), 0, s, B.ctl, B.gB, B.flag, B.gfirst);
  int64_t wb = (n + 3) / 4;
  int gb = (int)(wb > 8192 ? 8192 : (wb < 1 ? 1 : wb));
  const bool acc_mac = c->prm.mac == 1;
  hipLaunchKernelGGL(group_ball_k, dim3(gb), dim3(256), 0, s, n, B.ctl, B.alist, B.gfirst, B.pos,
                     B.ball, acc_mac ? B.amag : nullptr, B.gamin);
}

}  // namespace gothic
