// Active i-particles and their groups (Section 2.3; block time steps,
// Section 2.7).  The active particles are compacted in key order, cut into
// groups of G consecutive ones, and each group gets its pseudo i-particle:
// the geometric centre r_I of the group's bounding box and the radius b_I of
// the sphere about r_I that holds every member (the GEO ball of Appendix B).
// b_I is computed in FP32 and widened by a few ulp so the sphere provably
// holds the members despite rounding.
#include "common.h"
#include "primitives.h"

namespace gothic {

__global__ void __launch_bounds__(256)
compact_k(int64_t n, int G, const uint32_t *__restrict__ flag, const uint32_t *__restrict__ ofs,
          uint32_t *__restrict__ alist, Ctl *ctl) {
  const unsigned na = ctl->scan_total;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->n_active = na;
    ctl->n_groups = (na + (unsigned)G - 1) / (unsigned)G;
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    if (flag[k]) {
      if (ofs[k] < na) alist[ofs[k]] = (uint32_t)k;
      else atomicOr(&ctl->flags, kFlagBadIndex);
    }
}

// one wave per group; loop control is wave-uniform and the member load is
// predicated (lanes past the group's end re-read its first member)
__global__ void __launch_bounds__(256)
group_ball_k(int G, int64_t n, const Ctl *__restrict__ ctl, const uint32_t *__restrict__ alist,
             const float4 *__restrict__ pos, float4 *__restrict__ ball) {
  const unsigned ng = ctl->n_groups, na = ctl->n_active;
  const int lane = lane_id();
  const int64_t wid = __builtin_amdgcn_readfirstlane(
      (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t g = wid; g < ng; g += nw) {
    const int64_t s = g * G;
    const int cnt = (int)((int64_t)na - s < G ? (int64_t)na - s : G);
    const uint32_t ai = alist[s + (lane < cnt ? lane : 0)];
    const float4 p = pos[ai < n ? ai : 0];
    const float lx = wave_min(p.x), ly = wave_min(p.y), lz = wave_min(p.z);
    const float hx = wave_max(p.x), hy = wave_max(p.y), hz = wave_max(p.z);
    const float cx = 0.5f * (lx + hx), cy = 0.5f * (ly + hy), cz = 0.5f * (lz + hz);
    const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
    const float r = wave_max(sqrtf(dx * dx + dy * dy + dz * dz));
    ball[g] = make_float4(cx, cy, cz, r * (1.0f + 4.0f * 1.1920929e-7f));  // same from all lanes
  }
}

void launch_groups(gothic_ctx *c, int64_t n, hipStream_t s) {
  Buffers &B = c->b;
  scan_exclusive(B.flag, B.flag2, n, nullptr, nullptr, n, &B.ctl->scan_total, B.part, s);
  int64_t nb = (n + 255) / 256;
  int g = (int)(nb > 8192 ? 8192 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(compact_k, dim3(g), dim3(256), 0, s, n, c->prm.group_size, B.flag, B.flag2,
                     B.alist, B.ctl);
  int64_t gmax = (n + c->prm.group_size - 1) / c->prm.group_size;
  int64_t wb = (gmax + 3) / 4;
  int gb = (int)(wb > 8192 ? 8192 : (wb < 1 ? 1 : wb));
  hipLaunchKernelGGL(group_ball_k, dim3(gb), dim3(256), 0, s, c->prm.group_size, n, B.ctl, B.alist,
                     B.pos, B.ball);
}

}  // namespace gothic
