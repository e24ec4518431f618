// Active i-particles and their groups (Sections 2.3-2.4; block time steps,
// Section 2.7).  The active particles are compacted in key order.  Following
// Section 2.4, consecutive active particles farther apart than the critical
// separation r_crit (read from device memory, so a tuner can change it
// between replays of a captured step) start a new group (the squared gap is compared with
// r_crit^2 in float64 without fused operations, so the bounds are exact and
// reproducible); every run between such gaps is cut into groups of at most G.
// Each group gets its pseudo i-particle (r_I, b_I): an enclosing ball of the
// kind params.ball selects (Appendix B; the geometric centre of the bounding
// box by default), see group_ball_k.
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

// ---------------------------------------------------------------- balls
// Enclosing balls of a group (pseudo i-particles, Appendix B): a centre of
// the chosen kind, and the largest member distance from it as the radius
// (float32, widened by 4 ulp so the sphere provably holds the members).
//   GEO bounding-box centre; SEB smallest enclosing ball; EBS Ritter's
//   sphere; COM centre of mass; CMP the smaller of GEO and COM.
// One wave per group, member q in lane q (G <= 64).  SEB and EBS centres are
// computed in float64 with wave-uniform control: ballots find the next
// member outside the current ball.
struct DBall {
  double x, y, z, r2;
};

__device__ __forceinline__ double d2of(double ax, double ay, double az, double bx, double by,
                                       double bz) {
  const double x = ax - bx, y = ay - by, z = az - bz;
  return x * x + y * y + z * z;
}

__device__ __forceinline__ bool in_ball(const DBall &B, double x, double y, double z) {
  return d2of(x, y, z, B.x, B.y, B.z) <= B.r2 * (1.0 + 1e-12);
}

__device__ DBall dball2(double ax, double ay, double az, double bx, double by, double bz) {
  return DBall{0.5 * (ax + bx), 0.5 * (ay + by), 0.5 * (az + bz), 0.25 * d2of(ax, ay, az, bx, by, bz)};
}

// smallest ball with the three points on its boundary (their circumcircle);
// nearly collinear points: the ball of the farthest pair
__device__ DBall dball3(const double *a, const double *b, const double *c) {
  const double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
  const double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
  const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
  const double uu = ux * ux + uy * uy + uz * uz, vv = vx * vx + vy * vy + vz * vz;
  const double ww = wx * wx + wy * wy + wz * wz;
  if (ww <= 1e-24 * uu * vv) {
    const double dab = uu, dac = vv, dbc = d2of(b[0], b[1], b[2], c[0], c[1], c[2]);
    if (dab >= dac && dab >= dbc) return dball2(a[0], a[1], a[2], b[0], b[1], b[2]);
    if (dac >= dbc) return dball2(a[0], a[1], a[2], c[0], c[1], c[2]);
    return dball2(b[0], b[1], b[2], c[0], c[1], c[2]);
  }
  const double tx = uu * vx - vv * ux, ty = uu * vy - vv * uy, tz = uu * vz - vv * uz;
  const double h = 0.5 / ww;
  DBall B;
  B.x = a[0] + (ty * wz - tz * wy) * h;
  B.y = a[1] + (tz * wx - tx * wz) * h;
  B.z = a[2] + (tx * wy - ty * wx) * h;
  B.r2 = d2of(a[0], a[1], a[2], B.x, B.y, B.z);
  return B;
}

// the sphere through four points; nearly coplanar: the smallest ball of
// two or three of them that holds all four
__device__ DBall dball4(const double *a, const double *b, const double *c, const double *d) {
  const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double t[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
  const double c0 = v[1] * t[2] - v[2] * t[1], c1 = v[0] * t[2] - v[2] * t[0],
               c2 = v[0] * t[1] - v[1] * t[0];
  const double det = u[0] * c0 - u[1] * c1 + u[2] * c2;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  if (fabs(det) <= 1e-12 * sqrt(uu * vv * tt)) {
    const double *P[4] = {a, b, c, d};
    DBall best{0, 0, 0, -1.0};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        for (int k = j; k < 4; ++k) {  // k == j: the pair ball
          const DBall cand = (k == j) ? dball2(P[i][0], P[i][1], P[i][2], P[j][0], P[j][1], P[j][2])
                                      : dball3(P[i], P[j], P[k]);
          bool ok = true;
          for (int m = 0; m < 4; ++m) ok = ok && in_ball(cand, P[m][0], P[m][1], P[m][2]);
          if (ok && (best.r2 < 0 || cand.r2 < best.r2)) best = cand;
        }
    return best;
  }
  const double r0 = 0.5 * uu, r1 = 0.5 * vv, r2 = 0.5 * tt;
  const double x0 = (r0 * c0 - u[1] * (r1 * t[2] - v[2] * r2) + u[2] * (r1 * t[1] - v[1] * r2)) / det;
  const double x1 = (u[0] * (r1 * t[2] - v[2] * r2) - r0 * c1 + u[2] * (v[0] * r2 - r1 * t[0])) / det;
  const double x2 = (u[0] * (v[1] * r2 - r1 * t[1]) - u[1] * (v[0] * r2 - r1 * t[0]) + r0 * c2) / det;
  return DBall{a[0] + x0, a[1] + x1, a[2] + x2, x0 * x0 + x1 * x1 + x2 * x2};
}

__device__ __forceinline__ int first_lane(unsigned long long m) {
  return __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1);
}

// smallest enclosing ball: the incremental algorithm with up to four
// boundary points; every loop index only grows, so it ends
__device__ DBall seb_wave(double px, double py, double pz, int cnt) {
  const int lane = lane_id();
  const double P0[3] = {__shfl(px, 0, 64), __shfl(py, 0, 64), __shfl(pz, 0, 64)};
  DBall B{P0[0], P0[1], P0[2], 0.0};
  int i = 0;
  for (;;) {
    const unsigned long long mi = __ballot(lane > i && lane < cnt && !in_ball(B, px, py, pz));
    if (!mi) break;
    i = first_lane(mi);
    const double Pi[3] = {__shfl(px, i, 64), __shfl(py, i, 64), __shfl(pz, i, 64)};
    B = DBall{Pi[0], Pi[1], Pi[2], 0.0};
    int j = -1;
    for (;;) {
      const unsigned long long mj = __ballot(lane > j && lane < i && !in_ball(B, px, py, pz));
      if (!mj) break;
      j = first_lane(mj);
      const double Pj[3] = {__shfl(px, j, 64), __shfl(py, j, 64), __shfl(pz, j, 64)};
      B = dball2(Pi[0], Pi[1], Pi[2], Pj[0], Pj[1], Pj[2]);
      int k = -1;
      for (;;) {
        const unsigned long long mk = __ballot(lane > k && lane < j && !in_ball(B, px, py, pz));
        if (!mk) break;
        k = first_lane(mk);
        const double Pk[3] = {__shfl(px, k, 64), __shfl(py, k, 64), __shfl(pz, k, 64)};
        B = dball3(Pi, Pj, Pk);
        int l = -1;
        for (;;) {
          const unsigned long long ml = __ballot(lane > l && lane < k && !in_ball(B, px, py, pz));
          if (!ml) break;
          l = first_lane(ml);
          const double Pl[3] = {__shfl(px, l, 64), __shfl(py, l, 64), __shfl(pz, l, 64)};
          B = dball4(Pi, Pj, Pk, Pl);
        }
      }
    }
  }
  return B;
}

// smallest / largest float over the wave (all lanes active): an inclusive
// DPP scan whose missing sources read the identity (+inf / -inf), then the
// last lane is read back
template <bool MAX>
__device__ __forceinline__ float wave_extreme(float x) {
  constexpr int ident = MAX ? (int)0xff800000 : (int)0x7f800000;
  float v = x;
#define GOTHIC_EXT_STEP(ctrl, rows)                                                    \
  {                                                                                    \
    const float o = __int_as_float(                                                    \
        __builtin_amdgcn_update_dpp(ident, __float_as_int(v), ctrl, rows, 0xf, false)); \
    v = MAX ? fmaxf(v, o) : fminf(v, o);                                               \
  }
  GOTHIC_EXT_STEP(0x111, 0xf)
  GOTHIC_EXT_STEP(0x112, 0xf)
  GOTHIC_EXT_STEP(0x114, 0xf)
  GOTHIC_EXT_STEP(0x118, 0xf)
  GOTHIC_EXT_STEP(0x142, 0xa)
  GOTHIC_EXT_STEP(0x143, 0xc)
#undef GOTHIC_EXT_STEP
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// uniform-lane broadcast of a double (two readlanes, no LDS)
__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// a 64-bit value moved by DPP (both halves); lanes without a source read 0
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp64(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROWS, 0xf, false);
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// largest value over the wave for values that are >= 0 or exactly -1 (their
// bit patterns, read as signed 64-bit integers, order like the values): an
// inclusive max scan by DPP whose last lane is read back
__device__ __forceinline__ double wave_max_nonneg(double x) {
  long long v = __double_as_longlong(x);
#define GOTHIC_MAX_STEP(ctrl, rows)            \
  {                                            \
    const long long o = dpp64<ctrl, rows>(v);  \
    v = o > v ? o : v;                         \
  }
  GOTHIC_MAX_STEP(0x111, 0xf)
  GOTHIC_MAX_STEP(0x112, 0xf)
  GOTHIC_MAX_STEP(0x114, 0xf)
  GOTHIC_MAX_STEP(0x118, 0xf)
  GOTHIC_MAX_STEP(0x142, 0xa)
  GOTHIC_MAX_STEP(0x143, 0xc)
#undef GOTHIC_MAX_STEP
  return lane_d(__longlong_as_double(v), 63);
}

// Ritter's sphere: the diameter of two far members, grown in member order
__device__ void ebs_wave(double px, double py, double pz, int cnt, double &cx, double &cy,
                         double &cz) {
  const int lane = lane_id();
  const bool v = lane < cnt;
  const double x0 = lane_d(px, 0), y0 = lane_d(py, 0), z0 = lane_d(pz, 0);
  // farthest member from member 0 (first one on ties), then farthest from it
  double d = v ? d2of(px, py, pz, x0, y0, z0) : -1.0;
  double dm = wave_max_nonneg(d);
  const int y = first_lane(__ballot(v && d == dm));
  const double yx = lane_d(px, y), yy = lane_d(py, y), yz = lane_d(pz, y);
  d = v ? d2of(px, py, pz, yx, yy, yz) : -1.0;
  dm = wave_max_nonneg(d);
  const int z = first_lane(__ballot(v && d == dm));
  const double zx = lane_d(px, z), zy = lane_d(py, z), zz = lane_d(pz, z);
  cx = 0.5 * (yx + zx);
  cy = 0.5 * (yy + zy);
  cz = 0.5 * (yz + zz);
  double r = 0.5 * sqrt(d2of(yx, yy, yz, zx, zy, zz));
  // members are visited in order; the ball only grows, so a member inside it
  // stays inside and the next member outside is the next one to take in
  int q = -1;
  for (;;) {
    const double dq = sqrt(d2of(px, py, pz, cx, cy, cz));
    const unsigned long long m = __ballot(v && lane > q && dq > r);
    if (!m) break;
    q = first_lane(m);
    const double dd = lane_d(dq, q);
    const double qx = lane_d(px, q), qy = lane_d(py, q), qz = lane_d(pz, q);
    const double rn = 0.5 * (r + dd);
    const double f = (rn - r) / dd;
    cx += (qx - cx) * f;
    cy += (qy - cy) * f;
    cz += (qz - cz) * f;
    r = rn;
  }
}

__device__ __forceinline__ float ball_radius(float4 p, float cx, float cy, float cz) {
  const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
  return wave_extreme<true>(sqrtf(dx * dx + dy * dy + dz * dz));
}

// one wave per group; loop control is wave-uniform and the member load is
// predicated (lanes past the group's end re-read its first member)
// (one instantiation per ball kind, so that a kernel trace times each kind)
template <int kind>
__global__ void __launch_bounds__(256)
group_ball_k(int64_t n, const Ctl *__restrict__ ctl, const uint32_t *__restrict__ alist,
             const uint32_t *__restrict__ gfirst, const float4 *__restrict__ pos,
             float4 *__restrict__ ball, const float *__restrict__ amag,
             float *__restrict__ gamin) {
  const unsigned ng = ctl->n_groups;
  const int lane = lane_id();
  const int64_t wid = __builtin_amdgcn_readfirstlane(
      (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  constexpr float kWiden = 1.0f + 4.0f * 1.1920929e-7f;
  for (int64_t g = wid; g < ng; g += nw) {
    const int64_t s = gfirst[g];
    const int64_t e = gfirst[g + 1];
    const int cnt = (int)(e - s < 64 ? (e > s ? e - s : 1) : 64);
    // SEB visits the members in a fixed pseudo-random order (lane q holds
    // member (97 q + 13) mod cnt), which keeps its expected work linear
    const int mem = (kind == 1) ? (int)((97u * (unsigned)lane + 13u) % (unsigned)cnt)
                                : (lane < cnt ? lane : 0);
    const uint32_t ai = alist[s + (lane < cnt ? mem : 0)];
    const float4 p = pos[ai < n ? ai : 0];
    float cx, cy, cz;
    // GEO (also the fallback half of CMP)
    const float lx = wave_extreme<false>(p.x), ly = wave_extreme<false>(p.y),
                lz = wave_extreme<false>(p.z);
    const float hx = wave_extreme<true>(p.x), hy = wave_extreme<true>(p.y),
                hz = wave_extreme<true>(p.z);
    cx = 0.5f * (lx + hx);
    cy = 0.5f * (ly + hy);
    cz = 0.5f * (lz + hz);
    if (kind == 1 || kind == 2) {
      double dx, dy, dz;
      if (kind == 1) {
        const DBall B = seb_wave((double)p.x, (double)p.y, (double)p.z, cnt);
        dx = B.x; dy = B.y; dz = B.z;
      } else {
        ebs_wave((double)p.x, (double)p.y, (double)p.z, cnt, dx, dy, dz);
      }
      cx = (float)dx; cy = (float)dy; cz = (float)dz;
    } else if (kind == 3 || kind == 4) {
      const double m = lane < cnt ? (double)p.w : 0.0;
      double M = m, sx = m * p.x, sy = m * p.y, sz = m * p.z;
      for (int o = 32; o >= 1; o >>= 1) {
        M += __shfl_xor(M, o, 64);
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sz += __shfl_xor(sz, o, 64);
      }
      if (M > 0.0) {
        const float mx = (float)(sx / M), my = (float)(sy / M), mz = (float)(sz / M);
        if (kind == 3) {
          cx = mx; cy = my; cz = mz;
        } else {  // CMP: COM only if clearly smaller than GEO
          const float rg = ball_radius(p, cx, cy, cz), rm = ball_radius(p, mx, my, mz);
          if (rm < rg * (1.0f - 1e-5f)) {
            cx = mx; cy = my; cz = mz;
          }
        }
      }
    }
    const float r = ball_radius(p, cx, cy, cz);
    ball[g] = make_float4(cx, cy, cz, r * kWiden);  // same from all lanes
    if (amag) {  // acceleration MAC: the group's smallest |a_old|
      const float am = wave_extreme<false>(amag[ai < n ? ai : 0]);
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
  hipLaunchKernelGGL(compact_k, dim3(g), dim3(256), 0, s, n, c->cur_G, B.flag, B.flag2,
                     B.alist, B.ctl);
  // runs between gaps > r_crit (flag: run breaks, flag2: run index, gA: run starts)
  hipLaunchKernelGGL(group_breaks_k, dim3(g), dim3(256), 0, s, n, B.rcrit, B.ctl, B.soff,
                     B.sys, B.alist, B.pos, B.flag);
  scan_exclusive(B.flag, B.flag2, 0, na_dev, nullptr, n, &B.ctl->scan_total, B.part, s);
  hipLaunchKernelGGL(group_runs_k, dim3(g), dim3(256), 0, s, B.ctl, B.flag, B.flag2, B.gA);
  // groups: every G-th particle of a run starts one (gB: starts, flag: group index)
  hipLaunchKernelGGL(group_starts_k, dim3(g), dim3(256), 0, s, c->cur_G, B.ctl, B.flag,
                     B.flag2, B.gA, B.gB);
  scan_exclusive(B.gB, B.flag, 0, na_dev, nullptr, n, &B.ctl->scan_total, B.part, s);
  hipLaunchKernelGGL(group_first_k, dim3(g), dim3(256), 0, s, B.ctl, B.gB, B.flag, B.gfirst);
  int64_t wb = (n + 3) / 4;
  int gb = (int)(wb > 8192 ? 8192 : (wb < 1 ? 1 : wb));
  const bool acc_mac = c->prm.mac == 1;
  decltype(&group_ball_k<0>) ball_fn;
  switch (c->prm.ball) {
    case 1: ball_fn = group_ball_k<1>; break;
    case 2: ball_fn = group_ball_k<2>; break;
    case 3: ball_fn = group_ball_k<3>; break;
    case 4: ball_fn = group_ball_k<4>; break;
    default: ball_fn = group_ball_k<0>; break;
  }
  hipLaunchKernelGGL(ball_fn, dim3(gb), dim3(256), 0, s, n, B.ctl, B.alist, B.gfirst, B.pos,
                     B.ball, acc_mac ? B.amag : nullptr, B.gamin);
}

}  // namespace gothic
