// Bounding cube, quantisation and space-filling-curve keys (Section 2.1 and
// Appendix A of the paper).
//
// Quantisation (the paper leaves it open): cube origin = bounding-box minimum,
// side L = smallest power of two >= the largest extent (1 when all positions
// coincide), q = min(floor((x - x_min) * 2^21 / L), 2^21 - 1) per axis in
// float64.  The subtraction is one IEEE rounding and the scaling by a power of
// two is exact, so the integer codes are reproducible on any IEEE machine.
//
// Morton key: the three 21-bit codes interleaved, x in bit 3b+2, y in 3b+1,
// z in 3b.  Peano-Hilbert key: level by level from the coarsest, the octant
// of the point in the current frame gives the 3-bit digit (inverse Gray code)
// and selects how the frame is inverted and rotated for the finer levels.
// Here the frame is a state of a 48-state automaton (6 axis permutations x 8
// inversion masks) whose transition table is generated at compile time.
#include <float.h>

#include "common.h"
#include "primitives.h"

namespace gothic {

constexpr int kBboxBlocks = 1024;
constexpr int kBboxThreads = 256;

// ---------------------------------------------------------------- PH table
struct PhTable {
  unsigned short e[48 * 8];  // digit | next_state << 3, index state*8 + original octant
};

// frame axis a reads original axis kPerm[p][a]
constexpr int kPerm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}, {0, 2, 1}, {1, 0, 2}};

constexpr int perm_index(int a0, int a1, int a2) {
  for (int p = 0; p < 6; ++p)
    if (kPerm[p][0] == a0 && kPerm[p][1] == a1 && kPerm[p][2] == a2) return p;
  return -1;
}

// Per frame octant o (bits: axis0 axis1 axis2): axes inverted before the
// rotation (mask, axis0 = 4) and the rotation (0 keep, 1 cycle new(0,1,2) =
// old(1,2,0), 2 exchange axes 0 and 2).  These encode the curve of Appendix A.
constexpr unsigned kInvByOct = 0x63650300u;  // nibble o: mask   (o=7..0: 6 3 6 5 0 3 0 0)
constexpr unsigned kRotByOct = 0x10121012u;  // nibble o: rotation (o=7..0: 1 0 1 2 1 0 1 2)

constexpr PhTable make_ph_table() {
  PhTable t{};
  for (int p = 0; p < 6; ++p)
    for (int f = 0; f < 8; ++f)
      for (int ob = 0; ob < 8; ++ob) {
        int fb[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) fb[a] = ((ob >> (2 - kPerm[p][a])) & 1) ^ ((f >> (2 - a)) & 1);
        const int fo = (fb[0] << 2) | (fb[1] << 1) | fb[2];
        const int digit = fo ^ (fo >> 1) ^ (fo >> 2);  // inverse Gray code, 3 bits
        const int inv = (int)((kInvByOct >> (4 * fo)) & 15u);
        const int rot = (int)((kRotByOct >> (4 * fo)) & 15u);
        int nf[3] = {((f >> 2) ^ (inv >> 2)) & 1, ((f >> 1) ^ (inv >> 1)) & 1, (f ^ inv) & 1};
        int src[3] = {kPerm[p][0], kPerm[p][1], kPerm[p][2]};
        int order[3] = {0, 1, 2};
        if (rot == 1) { order[0] = 1; order[1] = 2; order[2] = 0; }
        if (rot == 2) { order[0] = 2; order[1] = 1; order[2] = 0; }
        const int np = perm_index(src[order[0]], src[order[1]], src[order[2]]);
        const int nfm = (nf[order[0]] << 2) | (nf[order[1]] << 1) | nf[order[2]];
        t.e[(p * 8 + f) * 8 + ob] = (unsigned short)(digit | ((np * 8 + nfm) << 3));
      }
  return t;
}

__constant__ PhTable kPh = make_ph_table();

// ---------------------------------------------------------------- Morton
// spread the low 21 bits of v to every third bit
__host__ __device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// ---------------------------------------------------------------- bbox
// Grid (partials per system, systems): workgroup (b, s) reduces every
// gridDim.x-th tile of system s.
__device__ __forceinline__ bool finite4(float4 p) {
  return isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w);
}

__global__ void __launch_bounds__(kBboxThreads)
bbox_partial_k(const float4 *__restrict__ xyzm, const uint32_t *__restrict__ soff,
               float *__restrict__ part, Ctl *ctl) {
  const int64_t i0 = soff[blockIdx.y], i1 = soff[blockIdx.y + 1];
  float lo0 = FLT_MAX, lo1 = FLT_MAX, lo2 = FLT_MAX;
  float hi0 = -FLT_MAX, hi1 = -FLT_MAX, hi2 = -FLT_MAX;
  bool bad = false;
  for (int64_t i = i0 + (int64_t)blockIdx.x * kBboxThreads + threadIdx.x; i < i1;
       i += (int64_t)gridDim.x * kBboxThreads) {
    const float4 p = xyzm[i];
    bad |= !finite4(p);
    lo0 = fminf(lo0, p.x); lo1 = fminf(lo1, p.y); lo2 = fminf(lo2, p.z);
    hi0 = fmaxf(hi0, p.x); hi1 = fmaxf(hi1, p.y); hi2 = fmaxf(hi2, p.z);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(&ctl->flags, kFlagNonFinite);
  lo0 = wave_min(lo0); lo1 = wave_min(lo1); lo2 = wave_min(lo2);
  hi0 = wave_max(hi0); hi1 = wave_max(hi1); hi2 = wave_max(hi2);
  __shared__ float sh[kBboxThreads / 64][6];
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sh[w][0] = lo0; sh[w][1] = lo1; sh[w][2] = lo2;
    sh[w][3] = hi0; sh[w][4] = hi1; sh[w][5] = hi2;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    float v = sh[0][threadIdx.x];
    for (int k = 1; k < kBboxThreads / 64; ++k)
      v = threadIdx.x < 3 ? fminf(v, sh[k][threadIdx.x]) : fmaxf(v, sh[k][threadIdx.x]);
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = v;
  }
}

// one wave per system
__global__ void __launch_bounds__(64) bbox_final_k(const float *__restrict__ part, int nblk,
                                                   SysRec *__restrict__ sys) {
  const float *ps = part + (int64_t)blockIdx.x * nblk * 6;
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int b = lane_id(); b < nblk; b += 64)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], ps[b * 6 + a]);
      hi[a] = fmaxf(hi[a], ps[b * 6 + 3 + a]);
    }
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min(lo[a]);
    hi[a] = wave_max(hi[a]);
  }
  if (lane_id() == 0) {
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double e = __dsub_rn((double)hi[a], (double)lo[a]);
      if (e > ext) ext = e;
    }
    double L = 1.0;
    if (ext > 0.0) {
      int ex = 0;
      const double f = frexp(ext, &ex);
      L = (f == 0.5) ? ext : ldexp(1.0, ex);
    }
    SysRec &r = sys[blockIdx.x];
    for (int a = 0; a < 3; ++a) r.cube[a] = (double)lo[a];
    r.cube[3] = L;
  }
}

// ---------------------------------------------------------------- keys
// Grid (workgroups per system, systems).
__global__ void __launch_bounds__(256)
keys_k(const float4 *__restrict__ xyzm, const uint32_t *__restrict__ soff, int key_kind,
       const SysRec *__restrict__ sys, uint64_t *__restrict__ keys, uint32_t *__restrict__ idx) {
  __shared__ unsigned short tab[48 * 8];
  if (key_kind == GOTHIC_KEY_PEANO_HILBERT) {
    for (int t = threadIdx.x; t < 48 * 8; t += blockDim.x) tab[t] = kPh.e[t];
    __syncthreads();
  }
  const int64_t i0 = soff[blockIdx.y], i1 = soff[blockIdx.y + 1];
  const SysRec &r = sys[blockIdx.y];
  const double x0 = r.cube[0], y0 = r.cube[1], z0 = r.cube[2];
  const double scale = ldexp(1.0, kNlev) / r.cube[3];
  const uint64_t qmax = (1ull << kNlev) - 1;
  for (int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < i1;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 p = xyzm[i];
    const double tx = floor(__dmul_rn(__dsub_rn((double)p.x, x0), scale));
    const double ty = floor(__dmul_rn(__dsub_rn((double)p.y, y0), scale));
    const double tz = floor(__dmul_rn(__dsub_rn((double)p.z, z0), scale));
    uint64_t qx = (uint64_t)tx, qy = (uint64_t)ty, qz = (uint64_t)tz;
    qx = qx > qmax ? qmax : qx;
    qy = qy > qmax ? qmax : qy;
    qz = qz > qmax ? qmax : qz;
    uint64_t key;
    if (key_kind == GOTHIC_KEY_PEANO_HILBERT) {
      key = 0;
      unsigned st = 0;  // identity frame
      for (int lev = kNlev - 1; lev >= 0; --lev) {
        const unsigned ob = (unsigned)((((qx >> lev) & 1u) << 2) | (((qy >> lev) & 1u) << 1) |
                                       ((qz >> lev) & 1u));
        const unsigned e = tab[st * 8 + ob];
        key = (key << 3) | (e & 7u);
        st = e >> 3;
      }
    } else {
      key = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    }
    keys[i] = key;
    idx[i] = (uint32_t)i;
  }
}

// partial bounding boxes per system: enough workgroups to cover the largest
// system, about kBboxBlocks in all
int bbox_partials(int nsys, int64_t max_n) {
  int64_t b = (max_n + kBboxThreads - 1) / kBboxThreads;
  int64_t cap = kBboxBlocks / (nsys > 0 ? nsys : 1);
  if (cap < 1) cap = 1;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

void launch_bbox_keys(gothic_ctx *c, const float4 *xyzm, int64_t n, int nsys, int64_t max_n,
                      hipStream_t s) {
  (void)n;
  const int nb = bbox_partials(nsys, max_n);
  hipLaunchKernelGGL(bbox_partial_k, dim3(nb, nsys), dim3(kBboxThreads), 0, s, xyzm, c->b.soff,
                     c->b.bbox_part, c->b.ctl);
  hipLaunchKernelGGL(bbox_final_k, dim3(nsys), dim3(64), 0, s, c->b.bbox_part, nb, c->b.sys);
  int64_t kb = (max_n + 255) / 256;
  int64_t kcap = 8192 / nsys;
  if (kcap < 1) kcap = 1;
  const int kx = (int)(kb > kcap ? kcap : (kb < 1 ? 1 : kb));
  const bool toB = keys_to_B(nsys);
  hipLaunchKernelGGL(keys_k, dim3(kx, nsys), dim3(256), 0, s, xyzm, c->b.soff, c->prm.key_kind,
                     c->b.sys, toB ? c->b.keyB : c->b.keyA, toB ? c->b.idxB : c->b.idxA);
}

}  // namespace gothic
