// Softened direct summation in float64 (the Plummer-softened force and
// potential of Section 1 with G = 1) for a set of target particles: the
// accuracy reference that the errors of the tree force are measured against
// (Section 3.2 measures them against direct summation, Fig. 3).
//
// Layout: targets run along x of the grid (one per thread), the j-particles
// along y in chunks of whole 256-particle tiles staged through LDS.  Each
// (target, chunk) pair writes one float64 partial; a second kernel adds the
// chunks of a target in chunk order, so the result does not depend on timing.
#include <cmath>

#include "api_internal.h"

namespace gothic {
namespace {

constexpr int kDirectThreads = 256;
constexpr int kDirectBlocks = 4096;  // target tiles x chunks aimed for

__global__ void __launch_bounds__(kDirectThreads)
direct_part_k(int64_t n, const float4 *__restrict__ xyzm, double eps2, int64_t ni,
              const int64_t *__restrict__ idx, int64_t chunk, double4 *__restrict__ part) {
  __shared__ float4 tile[kDirectThreads];
  const int64_t k = (int64_t)blockIdx.x * kDirectThreads + threadIdx.x;
  const int64_t kc = k < ni ? k : ni - 1;
  const int64_t want = idx ? idx[kc] : kc;
  const bool valid = want >= 0 && want < n;
  const int64_t i = valid ? want : 0;
  const float4 pi = xyzm[i];
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
  for (int64_t t = j0; t < j1; t += kDirectThreads) {
    const int64_t j = t + threadIdx.x;
    __syncthreads();
    tile[threadIdx.x] = j < j1 ? xyzm[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int m = (int)(j1 - t < kDirectThreads ? j1 - t : kDirectThreads);
    for (int q = 0; q < m; ++q) {
      const float4 pj = tile[q];
      const double dx = (double)pj.x - xi, dy = (double)pj.y - yi, dz = (double)pj.z - zi;
      const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
      const double rinv = rsqrt(r2);
      const double mr = (t + q == i) ? 0.0 : (double)pj.w * rinv;  // the pair j = i is left out
      const double mr3 = mr * rinv * rinv;
      ax = fma(mr3, dx, ax);
      ay = fma(mr3, dy, ay);
      az = fma(mr3, dz, az);
      ph -= mr;
    }
  }
  if (k < ni) {
    const double bad = __longlong_as_double(0x7ff8000000000000ll);
    part[(int64_t)blockIdx.y * ni + k] =
        valid ? make_double4(ax, ay, az, ph) : make_double4(bad, bad, bad, bad);
  }
}

__global__ void direct_sum_k(int64_t ni, int nchunk, const double4 *__restrict__ part,
                             double *__restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ni;
       k += (int64_t)gridDim.x * blockDim.x) {
    double4 s = part[k];
    for (int c = 1; c < nchunk; ++c) {
      const double4 p = part[(int64_t)c * ni + k];
      s.x += p.x;
      s.y += p.y;
      s.z += p.z;
      s.w += p.w;
    }
    out[4 * k] = s.x;
    out[4 * k + 1] = s.y;
    out[4 * k + 2] = s.z;
    out[4 * k + 3] = s.w;
  }
}

}  // namespace

// chunks of j-particles for ni targets among n particles, and the chunk length
void direct_plan(int64_t n, int64_t ni, int *nchunk, int64_t *chunk) {
  const int64_t tiles_i = (ni + kDirectThreads - 1) / kDirectThreads;
  const int64_t tiles_j = (n + kDirectThreads - 1) / kDirectThreads;
  int64_t want = (kDirectBlocks + tiles_i - 1) / tiles_i;
  if (want > tiles_j) want = tiles_j;
  if (want < 1) want = 1;
  const int64_t per = (tiles_j + want - 1) / want;  // tiles per chunk
  *chunk = per * kDirectThreads;
  *nchunk = (int)((tiles_j + per - 1) / per);
}

void launch_direct(int64_t n, const float4 *xyzm, double eps, int64_t ni, const int64_t *idx,
                   double4 *part, double *out, hipStream_t s) {
  int nchunk;
  int64_t chunk;
  direct_plan(n, ni, &nchunk, &chunk);
  const dim3 grid((unsigned)((ni + kDirectThreads - 1) / kDirectThreads), (unsigned)nchunk);
  hipLaunchKernelGGL(direct_part_k, grid, dim3(kDirectThreads), 0, s, n, xyzm, eps * eps, ni,
                     idx, chunk, part);
  const int64_t nb = (ni + 255) / 256;
  hipLaunchKernelGGL(direct_sum_k, dim3((unsigned)(nb > 4096 ? 4096 : nb)), dim3(256), 0, s, ni,
                     nchunk, part, out);
}

}  // namespace gothic

using namespace gothic;

extern "C" {

int gothic_direct_forces(gothic_ctx *c, int64_t n, const float *xyzm, float eps, int64_t ni,
                         const int64_t *idx, double *acc_pot, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (n < 0 || n >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "n must be in [0, 2^31)");
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(GOTHIC_EINVAL, "eps must be finite and > 0");
  if (ni < 0 || ni >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "ni must be in [0, 2^31)");
  if (ni == 0) return GOTHIC_OK;
  if (n == 0) return set_error(GOTHIC_EINVAL, "targets need particles (n = 0)");
  if (!idx && ni > n) return set_error(GOTHIC_EINVAL, "without idx, ni must be <= n");
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  DeviceGuard guard(c->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int nchunk;
  int64_t chunk;
  direct_plan(n, ni, &nchunk, &chunk);
  const int64_t want = (int64_t)nchunk * ni;
  int rc;
  if (want > c->cap_direct) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cap);
    if (cap != hipStreamCaptureStatusNone)
      return set_error(GOTHIC_ECAPTURE, "direct-sum scratch must grow; call once uncaptured first");
    if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    if ((rc = dev_alloc(&c->direct_part, want))) {
      c->cap_direct = 0;
      return rc;
    }
    c->cap_direct = want;
  }
  launch_direct(n, reinterpret_cast<const float4 *>(xyzm), (double)eps, ni, idx, c->direct_part,
                acc_pot, s);
  return hip_check(hipGetLastError(), "direct-sum launch");
}


}  // extern "C"
