// Scratch-free evaluation (gothic_tree_forces_noalloc): the pipeline of
// gothic_tree_forces run in one fixed device array instead of the context's
// growable scratch, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy of kStaticScratchBytes from the first context created
// on it until the process ends.  In host code its name is only a host-side
// stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, device current) and only that address is ever handed
// to kernels.  Every scratch-free call on one GPU works in the same array and
// leaves its contents behind: the control block is cleared by a kernel at the
// start of each call, and calls that overlap in time on one GPU race.
#include <cmath>
#include <mutex>
#include <string>

#include "api_internal.h"

namespace gothic {

constexpr int64_t kStaticScratchBytes = 256ll << 20;  // per GPU
constexpr int64_t kStaticSpill = 4096;                 // pending entries per walk wave
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices];

// Look up this device's copy of the array (the device must be current).
int static_scratch_attach(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GOTHIC_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return GOTHIC_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                              "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[dev] = static_cast<char *>(p);
  return GOTHIC_OK;
}

static char *static_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

// the whole control block, sticky word included, starts at zero
__global__ void ctl_zero_k(Ctl *ctl) {
  unsigned *w = reinterpret_cast<unsigned *>(ctl);
  for (unsigned i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0u;
}

// Capacities of one scratch-free evaluation of n particles.
static Caps static_caps(gothic_ctx *c, int64_t n) {
  Caps k;
  k.n = n;
  k.sys = 1;
  k.nodes = c->prm.node_capacity > 0 ? c->prm.node_capacity
                                     : n + 8 * (n / c->prm.n_leaf) + 1024 + 1;
  k.anc = n;
  k.waves = walk_slots(c);
  k.spill = c->prm.spill_per_wave > 0 ? c->prm.spill_per_wave : kStaticSpill;
  return k;
}

// The launchers read the context's buffers and capacities: lend them the
// carved ones for the duration of the enqueue, then put the context's back.
// The carved set stays in c->sb for the read-back calls.
struct LendBuffers {
  gothic_ctx *c;
  Buffers own;
  int64_t cap_n, cap_nodes, spill;
  int waves;
  LendBuffers(gothic_ctx *ctx, const Buffers &carved, const Caps &k)
      : c(ctx), own(ctx->b), cap_n(ctx->cap_n), cap_nodes(ctx->cap_nodes),
        spill(ctx->spill_per_wave), waves(ctx->walk_waves) {
    c->b = carved;
    c->cap_n = k.n;
    c->cap_nodes = k.nodes;
    c->spill_per_wave = k.spill;
    c->walk_waves = (int)k.waves;
  }
  ~LendBuffers() {
    c->sb = c->b;
    c->b = own;
    c->cap_n = cap_n;
    c->cap_nodes = cap_nodes;
    c->spill_per_wave = spill;
    c->walk_waves = waves;
  }
};

}  // namespace gothic

using namespace gothic;

extern "C" {

int gothic_tree_forces_noalloc(gothic_ctx *c, int64_t n, const float *xyzm, float eps,
                               float theta, const uint8_t *active, float *acc_pot, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (n < 0 || n >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "n must be in [0, 2^31)");
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(GOTHIC_EINVAL, "eps must be finite and > 0");
  if (!(theta >= 0.f && theta < 1.f)) return set_error(GOTHIC_EINVAL, "theta must be in [0, 1)");
  if (n == 0) return GOTHIC_OK;
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  if ((const void *)xyzm == (const void *)acc_pot)
    return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not overlap");
  if (c->prm.mac == 1)
    return set_error(GOTHIC_EINVAL, "the acceleration MAC needs the previous accelerations");
  DeviceGuard guard(c->device);
  char *base = static_scratch(c->device);
  if (!base) return set_error(GOTHIC_EDEVICE, "static scratch not attached to this device");
  const int64_t off[2] = {0, n};
  Systems sy;
  int rc = make_systems(1, off, &eps, &theta, false, &sy);
  if (rc) return rc;
  c->cur_G = c->prm.group_size;
  c->cur_W = walk_width_of(c->prm);
  const Caps k = static_caps(c, n);
  const int64_t need = scratch_bytes(k);
  if (need > kStaticScratchBytes) {
    c->scratch_required = need;
    return set_error(GOTHIC_ENOMEM, "n = " + std::to_string(n) + " needs " +
                                        std::to_string(need) + " bytes of scratch, above the " +
                                        std::to_string(kStaticScratchBytes) +
                                        " bytes of the scratch-free entry point");
  }
  Buffers carved;
  carve_buffers(carved, k, base);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  {
    LendBuffers lend(c, carved, k);
    hipLaunchKernelGGL(ctl_zero_k, dim3(1), dim3(256), 0, s, c->b.ctl);
    rc = enqueue_forces(c, sy, reinterpret_cast<const float4 *>(xyzm), active, nullptr,
                        reinterpret_cast<float4 *>(acc_pot), s, c->prm.r_crit, true, false,
                        false);
  }
  if (rc) return rc;
  mark_last(c, sy, s, &c->sb);
  return GOTHIC_OK;
}

}  // extern "C"
