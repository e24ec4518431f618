// C ABI (include/gothic.h): errors, tunables, context creation and
// destruction, scratch accounting and the sticky device flags.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "api_internal.h"

namespace gothic {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return GOTHIC_OK;
  return set_error(e == hipErrorOutOfMemory ? GOTHIC_ENOMEM : GOTHIC_EDEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

int validate_params(const gothic_params *p) {
  if (p->key_kind != GOTHIC_KEY_MORTON && p->key_kind != GOTHIC_KEY_PEANO_HILBERT)
    return set_error(GOTHIC_EINVAL, "key_kind must be 0 (Morton) or 1 (Peano-Hilbert)");
  if (p->n_leaf < 1 || p->n_leaf > 64) return set_error(GOTHIC_EINVAL, "n_leaf must be in 1..64");
  if (p->multipole != 1 && p->multipole != 2)
    return set_error(GOTHIC_EINVAL, "multipole must be 1 or 2");
  const int G = p->group_size;
  if (G < 1 || G > 64 || (G & (G - 1)))
    return set_error(GOTHIC_EINVAL, "group_size must be a power of two in 1..64");
  if (p->list_depth < 64 || p->list_depth > 1024 || (p->list_depth % 64))
    return set_error(GOTHIC_EINVAL, "list_depth must be a multiple of 64 in 64..1024");
  if (p->compensated != 0 && p->compensated != 1)
    return set_error(GOTHIC_EINVAL, "compensated must be 0 or 1");
  if (p->check != 0 && p->check != 1) return set_error(GOTHIC_EINVAL, "check must be 0 or 1");
  if (p->node_capacity < 0) return set_error(GOTHIC_EINVAL, "node_capacity must be >= 0");
  if (p->timing != 0 && p->timing != 1) return set_error(GOTHIC_EINVAL, "timing must be 0 or 1");
  if (!std::isfinite(p->r_crit)) return set_error(GOTHIC_EINVAL, "r_crit must be finite");
  if (p->graph != 0 && p->graph != 1) return set_error(GOTHIC_EINVAL, "graph must be 0 or 1");
  if (p->autotune < 0 || p->autotune > 2)
    return set_error(GOTHIC_EINVAL, "autotune must be 0, 1 or 2");
  if (p->rebuild_interval < 0 || p->rebuild_interval > (1 << 20))
    return set_error(GOTHIC_EINVAL, "rebuild_interval must be in 0..2^20");
  if (p->mac < 0 || p->mac > 2) return set_error(GOTHIC_EINVAL, "mac must be 0, 1 or 2");
  if (!(p->mac_delta > 0.f) || !std::isfinite(p->mac_delta))
    return set_error(GOTHIC_EINVAL, "mac_delta must be finite and > 0");
  if (p->ball < 0 || p->ball > 4) return set_error(GOTHIC_EINVAL, "ball must be in 0..4");
  if (p->max_scratch_bytes < 0) return set_error(GOTHIC_EINVAL, "max_scratch_bytes must be >= 0");
  if (p->spill_per_wave != 0 && (p->spill_per_wave < 256 || p->spill_per_wave > (1 << 24)))
    return set_error(GOTHIC_EINVAL, "spill_per_wave must be 0 or in 256..2^24");
  if (p->walk_width != 0 && p->walk_width != 16 && p->walk_width != 32 && p->walk_width != 64)
    return set_error(GOTHIC_EINVAL, "walk_width must be 0, 16, 32 or 64");
  if (G > walk_width_of(*p))
    return set_error(GOTHIC_EINVAL, "group_size must not exceed walk_width");
  return GOTHIC_OK;
}

// Make sure every buffer can hold n particles (and the current node / spill

__global__ void clear_flags_k(Ctl *ctl) {
  if (threadIdx.x == 0) {
    ctl->flags = 0u;
    ctl->sticky = 0u;
  }
}

}  // namespace gothic

using namespace gothic;

extern "C" {

void gothic_default_params(gothic_params *p) {
  if (!p) return;
  p->key_kind = GOTHIC_KEY_MORTON;
  p->n_leaf = 16;
  p->multipole = 1;
  p->group_size = 32;
  p->list_depth = 384;
  p->compensated = 1;
  p->check = 1;
  p->timing = 0;
  p->r_crit = -0.0625f;
  p->graph = 0;
  p->autotune = 0;
  p->rebuild_interval = 1;
  p->mac = 0;
  p->mac_delta = 0.0078125f;  // 2^-7
  p->ball = 0;
  p->node_capacity = 0;
  p->max_scratch_bytes = 0;
  p->spill_per_wave = 0;
  p->walk_width = 64;
}

const char *gothic_last_error(void) { return g_last_error.c_str(); }

int gothic_create(gothic_ctx **out, int hip_device, const gothic_params *p) {
  if (!out) return set_error(GOTHIC_EINVAL, "out is NULL");
  *out = nullptr;
  gothic_params prm;
  gothic_default_params(&prm);
  if (p) prm = *p;
  int rc = validate_params(&prm);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return set_error(GOTHIC_EDEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= ndev) return set_error(GOTHIC_EINVAL, "bad device index");
  DeviceGuard guard(hip_device);
  hipDeviceProp_t prop;
  if ((rc = hip_check(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties")))
    return rc;
  if ((rc = static_scratch_attach(hip_device))) return rc;
  gothic_ctx *c = new gothic_ctx();
  c->device = hip_device;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  c->prm = prm;
  c->lb = &c->b;
  *out = c;
  return GOTHIC_OK;
}

int gothic_destroy(gothic_ctx *c) {
  if (!c) return GOTHIC_OK;
  {
    DeviceGuard guard(c->device);
    (void)hipDeviceSynchronize();
    free_graphs(c);
    if (c->graphs.cap_stream) (void)hipStreamDestroy(c->graphs.cap_stream);
    if (c->tune.ev0) (void)hipEventDestroy(c->tune.ev0);
    if (c->tune.ev1) (void)hipEventDestroy(c->tune.ev1);
    if (c->tree.mk0) (void)hipEventDestroy(c->tree.mk0);
    if (c->tree.mk1) (void)hipEventDestroy(c->tree.mk1);
    free_sim(c);
    free_events(c);
    free_all(c);
    if (c->direct_part) (void)hipFree(c->direct_part);
  }
  delete c;
  return GOTHIC_OK;
}

int gothic_set_params(gothic_ctx *c, const gothic_params *p) {
  if (!c || !p) return set_error(GOTHIC_EINVAL, "NULL argument");
  int rc = validate_params(p);
  if (rc) return rc;
  // r_crit is read from device memory and check, timing and autotune act
  // outside the captured segments: only the other fields invalidate them
  const gothic_params &a = c->prm, &b = *p;
  if (a.key_kind != b.key_kind || a.n_leaf != b.n_leaf || a.multipole != b.multipole ||
      a.group_size != b.group_size || a.list_depth != b.list_depth ||
      a.compensated != b.compensated || a.graph != b.graph || a.mac != b.mac ||
      a.mac_delta != b.mac_delta || a.ball != b.ball || a.node_capacity != b.node_capacity ||
      a.spill_per_wave != b.spill_per_wave || a.walk_width != b.walk_width)
    ++c->generation;
  c->prm = *p;
  return GOTHIC_OK;
}

int gothic_get_params(const gothic_ctx *c, gothic_params *p) {
  if (!c || !p) return set_error(GOTHIC_EINVAL, "NULL argument");
  *p = c->prm;
  return GOTHIC_OK;
}

int gothic_get_scratch(gothic_ctx *c, int64_t *held, int64_t *required) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (held) *held = c->scratch_held + (int64_t)sizeof(double4) * c->cap_direct;
  if (required) *required = c->scratch_required;
  return GOTHIC_OK;
}

int gothic_clear_flags(gothic_ctx *c, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  DeviceGuard guard(c->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (c->b.ctl) hipLaunchKernelGGL(clear_flags_k, dim3(1), dim3(64), 0, s, c->b.ctl);
  if (c->lb && c->lb != &c->b && c->lb->ctl)
    hipLaunchKernelGGL(clear_flags_k, dim3(1), dim3(64), 0, s, c->lb->ctl);
  return hip_check(hipGetLastError(), "clear_flags_k");
}

}  // extern "C"
