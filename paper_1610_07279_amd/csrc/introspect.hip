// Read-back of the last evaluation for tests and diagnostics: counts and
// flags, keys, tree, node moments, groups, walk timings, and the interaction
// lists of chosen groups.
#include <string.h>

#include <algorithm>
#include <string>

#include "api_internal.h"

namespace gothic {

__global__ void extract_cubes_k(int nsys, const SysRec *sys, double *cube) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x)
    for (int a = 0; a < 4; ++a) cube[4 * s + a] = sys[s].cube[a];
}

__global__ void extract_nodes_k(const Ctl *ctl, const float4 *nrec, const float4 *quad,
                                float4 *com_m, float *b, float *q6) {
  const int64_t nn = ctl->n_nodes;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (com_m) com_m[k] = nrec[2 * k];
    if (b) b[k] = nrec[2 * k + 1].x;
    if (q6) {
      const float4 a = quad[2 * k], c = quad[2 * k + 1];
      q6[6 * k + 0] = a.x; q6[6 * k + 1] = a.y; q6[6 * k + 2] = a.z;
      q6[6 * k + 3] = a.w; q6[6 * k + 4] = c.x; q6[6 * k + 5] = c.y;
    }
  }
}

__global__ void extract_groups_k(const Ctl *ctl, const uint32_t *gf, uint32_t *gfirst,
                                 uint32_t *gcount) {
  const unsigned ng = ctl->n_groups;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    if (gfirst) gfirst[g] = gf[g];
    if (gcount) gcount[g] = gf[g + 1] - gf[g];
  }
}

// copy the control block of the last evaluation to the host (synchronises)
static int fetch_ctl(gothic_ctx *c, Ctl *h) {
  Buffers *lb = c->lb ? c->lb : &c->b;
  if (!lb->ctl) return set_error(GOTHIC_EINVAL, "no evaluation yet");
  if (!c->b.ctl_host)
    GCHECK(hipHostMalloc(reinterpret_cast<void **>(&c->b.ctl_host), sizeof(Ctl),
                         hipHostMallocDefault));
  GCHECK(hipMemcpyAsync(c->b.ctl_host, lb->ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                        c->last_stream));
  GCHECK(hipStreamSynchronize(c->last_stream));
  *h = *c->b.ctl_host;
  return GOTHIC_OK;
}

static int d2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!dst || !bytes) return GOTHIC_OK;
  return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
}

}  // namespace gothic

using namespace gothic;

extern "C" {

int gothic_get_stats(gothic_ctx *c, gothic_stats *out) {
  if (!c || !out) return set_error(GOTHIC_EINVAL, "NULL argument");
  memset(out, 0, sizeof(*out));
  if (!c->have_last) return GOTHIC_OK;
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = fetch_ctl(c, &h);
  if (rc) return rc;
  out->n = c->last_n;
  out->n_active = h.n_active;
  out->n_nodes = h.n_nodes;
  out->n_groups = h.n_groups;
  int lev = 0;
  for (int l = 0; l < kMaxLevels; ++l)
    if (h.lvl_start[l + 1] > h.lvl_start[l]) lev = l + 1;
  out->n_levels = lev;
  out->node_entries = (int64_t)h.node_entries;
  out->part_entries = (int64_t)h.part_entries;
  out->interactions = (int64_t)h.interactions;
  out->node_interactions = (int64_t)h.node_interactions;
  out->mac_tests = (int64_t)h.mac_tests;
  out->flags = (int32_t)h.flags;
  out->n_systems = c->last_nsys;
  out->sticky_flags = (int32_t)((h.sticky | h.flags) & kFlagMask);
  if (h.flags & kFlagNonFinite) return set_error(GOTHIC_ENONFINITE, "non-finite position or mass");
  if (h.flags & (kFlagNodeOverflow | kFlagSpillOverflow))
    return set_error(GOTHIC_EOVERFLOW, "capacity exceeded in the last evaluation");
  if (h.flags & kFlagBadIndex) return set_error(GOTHIC_EDEVICE, "internal index check failed");
  return GOTHIC_OK;
}

static int last_counts(gothic_ctx *c, Ctl *h) {
  if (!c->have_last) return set_error(GOTHIC_EINVAL, "no evaluation yet");
  return fetch_ctl(c, h);
}

int gothic_get_keys(gothic_ctx *c, uint64_t *keys_sorted, uint32_t *perm, double *cube) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  const Buffers &L = *c->lb;
  hipStream_t s = c->last_stream;
  const size_t n = (size_t)c->last_n;
  if ((rc = d2d(keys_sorted, L.keyA, n * 8, s)) || (rc = d2d(perm, L.idxA, n * 4, s))) return rc;
  if (cube) {
    hipLaunchKernelGGL(extract_cubes_k, dim3(1), dim3(256), 0, s, c->last_nsys, L.sys, cube);
    if ((rc = hip_check(hipGetLastError(), "extract_cubes_k"))) return rc;
  }
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_positions(gothic_ctx *c, float *xyzm_sorted) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  const Buffers &L = *c->lb;
  hipStream_t s = c->last_stream;
  if ((rc = d2d(xyzm_sorted, L.pos, (size_t)c->last_n * 16, s))) return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_tree(gothic_ctx *c, int64_t *n_nodes, uint32_t *first, uint32_t *count,
                    uint32_t *child_first, uint8_t *n_child, uint8_t *level) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  const Buffers &L = *c->lb;
  hipStream_t s = c->last_stream;
  const size_t nn = h.n_nodes;
  if (n_nodes) *n_nodes = (int64_t)nn;
  if ((rc = d2d(first, L.first, nn * 4, s)) || (rc = d2d(count, L.count, nn * 4, s)) ||
      (rc = d2d(child_first, L.child_first, nn * 4, s)) ||
      (rc = d2d(n_child, L.n_child, nn, s)) || (rc = d2d(level, L.level, nn, s)))
    return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_nodes(gothic_ctx *c, float *com_m, float *b, float *quad) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  const Buffers &L = *c->lb;
  hipStream_t s = c->last_stream;
  hipLaunchKernelGGL(extract_nodes_k, dim3(1024), dim3(256), 0, s, L.ctl, L.nrec, L.quad,
                     reinterpret_cast<float4 *>(com_m), b, quad);
  if ((rc = hip_check(hipGetLastError(), "extract_nodes_k"))) return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_groups(gothic_ctx *c, int64_t *n_active, int64_t *n_groups, uint32_t *alist,
                      uint32_t *gfirst, uint32_t *gcount, float *ball, uint32_t *entries) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  const Buffers &L = *c->lb;
  hipStream_t s = c->last_stream;
  if (n_active) *n_active = h.n_active;
  if (n_groups) *n_groups = h.n_groups;
  if ((rc = d2d(alist, L.alist, (size_t)h.n_active * 4, s)) ||
      (rc = d2d(ball, L.ball, (size_t)h.n_groups * 16, s)) ||
      (rc = d2d(entries, L.gent, (size_t)h.n_groups * 8, s)))
    return rc;
  if (gfirst || gcount) {
    hipLaunchKernelGGL(extract_groups_k, dim3(256), dim3(256), 0, s, L.ctl, L.gfirst, gfirst,
                       gcount);
    if ((rc = hip_check(hipGetLastError(), "extract_groups_k"))) return rc;
  }
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_lists(gothic_ctx *c, int64_t ngsel, const uint32_t *gsel, int64_t cap,
                     uint32_t *entries, uint32_t *counts, float *acc_pot) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  if (ngsel < 0 || ngsel > (1 << 20)) return set_error(GOTHIC_EINVAL, "ngsel must be in 0..2^20");
  if (ngsel == 0) return GOTHIC_OK;
  if (!gsel || !entries || !counts || !acc_pot)
    return set_error(GOTHIC_EINVAL, "gsel, entries, counts and acc_pot must not be NULL");
  if (cap < 1 || cap > (int64_t)1 << 26) return set_error(GOTHIC_EINVAL, "cap must be in 1..2^26");
  if (c->lb != &c->b) return set_error(GOTHIC_EINVAL, "the last evaluation used no context scratch");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  for (int64_t k = 0; k < ngsel; ++k)
    if (gsel[k] >= h.n_groups) return set_error(GOTHIC_EINVAL, "gsel names a group past n_groups");
  if (h.flags & (kFlagNodeOverflow | kFlagSpillOverflow | kFlagBadIndex))
    return set_error(GOTHIC_EOVERFLOW, "the last evaluation did not finish its walk");
  hipStream_t s = c->last_stream;
  uint32_t *dsel = nullptr;
  if ((rc = dev_alloc(&dsel, ngsel))) return rc;
  Buffers &B = c->b;
  rc = hip_check(hipMemcpyAsync(dsel, gsel, 4 * (size_t)ngsel, hipMemcpyHostToDevice, s),
                 "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipMemsetAsync(counts, 0, 8 * (size_t)ngsel, s), "hipMemsetAsync");
  if (!rc) {
    B.gsel = dsel;
    B.ngsel = (unsigned)ngsel;
    B.rec = entries;
    B.rec_n = counts;
    B.rec_cap = cap;
    launch_walk(c, c->last_n, reinterpret_cast<float4 *>(acc_pot), s);
    B.gsel = nullptr;
    B.ngsel = 0;
    B.rec = B.rec_n = nullptr;
    B.rec_cap = 0;
    rc = hip_check(hipGetLastError(), "walk launch");
  }
  const int rs = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  (void)hipFree(dsel);
  return rc ? rc : rs;
}

int gothic_get_walk_time(gothic_ctx *c, double *ms_total, int64_t *launches) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  double tot = 0.0;
  for (int i = 0; i < c->ev_used; ++i) {
    int rc;
    if ((rc = hip_check(hipEventSynchronize(c->ev_stop[i]), "hipEventSynchronize"))) return rc;
    float ms = 0.f;
    if ((rc = hip_check(hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]),
                        "hipEventElapsedTime")))
      return rc;
    tot += ms;
  }
  if (ms_total) *ms_total = tot;
  if (launches) *launches = c->ev_used;
  c->ev_used = 0;
  return GOTHIC_OK;
}

}  // extern "C"
