// The force pipeline of one evaluation (keys, sort, octree, moments, groups,
// walk) as enqueued on a stream, the tree-reuse and metering state around it,
// and the C entry points of one evaluation.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "api_internal.h"

namespace gothic {

// ---------------------------------------------------------------- helpers
// Zero the control block before an evaluation.  keep_tree keeps the tree of
// the last build (node count, level starts, systems); a tree whose build
// overflowed is not reusable and is reported as a node overflow.  The flags
// of the previous evaluation are ORed into the sticky word (fold), unless the
// host has already handled them (a repeat after growing the scratch); the
// sticky word itself is kept.
__global__ void ctl_reset_k(Ctl *ctl, int keep_tree, int fold) {
  const unsigned keep_nodes = ctl->n_nodes, keep_sys = ctl->nsys, ok = ctl->tree_ok;
  const unsigned sticky = ctl->sticky | (fold ? (ctl->flags & kFlagMask) : 0u);
  unsigned lv = 0;
  if (threadIdx.x < kMaxLevels + 2) lv = ctl->lvl_start[threadIdx.x];
  __syncthreads();
  unsigned *w = reinterpret_cast<unsigned *>(ctl);
  for (unsigned i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) ctl->sticky = sticky;
  if (keep_tree) {
    if (threadIdx.x < kMaxLevels + 2) ctl->lvl_start[threadIdx.x] = lv;
    if (threadIdx.x == 0) {
      ctl->n_nodes = keep_nodes;
      ctl->nsys = keep_sys;
      ctl->tree_ok = ok;
      if (!ok) ctl->flags = kFlagNodeOverflow;
    }
  }
}

// Forget the flags of the last evaluation (the host has handled them), so the
// next reset does not make them sticky.
__global__ void drop_flags_k(Ctl *ctl) {
  if (threadIdx.x == 0) ctl->flags = 0u;
}

void enqueue_drop_flags(gothic_ctx *c, hipStream_t s) {
  hipLaunchKernelGGL(drop_flags_k, dim3(1), dim3(64), 0, s, c->b.ctl);
}

// The system table travels in kernel arguments (captured by value in a
// graph), kSysChunk systems per launch: no host staging buffer that a later
// call could overwrite before the copy runs.
constexpr int kSysChunk = 32;
struct SysChunk {
  int first, count;
  uint32_t off[kSysChunk + 1];
  float eps2[kSysChunk], theta[kSysChunk], inv_eps[kSysChunk];
};

__global__ void sys_upload_k(SysChunk ch, SysRec *sys, uint32_t *soff) {
  const int t = threadIdx.x;
  if (t < ch.count) {
    SysRec &r = sys[ch.first + t];
    r.eps2 = ch.eps2[t];
    r.theta = ch.theta[t];
    r.inv_eps = ch.inv_eps[t];
  }
  if (t <= ch.count) soff[ch.first + t] = ch.off[t];
}

__global__ void set_rcrit_k(float r, float *dst) {
  if (threadIdx.x == 0) *dst = r;
}


void enqueue_begin(gothic_ctx *c, bool keep_tree, float r_crit, hipStream_t s, bool fold) {
  hipLaunchKernelGGL(ctl_reset_k, dim3(1), dim3(64), 0, s, c->b.ctl, keep_tree ? 1 : 0,
                     fold ? 1 : 0);
  hipLaunchKernelGGL(set_rcrit_k, dim3(1), dim3(64), 0, s, r_crit, c->b.rcrit);
}

void enqueue_upload(gothic_ctx *c, const Systems &sy, hipStream_t s) {
  Buffers &B = c->b;
  for (int f = 0; f < sy.nsys; f += kSysChunk) {
    SysChunk ch;
    memset(&ch, 0, sizeof(ch));
    ch.first = f;
    ch.count = std::min(kSysChunk, sy.nsys - f);
    for (int t = 0; t <= ch.count; ++t) ch.off[t] = (uint32_t)sy.off[f + t];
    for (int t = 0; t < ch.count; ++t) {
      const float e = sy.eps[f + t];
      ch.eps2[t] = e * e;
      ch.theta[t] = sy.theta[f + t];
      ch.inv_eps[t] = 1.0f / e;
    }
    hipLaunchKernelGGL(sys_upload_k, dim3(1), dim3(64), 0, s, ch, B.sys, B.soff);
  }
}

void enqueue_make(gothic_ctx *c, const Systems &sy, const float4 *xyzm, hipStream_t s) {
  launch_bbox_keys(c, xyzm, sy.n, sy.nsys, sy.max_n, s);
  launch_radix_sort(c, sy.n, sy.nsys, s);
  launch_build(c, sy.n, sy.nsys, s);
  launch_ancestors(c, sy.n, s);
}

// sign_active: the active flags are the sign bits of the masses in xyzm
// (the block-step predictor's shadow); active is then not read
void enqueue_post(gothic_ctx *c, const Systems &sy, const float4 *xyzm, const uint8_t *active,
                  const float4 *acc_old, hipStream_t s, bool sign_active) {
  launch_permute(c, xyzm, active, sign_active, c->prm.mac == 1 ? acc_old : nullptr, sy.n, s);
  launch_moments(c, sy.n, sy.nsys, s);
  launch_groups(c, sy.n, s);
}

void enqueue_walk(gothic_ctx *c, int64_t n, float4 *out, hipStream_t s, bool timed) {
  timed = timed && c->prm.timing && c->ev_used < (int)c->ev_start.size();
  const bool tuned = c->tune.recording;
  if (tuned) (void)hipEventRecord(c->tune.ev0, s);
  if (timed) (void)hipEventRecord(c->ev_start[c->ev_used], s);
  launch_walk(c, n, out, s);
  if (timed) (void)hipEventRecord(c->ev_stop[c->ev_used++], s);
  if (tuned) (void)hipEventRecord(c->tune.ev1, s);
}

// One evaluation (eager).  rebuild = false walks the tree of the last build
// with the current positions.  The construction is timed when the rebuild
// models are being fed.
int enqueue_forces(gothic_ctx *c, const Systems &sy, const float4 *xyzm, const uint8_t *active,
                   const float4 *acc_old, float4 *out, hipStream_t s, float r_crit, bool rebuild,
                   bool sign_active, bool fold) {
  enqueue_begin(c, !rebuild, r_crit, s, fold);
  enqueue_upload(c, sy, s);
  if (rebuild) {
    const bool tm = c->tune.recording && c->tree.mk0;
    if (tm) (void)hipEventRecord(c->tree.mk0, s);
    enqueue_make(c, sy, xyzm, s);
    if (tm) (void)hipEventRecord(c->tree.mk1, s);
  }
  enqueue_post(c, sy, xyzm, active, acc_old, s, sign_active);
  enqueue_walk(c, sy.n, out, s, true);
  return hip_check(hipGetLastError(), "kernel launch");
}

// Checks a batched description and drops empty systems.
int make_systems(int nsys, const int64_t *offsets, const float *eps, const float *theta,
                 bool allow_empty, Systems *out) {
  if (nsys < 1 || nsys > kMaxSys) return set_error(GOTHIC_EINVAL, "nsys must be in 1..65535");
  if (!offsets || !eps || !theta)
    return set_error(GOTHIC_EINVAL, "offsets, eps and theta must not be NULL");
  if (offsets[0] != 0) return set_error(GOTHIC_EINVAL, "offsets[0] must be 0");
  Systems sy;
  sy.off.push_back(0);
  for (int k = 0; k < nsys; ++k) {
    const int64_t a = offsets[k], b = offsets[k + 1];
    if (b < a) return set_error(GOTHIC_EINVAL, "offsets must be non-decreasing");
    if (b >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "total particles must be < 2^31");
    if (!(eps[k] > 0.f) || !std::isfinite(eps[k]))
      return set_error(GOTHIC_EINVAL, "eps must be finite and > 0");
    if (!(theta[k] >= 0.f && theta[k] < 1.f))
      return set_error(GOTHIC_EINVAL, "theta must be in [0, 1)");
    if (b == a) {
      if (!allow_empty) return set_error(GOTHIC_EINVAL, "empty system");
      continue;
    }
    sy.off.push_back(b);
    sy.eps.push_back(eps[k]);
    sy.theta.push_back(theta[k]);
    sy.max_n = std::max(sy.max_n, b - a);
  }
  sy.nsys = (int)sy.eps.size();
  sy.n = offsets[nsys];
  *out = std::move(sy);
  return GOTHIC_OK;
}

void free_events(gothic_ctx *c) {
  for (auto e : c->ev_start) (void)hipEventDestroy(e);
  for (auto e : c->ev_stop) (void)hipEventDestroy(e);
  c->ev_start.clear();
  c->ev_stop.clear();
  c->ev_used = 0;
}

int ensure_events(gothic_ctx *c) {
  constexpr int kPool = 4096;
  if (!c->prm.timing || !c->ev_start.empty()) return GOTHIC_OK;
  c->ev_start.resize(kPool);
  c->ev_stop.resize(kPool);
  for (int i = 0; i < kPool; ++i) {
    int rc;
    if ((rc = hip_check(hipEventCreate(&c->ev_start[i]), "hipEventCreate")) ||
        (rc = hip_check(hipEventCreate(&c->ev_stop[i]), "hipEventCreate"))) {
      c->ev_start.resize(i);
      c->ev_stop.resize(i);
      return rc;
    }
  }
  return GOTHIC_OK;
}

// A new tree is built when the last one does not fit the call (no tree yet,
// other systems, grown buffers, another leaf size or key kind); otherwise by
// params.rebuild_interval: 1 every time, k > 1 after k evaluations on one
// tree, 0 when the paper's growth models say so.
bool must_rebuild(gothic_ctx *c, const Systems &sy) {
  const TreeState &T = c->tree;
  if (!T.valid || T.n != sy.n || T.off != sy.off || T.buffers != c->buffers ||
      T.n_leaf != c->prm.n_leaf || T.key_kind != c->prm.key_kind)
    return true;
  const int k = c->prm.rebuild_interval;
  if (k == 1) return true;
  if (k >= 2) return T.since >= k;
  return T.models.due();
}

void tree_used(gothic_ctx *c, const Systems &sy, bool rebuilt) {
  TreeState &T = c->tree;
  if (rebuilt) {
    T.valid = true;
    T.n = sy.n;
    T.off = sy.off;
    T.n_leaf = c->prm.n_leaf;
    T.key_kind = c->prm.key_kind;
    T.buffers = c->buffers;
    T.since = 1;
  } else {
    ++T.since;
  }
}

// ---------------------------------------------------------------- measurement
// The online tuners (params.autotune: r_crit per sub-step class;
// rebuild_interval = 0: the growth models) are fed with the walk time of each
// evaluation and the construction time of each rebuild, read one evaluation
// late so the host does not wait for the walk it has just enqueued.
bool metering(const gothic_ctx *c) {
  return c->prm.autotune || c->prm.rebuild_interval == 0;
}

int meter_prepare(gothic_ctx *c) {
  TuneState &T = c->tune;
  TreeState &R = c->tree;
  int rc;
  if (!T.ev0 && (rc = hip_check(hipEventCreate(&T.ev0), "hipEventCreate"))) return rc;
  if (!T.ev1 && (rc = hip_check(hipEventCreate(&T.ev1), "hipEventCreate"))) return rc;
  if (!R.mk0 && (rc = hip_check(hipEventCreate(&R.mk0), "hipEventCreate"))) return rc;
  if (!R.mk1 && (rc = hip_check(hipEventCreate(&R.mk1), "hipEventCreate"))) return rc;
  if (!T.ready) {
    for (auto &t : T.cls) t.init(-12.0, 0.0, 0.25, 20);
    for (auto &g : T.pick) g.init(2);
    T.ready = true;
    T.pending = -1;
  }
  return GOTHIC_OK;
}

// weight of sub-step class k among kmax + 1 classes (how often it occurs)
static double class_weight(int k, int kmax) {
  return std::ldexp(1.0, k < kmax ? -(k + 1) : -kmax);
}

int meter_collect(gothic_ctx *c, int kmax) {
  TuneState &T = c->tune;
  TreeState &R = c->tree;
  if (T.pending < 0) return GOTHIC_OK;
  const int k = T.pending;
  T.pending = -1;
  int rc;
  if ((rc = hip_check(hipEventSynchronize(T.ev1), "hipEventSynchronize"))) return rc;
  float walk = 0.f;
  if ((rc = hip_check(hipEventElapsedTime(&walk, T.ev0, T.ev1), "hipEventElapsedTime"))) return rc;
  if (T.pending_pick) {
    T.pick[k].observe((double)walk);
    if (T.pick[k].decided()) {
      T.class_G[k] = T.pick[k].current();
      T.class_W[k] = T.pick[k].current_width();
    }
  } else if (T.pending_tuned) {
    T.cls[k].observe((double)walk);
  }
  if (c->prm.rebuild_interval == 0) {
    if (T.pending_rebuilt) {
      float make = 0.f;
      if ((rc = hip_check(hipEventElapsedTime(&make, R.mk0, R.mk1), "hipEventElapsedTime")))
        return rc;
      R.models.rebuilt((double)make);
      for (bool &f : R.fresh) f = false;
    }
    // walk times of different sub-step classes (different due levels) are
    // put on one scale: relative to the class's time on a fresh tree, times
    // the mean over classes of those times
    if (!R.fresh[k]) {
      R.ref[k] = walk;
      R.have_ref[k] = true;
      R.fresh[k] = true;
    }
    double num = 0.0, den = 0.0;
    for (int j = 0; j <= kmax && j < 32; ++j)
      if (R.have_ref[j]) {
        num += class_weight(j, kmax) * R.ref[j];
        den += class_weight(j, kmax);
      }
    const double scaled = (R.ref[k] > 0.0 && den > 0.0) ? walk * (num / den) / R.ref[k] : walk;
    R.models.sample(scaled);
  }
  return GOTHIC_OK;
}

// note the evaluation just enqueued for the next collection
void meter_mark(gothic_ctx *c, int k, bool rebuilt, bool tuned, bool picked) {
  TuneState &T = c->tune;
  T.pending = k;
  T.pending_rebuilt = rebuilt;
  T.pending_tuned = tuned;
  T.pending_pick = picked;
}

// How a block sub-step's evaluation is run and metered (defaults: a plain

void mark_last(gothic_ctx *c, const Systems &sy, hipStream_t s, Buffers *lb) {
  c->last_n = sy.n;
  c->last_nsys = sy.nsys;
  c->last_stream = s;
  c->have_last = true;
  c->lb = lb;
}

int run_forces(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *active,
               const float4 *acc_old, float4 *o4, hipStream_t s, float r_crit,
               const EvalOpts &o) {
  const int64_t n = sy.n;
  c->cur_G = o.group_G > 0 ? o.group_G : c->prm.group_size;
  c->cur_W = o.walk_W > 0 ? o.walk_W : walk_width_of(c->prm);
  if (c->prm.mac == 1 && !acc_old)
    return set_error(GOTHIC_EINVAL,
                     "the acceleration MAC needs the previous accelerations (gothic_tree_forces_ex)");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const bool capturing = cap != hipStreamCaptureStatusNone;
  const int64_t want_nodes = nodes_wanted(c, n, sy.nsys);
  const bool must_grow = n > c->cap_n || sy.nsys > c->cap_sys || want_nodes > c->cap_nodes ||
                         !c->b.spill || walk_slots(c) != c->walk_waves ||
                         default_spill(c) > c->spill_per_wave ||
                         (c->prm.timing && c->ev_start.empty());
  if (capturing && must_grow) {
    c->scratch_required = ensure_bytes(c, n, sy.nsys, want_nodes, c->spill_per_wave);
    return set_error(GOTHIC_ECAPTURE, "scratch must grow to " +
                                          std::to_string(c->scratch_required) + " bytes for n = " +
                                          std::to_string(n) +
                                          "; make one uncaptured call of this size first");
  }
  int rc = ensure(c, n, sy.nsys, want_nodes, c->spill_per_wave);
  if (rc) return rc;
  if ((rc = ensure_events(c))) return rc;
  const bool meter = metering(c) && !capturing;
  if (meter && ((rc = meter_prepare(c)) || (rc = meter_collect(c, o.kmax)))) return rc;
  mark_last(c, sy, s, &c->b);
  bool rebuild = must_rebuild(c, sy);
  constexpr int kAttempts = 6;
  for (int attempt = 0; attempt < kAttempts; ++attempt) {
    c->tune.recording = meter;
    // a repeat follows flags the host has handled: they do not go sticky
    rc = enqueue_forces(c, sy, x4, active, acc_old, o4, s, r_crit, rebuild, o.sign_active,
                        attempt == 0);
    c->tune.recording = false;
    if (rc) return rc;
    tree_used(c, sy, rebuild);
    if (!c->prm.check || capturing) break;
    if ((rc = hip_check(hipMemcpyAsync(c->b.ctl_host, c->b.ctl, sizeof(Ctl),
                                       hipMemcpyDeviceToHost, s), "hipMemcpyAsync")))
      return rc;
    if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    const unsigned f = c->b.ctl_host->flags;
    if (f & kFlagNonFinite) return set_error(GOTHIC_ENONFINITE, "non-finite position or mass");
    if (f & kFlagBadIndex)
      return set_error(GOTHIC_EDEVICE, "internal index check failed (flags " + std::to_string(f) + ")");
    if (!(f & (kFlagNodeOverflow | kFlagSpillOverflow))) break;
    if (attempt == kAttempts - 1) {
      const Ctl &h = *c->b.ctl_host;
      std::string msg = "node or frontier capacity still exceeded after growing (flags " +
                        std::to_string(h.flags) + ", nodes " + std::to_string(h.n_nodes) +
                        " of " + std::to_string(c->cap_nodes) + ", groups " +
                        std::to_string(h.n_groups) + ", spill/wave " +
                        std::to_string(c->spill_per_wave) + ", level starts";
      for (int l = 0; l < kMaxLevels + 1; ++l) msg += " " + std::to_string(h.lvl_start[l]);
      c->tree.valid = false;
      return set_error(GOTHIC_EOVERFLOW, msg + ")");
    }
    // the abandoned level already knows how many nodes it needed at least
    int64_t need = 0;
    for (int l = 0; l < kMaxLevels + 1; ++l)
      if (c->b.ctl_host->lvl_start[l] != 0xffffffffu)
        need = std::max<int64_t>(need, c->b.ctl_host->lvl_start[l]);
    const int64_t nodes =
        (f & kFlagNodeOverflow) ? std::max<int64_t>(2 * c->cap_nodes, 2 * need) : c->cap_nodes;
    const int64_t spill = (f & kFlagSpillOverflow) ? 4 * c->spill_per_wave : c->spill_per_wave;
    if ((rc = ensure(c, n, sy.nsys, nodes, spill))) return rc;
    rebuild = true;  // the grown buffers hold no tree
  }
  if (meter) meter_mark(c, o.meter_class, rebuild, o.tuned, o.picked);
  return GOTHIC_OK;
}


}  // namespace gothic

using namespace gothic;

extern "C" {

int gothic_tree_forces(gothic_ctx *c, int64_t n, const float *xyzm, float eps, float theta,
                       const uint8_t *active, float *acc_pot, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (n < 0 || n >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "n must be in [0, 2^31)");
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(GOTHIC_EINVAL, "eps must be finite and > 0");
  if (!(theta >= 0.f && theta < 1.f)) return set_error(GOTHIC_EINVAL, "theta must be in [0, 1)");
  if (n == 0) return GOTHIC_OK;
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  if ((const void *)xyzm == (const void *)acc_pot)
    return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not overlap");
  DeviceGuard guard(c->device);
  const int64_t off[2] = {0, n};
  Systems sy;
  int rc = make_systems(1, off, &eps, &theta, false, &sy);
  if (rc) return rc;
  return run_forces(c, sy, reinterpret_cast<const float4 *>(xyzm), active, nullptr,
                    reinterpret_cast<float4 *>(acc_pot), reinterpret_cast<hipStream_t>(stream),
                    c->prm.r_crit);
}

int gothic_tree_forces_batched(gothic_ctx *c, int nsys, const int64_t *offsets, const float *xyzm,
                               const float *eps, const float *theta, const uint8_t *active,
                               float *acc_pot, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  Systems sy;
  int rc = make_systems(nsys, offsets, eps, theta, true, &sy);
  if (rc) return rc;
  if (sy.n == 0) return GOTHIC_OK;
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  if ((const void *)xyzm == (const void *)acc_pot)
    return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not overlap");
  DeviceGuard guard(c->device);
  return run_forces(c, sy, reinterpret_cast<const float4 *>(xyzm), active, nullptr,
                    reinterpret_cast<float4 *>(acc_pot), reinterpret_cast<hipStream_t>(stream),
                    c->prm.r_crit);
}

int gothic_tree_forces_ex(gothic_ctx *c, int nsys, const int64_t *offsets, const float *xyzm,
                          const float *eps, const float *theta, const uint8_t *active,
                          const float *acc_old, float *acc_pot, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  Systems sy;
  int rc = make_systems(nsys, offsets, eps, theta, true, &sy);
  if (rc) return rc;
  if (sy.n == 0) return GOTHIC_OK;
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  if ((const void *)xyzm == (const void *)acc_pot || (const void *)acc_old == (const void *)acc_pot)
    return set_error(GOTHIC_EINVAL, "acc_pot must not overlap xyzm or acc_old");
  DeviceGuard guard(c->device);
  return run_forces(c, sy, reinterpret_cast<const float4 *>(xyzm), active,
                    reinterpret_cast<const float4 *>(acc_old), reinterpret_cast<float4 *>(acc_pot),
                    reinterpret_cast<hipStream_t>(stream), c->prm.r_crit);
}

}  // extern "C"
