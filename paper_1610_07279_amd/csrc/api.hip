// C ABI of the library (declared in include/gothic.h): context and scratch
// management, argument checks, the kernel pipeline of one force evaluation,
// and read-back of intermediate results for tests.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>

#include "common.h"

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

#define GCHECK(call)                                   \
  do {                                                 \
    int _rc = hip_check((call), #call);                \
    if (_rc != GOTHIC_OK) return _rc;                  \
  } while (0)

// ---------------------------------------------------------------- helpers
// Zero the control block before an evaluation.  keep_tree keeps the tree of
// the last build (node count, level starts, systems); a tree whose build
// overflowed is not reusable and is reported as a node overflow.
__global__ void ctl_reset_k(Ctl *ctl, int keep_tree) {
  const unsigned keep_nodes = ctl->n_nodes, keep_sys = ctl->nsys, ok = ctl->tree_ok;
  unsigned lv = 0;
  if (threadIdx.x < kMaxLevels + 2) lv = ctl->lvl_start[threadIdx.x];
  __syncthreads();
  unsigned *w = reinterpret_cast<unsigned *>(ctl);
  for (unsigned i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0u;
  __syncthreads();
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

// The system table travels in kernel arguments (captured by value in a
// graph), kSysChunk systems per launch: no host staging buffer that a later
// call could overwrite before the copy runs.
constexpr int kSysChunk = 32;
constexpr int kMaxSys = 65535;  // grid y limit of the per-system kernels
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

// Debugging aid: with the environment variable GOTHIC_POISON_ALLOC set (to
// anything but "0"), every new floating-point buffer starts as all-ones bytes
// (NaN in every lane), so a kernel that reads memory no kernel of the
// evaluation wrote gives visibly wrong results instead of results that depend
// on what the memory held before.  Index buffers are left alone.
template <class T>
static constexpr bool kFloatBuffer =
    std::is_floating_point<T>::value || std::is_same<T, float4>::value ||
    std::is_same<T, float2>::value || std::is_same<T, double4>::value;

static bool poison_alloc() {
  const char *v = getenv("GOTHIC_POISON_ALLOC");
  return v && v[0] && strcmp(v, "0") != 0;
}

template <class T>
static int dev_alloc(T **p, int64_t count) {
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)count);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_check(e, "hipMalloc");
  }
  if (kFloatBuffer<T> && poison_alloc()) {
    // synchronous, so no later launch on any stream can overtake it
    if ((e = hipMemset(*p, 0xff, sizeof(T) * (size_t)count)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
      return hip_check(e, "poison fill");
  }
  return GOTHIC_OK;
}

static void free_all(gothic_ctx *c) {
  Buffers &B = c->b;
  void *ptrs[] = {B.keyA, B.keyB, B.idxA, B.idxB, B.pos, B.leaf_of, B.flag, B.flag2, B.alist,
                  B.gA, B.gB, B.gfirst,
                  B.first, B.count, B.child_first, B.parent, B.n_child, B.level, B.nch, B.bnd,
                  B.nrec, B.quad, B.ball, B.gent, B.hist, B.part, B.bbox_part, B.spill, B.sys,
                  B.soff, B.rcrit, B.mcrit, B.amag, B.gamin, B.anc, B.leaflev, B.ctl};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (B.ctl_host) (void)hipHostFree(B.ctl_host);
  B = Buffers();
  c->cap_n = c->cap_nodes = c->cap_groups = c->cap_hist = c->cap_sys = c->cap_anc = 0;
  ++c->generation;
  ++c->buffers;
}

static int validate_params(const gothic_params *p) {
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
  return GOTHIC_OK;
}

// Make sure every buffer can hold n particles (and the current node / spill
// capacities).  Never called while the stream is being captured.
static int ensure(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes, int64_t want_spill) {
  Buffers &B = c->b;
  if (!B.ctl) {
    GCHECK(hipMalloc(reinterpret_cast<void **>(&B.ctl), sizeof(Ctl)));
    GCHECK(hipHostMalloc(reinterpret_cast<void **>(&B.ctl_host), sizeof(Ctl), hipHostMallocDefault));
    int rc;
    if ((rc = dev_alloc(&B.part, scan_blocks() + 64)) != GOTHIC_OK) return rc;
    if ((rc = dev_alloc(&B.rcrit, 1)) != GOTHIC_OK) return rc;
    ++c->generation;
    ++c->buffers;
  }
  int rc;
  if (nsys > c->cap_sys) {
    const int64_t cs = std::max<int64_t>(nsys, 64);
    // bbox partials: nsys x bbox_partials(nsys, .) <= max(1024, nsys) workgroups
    if ((rc = dev_alloc(&B.sys, cs)) || (rc = dev_alloc(&B.soff, cs + 1)) ||
        (rc = dev_alloc(&B.bbox_part, 6 * std::max<int64_t>(1024, cs))))
      return rc;
    c->cap_sys = cs;
    ++c->generation;
    ++c->buffers;
  }
  if (n > c->cap_n) {
    const int64_t cn = std::max<int64_t>(n, 1024);
    if ((rc = dev_alloc(&B.keyA, cn)) || (rc = dev_alloc(&B.keyB, cn)) ||
        (rc = dev_alloc(&B.idxA, cn)) || (rc = dev_alloc(&B.idxB, cn)) ||
        (rc = dev_alloc(&B.pos, cn)) || (rc = dev_alloc(&B.leaf_of, cn)) ||
        (rc = dev_alloc(&B.flag, cn)) || (rc = dev_alloc(&B.flag2, cn)) ||
        (rc = dev_alloc(&B.alist, cn)) || (rc = dev_alloc(&B.nch, cn + 1)) ||
        (rc = dev_alloc(&B.gA, cn + 1)) || (rc = dev_alloc(&B.gB, cn + 1)) ||
        (rc = dev_alloc(&B.gfirst, cn + 1)) ||
        (rc = dev_alloc(&B.bnd, 8 * cn + 8)) || (rc = dev_alloc(&B.ball, cn)) ||
        (rc = dev_alloc(&B.gent, 2 * cn)) || (rc = dev_alloc(&B.amag, cn)) ||
        (rc = dev_alloc(&B.gamin, cn)))
      return rc;
    const int64_t hist = 2 * radix_hist_entries(cn);
    if ((rc = dev_alloc(&B.hist, hist))) return rc;
    c->cap_n = cn;
    c->cap_groups = cn;
    c->cap_hist = hist;
    ++c->generation;
    ++c->buffers;
  }
  const int64_t nodes = std::max<int64_t>(want_nodes, 64);
  if (nodes > c->cap_nodes) {
    if ((rc = dev_alloc(&B.first, nodes)) || (rc = dev_alloc(&B.count, nodes)) ||
        (rc = dev_alloc(&B.child_first, nodes)) || (rc = dev_alloc(&B.parent, nodes)) ||
        (rc = dev_alloc(&B.n_child, nodes)) || (rc = dev_alloc(&B.level, nodes)) ||
        (rc = dev_alloc(&B.nrec, 2 * nodes)) || (rc = dev_alloc(&B.quad, 2 * nodes)) ||
        (rc = dev_alloc(&B.mcrit, nodes)))
      return rc;
    c->cap_nodes = nodes;
    ++c->generation;
    ++c->buffers;
  }
  if (c->cap_anc < c->cap_n) {
    if ((rc = dev_alloc(&B.anc, (int64_t)kMaxLevels * c->cap_n)) ||
        (rc = dev_alloc(&B.leaflev, c->cap_n)))
      return rc;
    c->cap_anc = c->cap_n;
    ++c->generation;
    ++c->buffers;
  }
  const int slots = walk_slots(c);
  const int64_t spill = std::max<int64_t>(want_spill, 16384);
  if (slots != c->walk_waves || spill > c->spill_per_wave || !B.spill) {
    if ((rc = dev_alloc(&B.spill, (int64_t)slots * spill))) return rc;
    c->walk_waves = slots;
    c->spill_per_wave = spill;
    ++c->generation;
    ++c->buffers;
  }
  return GOTHIC_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// The systems of one evaluation, non-empty ones only (host side).
struct Systems {
  int nsys = 0;
  int64_t n = 0, max_n = 0;
  std::vector<int64_t> off;  // nsys + 1
  std::vector<float> eps, theta;
};

// The pipeline of one evaluation, in the pieces a captured sub-step is cut
// into:  begin (control block, r_crit; never captured), upload (system
// table), make (keys, sort, octree; skipped when the last tree is reused),
// post (permute to key order, moments, groups), walk.
static void enqueue_begin(gothic_ctx *c, bool keep_tree, float r_crit, hipStream_t s) {
  hipLaunchKernelGGL(ctl_reset_k, dim3(1), dim3(64), 0, s, c->b.ctl, keep_tree ? 1 : 0);
  hipLaunchKernelGGL(set_rcrit_k, dim3(1), dim3(64), 0, s, r_crit, c->b.rcrit);
}

static void enqueue_upload(gothic_ctx *c, const Systems &sy, hipStream_t s) {
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

static void enqueue_make(gothic_ctx *c, const Systems &sy, const float4 *xyzm, hipStream_t s) {
  launch_bbox_keys(c, xyzm, sy.n, sy.nsys, sy.max_n, s);
  launch_radix_sort(c, sy.n, sy.nsys, s);
  launch_build(c, sy.n, sy.nsys, s);
  launch_ancestors(c, sy.n, s);
}

// sign_active: the active flags are the sign bits of the masses in xyzm
// (the block-step predictor's shadow); active is then not read
static void enqueue_post(gothic_ctx *c, const Systems &sy, const float4 *xyzm,
                         const uint8_t *active, const float4 *acc_old, hipStream_t s,
                         bool sign_active = false) {
  launch_permute(c, xyzm, active, sign_active, c->prm.mac == 1 ? acc_old : nullptr, sy.n, s);
  launch_moments(c, sy.n, sy.nsys, s);
  launch_groups(c, sy.n, s);
}

static void enqueue_walk(gothic_ctx *c, int64_t n, float4 *out, hipStream_t s, bool timed) {
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
static int enqueue_forces(gothic_ctx *c, const Systems &sy, const float4 *xyzm,
                          const uint8_t *active, const float4 *acc_old, float4 *out,
                          hipStream_t s, float r_crit, bool rebuild, bool sign_active = false) {
  enqueue_begin(c, !rebuild, r_crit, s);
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
static int make_systems(int nsys, const int64_t *offsets, const float *eps, const float *theta,
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

static void free_events(gothic_ctx *c) {
  for (auto e : c->ev_start) (void)hipEventDestroy(e);
  for (auto e : c->ev_stop) (void)hipEventDestroy(e);
  c->ev_start.clear();
  c->ev_stop.clear();
  c->ev_used = 0;
}

static int ensure_events(gothic_ctx *c) {
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

static void free_graphs(gothic_ctx *c) {
  SimGraphs &G = c->graphs;
  for (auto &e : G.exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  for (auto &pair : G.exec_g)
    for (auto &e : pair)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
  G.valid = false;
}

static void free_sim(gothic_ctx *c) {
  SimState &S = c->sim;
  void *ptrs[] = {S.shadow, S.aold, S.anew, S.si, S.lev, S.act, S.soff, S.ss, S.sc};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (S.sc_host) (void)hipHostFree(S.sc_host);
  if (S.ss_host) (void)hipHostFree(S.ss_host);
  S = SimState();
  ++c->generation;
}

// The force pipeline with argument checks done: capacity, enqueue, and in
// check mode the synchronous flag check with grow-and-repeat.
static int64_t nodes_wanted(gothic_ctx *c, int64_t n, int nsys) {
  // typical trees hold ~0.25 n nodes at n_leaf = 16 and ~2-3 n at n_leaf = 1
  return std::max<int64_t>(c->cap_nodes, c->prm.node_capacity > 0
                                             ? c->prm.node_capacity
                                             : n + 8 * (n / c->prm.n_leaf) + 1024 + nsys);
}

// ---------------------------------------------------------------- tree reuse
// Does this evaluation build a new tree?  Always when there is no tree for
// these systems (or the buffers or the tree parameters changed since it was
// built); otherwise by params.rebuild_interval: 1 every time, k > 1 after k
// evaluations on one tree, 0 when the paper's growth models say so.
static bool must_rebuild(gothic_ctx *c, const Systems &sy) {
  const TreeState &T = c->tree;
  if (!T.valid || T.n != sy.n || T.off != sy.off || T.buffers != c->buffers ||
      T.n_leaf != c->prm.n_leaf || T.key_kind != c->prm.key_kind)
    return true;
  const int k = c->prm.rebuild_interval;
  if (k == 1) return true;
  if (k >= 2) return T.since >= k;
  return T.models.due();
}

static void tree_used(gothic_ctx *c, const Systems &sy, bool rebuilt) {
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
static bool metering(const gothic_ctx *c) {
  return c->prm.autotune || c->prm.rebuild_interval == 0;
}

static int meter_prepare(gothic_ctx *c) {
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

static int meter_collect(gothic_ctx *c, int kmax) {
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
    if (T.pick[k].decided()) T.class_G[k] = T.pick[k].current();
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
static void meter_mark(gothic_ctx *c, int k, bool rebuilt, bool tuned, bool picked) {
  TuneState &T = c->tune;
  T.pending = k;
  T.pending_rebuilt = rebuilt;
  T.pending_tuned = tuned;
  T.pending_pick = picked;
}

// How a block sub-step's evaluation is run and metered (defaults: a plain
// evaluation with params.group_size and the caller's active flags).
struct EvalOpts {
  int meter_class = 0;       // sub-step class the walk time is booked to
  bool tuned = false;        // r_crit came from the class's Brent search
  bool picked = false;       // the group size came from the class's picker
  int kmax = 0;              // finest level (class weights of the rebuild models)
  int group_G = 0;           // group size; 0 = params.group_size
  bool sign_active = false;  // active flags are the sign bits of the masses in x4
};

static int run_forces(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *active,
                      const float4 *acc_old, float4 *o4, hipStream_t s, float r_crit,
                      const EvalOpts &o = EvalOpts()) {
  const int64_t n = sy.n;
  c->cur_G = o.group_G > 0 ? o.group_G : c->prm.group_size;
  if (c->prm.mac == 1 && !acc_old)
    return set_error(GOTHIC_EINVAL,
                     "the acceleration MAC needs the previous accelerations (gothic_tree_forces_ex)");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const bool capturing = cap != hipStreamCaptureStatusNone;
  const int64_t want_nodes = nodes_wanted(c, n, sy.nsys);
  const bool must_grow = n > c->cap_n || sy.nsys > c->cap_sys || want_nodes > c->cap_nodes ||
                         !c->b.spill || walk_slots(c) != c->walk_waves ||
                         (c->prm.timing && c->ev_start.empty());
  if (capturing && must_grow)
    return set_error(GOTHIC_ECAPTURE, "scratch must grow for n = " + std::to_string(n) +
                                          "; make one uncaptured call of this size first");
  int rc = ensure(c, n, sy.nsys, want_nodes, c->spill_per_wave);
  if (rc) return rc;
  if ((rc = ensure_events(c))) return rc;
  const bool meter = metering(c) && !capturing;
  if (meter && ((rc = meter_prepare(c)) || (rc = meter_collect(c, o.kmax)))) return rc;
  c->last_n = n;
  c->last_nsys = sy.nsys;
  c->last_stream = s;
  c->have_last = true;
  bool rebuild = must_rebuild(c, sy);
  constexpr int kAttempts = 6;
  for (int attempt = 0; attempt < kAttempts; ++attempt) {
    c->tune.recording = meter;
    rc = enqueue_forces(c, sy, x4, active, acc_old, o4, s, r_crit, rebuild, o.sign_active);
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
  gothic_ctx *c = new gothic_ctx();
  c->device = hip_device;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  c->prm = prm;
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
      a.mac_delta != b.mac_delta || a.ball != b.ball || a.node_capacity != b.node_capacity)
    ++c->generation;
  c->prm = *p;
  return GOTHIC_OK;
}

int gothic_get_params(const gothic_ctx *c, gothic_params *p) {
  if (!c || !p) return set_error(GOTHIC_EINVAL, "NULL argument");
  *p = c->prm;
  return GOTHIC_OK;
}

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

int gothic_get_stats(gothic_ctx *c, gothic_stats *out) {
  if (!c || !out) return set_error(GOTHIC_EINVAL, "NULL argument");
  memset(out, 0, sizeof(*out));
  if (!c->have_last) return GOTHIC_OK;
  DeviceGuard guard(c->device);
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(c->b.ctl_host, c->b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                                     c->last_stream), "hipMemcpyAsync")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(c->last_stream), "hipStreamSynchronize"))) return rc;
  const Ctl &h = *c->b.ctl_host;
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
  if (h.flags & kFlagNonFinite) return set_error(GOTHIC_ENONFINITE, "non-finite position or mass");
  if (h.flags & (kFlagNodeOverflow | kFlagSpillOverflow))
    return set_error(GOTHIC_EOVERFLOW, "capacity exceeded in the last evaluation");
  if (h.flags & kFlagBadIndex) return set_error(GOTHIC_EDEVICE, "internal index check failed");
  return GOTHIC_OK;
}

static int last_counts(gothic_ctx *c, Ctl *h) {
  if (!c->have_last) return set_error(GOTHIC_EINVAL, "no evaluation yet");
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(c->b.ctl_host, c->b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                                     c->last_stream), "hipMemcpyAsync")))
    return rc;
  if ((rc = hip_check(hipStreamSynchronize(c->last_stream), "hipStreamSynchronize"))) return rc;
  *h = *c->b.ctl_host;
  return GOTHIC_OK;
}

static int d2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!dst || !bytes) return GOTHIC_OK;
  return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
}

int gothic_get_keys(gothic_ctx *c, uint64_t *keys_sorted, uint32_t *perm, double *cube) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  hipStream_t s = c->last_stream;
  const size_t n = (size_t)c->last_n;
  if ((rc = d2d(keys_sorted, c->b.keyA, n * 8, s)) || (rc = d2d(perm, c->b.idxA, n * 4, s)))
    return rc;
  if (cube) {
    hipLaunchKernelGGL(extract_cubes_k, dim3(1), dim3(256), 0, s, c->last_nsys, c->b.sys, cube);
    if ((rc = hip_check(hipGetLastError(), "extract_cubes_k"))) return rc;
  }
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}
int gothic_get_tree(gothic_ctx *c, uint32_t *first, uint32_t *count, uint32_t *child_first,
                    uint8_t *n_child, uint8_t *level) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  hipStream_t s = c->last_stream;
  const size_t nn = h.n_nodes;
  if ((rc = d2d(first, c->b.first, nn * 4, s)) || (rc = d2d(count, c->b.count, nn * 4, s)) ||
      (rc = d2d(child_first, c->b.child_first, nn * 4, s)) ||
      (rc = d2d(n_child, c->b.n_child, nn, s)) || (rc = d2d(level, c->b.level, nn, s)))
    return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_nodes(gothic_ctx *c, float *com_m, float *b, float *quad) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  hipStream_t s = c->last_stream;
  hipLaunchKernelGGL(extract_nodes_k, dim3(1024), dim3(256), 0, s, c->b.ctl, c->b.nrec, c->b.quad,
                     reinterpret_cast<float4 *>(com_m), b, quad);
  if ((rc = hip_check(hipGetLastError(), "extract_nodes_k"))) return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_get_groups(gothic_ctx *c, uint32_t *alist, uint32_t *gfirst, uint32_t *gcount,
                      float *ball, uint32_t *entries) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  DeviceGuard guard(c->device);
  Ctl h;
  int rc = last_counts(c, &h);
  if (rc) return rc;
  hipStream_t s = c->last_stream;
  if ((rc = d2d(alist, c->b.alist, (size_t)h.n_active * 4, s)) ||
      (rc = d2d(ball, c->b.ball, (size_t)h.n_groups * 16, s)) ||
      (rc = d2d(entries, c->b.gent, (size_t)h.n_groups * 8, s)))
    return rc;
  if (gfirst || gcount) {
    hipLaunchKernelGGL(extract_groups_k, dim3(256), dim3(256), 0, s, c->b.ctl, c->b.gfirst,
                       gfirst, gcount);
    if ((rc = hip_check(hipGetLastError(), "extract_groups_k"))) return rc;
  }
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
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

static int sim_bind_impl(gothic_ctx *c, const Systems &sy, double *pos, double *vel,
                         const float *mass, double eta, int kmax, int shared_step,
                         hipStream_t s) {
  if (!pos || !vel || !mass) return set_error(GOTHIC_EINVAL, "pos, vel and mass must not be NULL");
  if (!(eta > 0.0) || !std::isfinite(eta)) return set_error(GOTHIC_EINVAL, "eta must be finite and > 0");
  if (kmax < 0 || kmax > 30) return set_error(GOTHIC_EINVAL, "kmax must be in 0..30");
  SimState &S = c->sim;
  const int64_t n = sy.n;
  int rc;
  free_graphs(c);
  S.bound = false;
  if (n > S.cap || sy.nsys > S.cap_sys || !S.sc) {
    free_sim(c);
    const int cs = std::max(sy.nsys, 64);
    if ((rc = dev_alloc(&S.shadow, n)) || (rc = dev_alloc(&S.aold, n)) ||
        (rc = dev_alloc(&S.anew, n)) || (rc = dev_alloc(&S.si, n)) ||
        (rc = dev_alloc(&S.lev, n)) || (rc = dev_alloc(&S.act, n)) ||
        (rc = dev_alloc(&S.soff, cs + 1)) || (rc = dev_alloc(&S.ss, cs)) ||
        (rc = dev_alloc(&S.sc, 1)))
      return rc;
    if ((rc = hip_check(hipHostMalloc(reinterpret_cast<void **>(&S.sc_host), sizeof(SimCtl),
                                      hipHostMallocDefault), "hipHostMalloc")) ||
        (rc = hip_check(hipHostMalloc(reinterpret_cast<void **>(&S.ss_host), sizeof(SimSys) * cs,
                                      hipHostMallocDefault), "hipHostMalloc")))
      return rc;
    S.cap = n;
    S.cap_sys = cs;
  }
  S.n = n;
  S.nsys = sy.nsys;
  S.pos = pos;
  S.vel = vel;
  S.mass = mass;
  S.offsets = sy.off;
  S.eps = sy.eps;
  S.theta = sy.theta;
  S.host_s = 0;
  S.builds = 0;
  S.kmax = kmax;
  c->tune.ready = false;
  c->tune.pending = -1;
  for (int &g : c->tune.class_G) g = 0;
  {  // a new system: no tree to reuse, no growth history (the events stay)
    hipEvent_t m0 = c->tree.mk0, m1 = c->tree.mk1;
    c->tree = TreeState();
    c->tree.mk0 = m0;
    c->tree.mk1 = m1;
  }
  ++c->generation;
  // per-system clocks and offsets (the host copies stay alive until the
  // stream has synchronised)
  for (int k = 0; k < sy.nsys; ++k) {
    S.ss_host[k].dt_fine = 1.0;
    S.ss_host[k].dt_max = 1.0;
    S.ss_host[k].eps = (double)sy.eps[k];
    S.ss_host[k].min_dt_bits = ~0ull;
  }
  std::vector<uint32_t> off32(sy.off.begin(), sy.off.end());
  if ((rc = hip_check(hipMemcpyAsync(S.ss, S.ss_host, sizeof(SimSys) * sy.nsys,
                                     hipMemcpyHostToDevice, s), "hipMemcpyAsync")) ||
      (rc = hip_check(hipMemcpyAsync(S.soff, off32.data(), 4 * off32.size(),
                                     hipMemcpyHostToDevice, s), "hipMemcpyAsync")) ||
      (rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")))
    return rc;
  sim_launch_setup(c, s, eta, kmax, shared_step ? 1 : 0);
  sim_launch_reset(c, s);
  sim_launch_shadow(c, s);
  if ((rc = hip_check(hipGetLastError(), "kernel launch"))) return rc;
  // t = 0 forces on every particle (synchronous, checked; the acceleration
  // MAC has no a_old yet and uses the opening angle here)
  const gothic_params saved = c->prm;
  c->prm.check = 1;
  if (c->prm.mac == 1) c->prm.mac = 0;
  rc = run_forces(c, sy, S.shadow, nullptr, nullptr, S.anew, s, c->prm.r_crit);
  c->prm = saved;
  if (rc) return rc;
  sim_launch_init(c, s);
  sim_launch_reset(c, s);
  if ((rc = hip_check(hipGetLastError(), "kernel launch"))) return rc;
  if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
  S.bound = true;
  return GOTHIC_OK;
}

int gothic_sim_bind(gothic_ctx *c, int64_t n, double *pos, double *vel, const float *mass,
                    float eps, float theta, double eta, int kmax, int shared_step, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (n <= 0 || n >= (int64_t)1 << 31) return set_error(GOTHIC_EINVAL, "n must be in [1, 2^31)");
  const int64_t off[2] = {0, n};
  Systems sy;
  int rc = make_systems(1, off, &eps, &theta, false, &sy);
  if (rc) return rc;
  DeviceGuard guard(c->device);
  return sim_bind_impl(c, sy, pos, vel, mass, eta, kmax, shared_step,
                       reinterpret_cast<hipStream_t>(stream));
}

int gothic_sim_bind_batched(gothic_ctx *c, int nsys, const int64_t *offsets, double *pos,
                            double *vel, const float *mass, const float *eps,
                            const float *theta, double eta, int kmax, int shared_step,
                            void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  Systems sy;
  int rc = make_systems(nsys, offsets, eps, theta, false, &sy);
  if (rc) return rc;
  DeviceGuard guard(c->device);
  return sim_bind_impl(c, sy, pos, vel, mass, eta, kmax, shared_step,
                       reinterpret_cast<hipStream_t>(stream));
}

static Systems sim_systems(const SimState &S) {
  Systems sy;
  sy.nsys = S.nsys;
  sy.n = S.n;
  sy.off = S.offsets;
  sy.eps = S.eps;
  sy.theta = S.theta;
  for (int k = 0; k < S.nsys; ++k) sy.max_n = std::max(sy.max_n, S.offsets[k + 1] - S.offsets[k]);
  return sy;
}

// Capture the segments of a sub-step on the context's own stream; buffers
// are already sized by the bind.
// capture one segment of a sub-step on the context's capture stream
static int capture_segment(gothic_ctx *c, int seg, hipGraphExec_t *out) {
  SimGraphs &G = c->graphs;
  SimState &S = c->sim;
  const Systems sy = sim_systems(S);
  hipGraph_t g = nullptr;
  int rc;
  if ((rc = hip_check(hipStreamBeginCapture(G.cap_stream, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture")))
    return rc;
  switch (seg) {
    case 0:
      sim_launch_predict(c, G.cap_stream);
      enqueue_upload(c, sy, G.cap_stream);
      break;
    case 1: enqueue_make(c, sy, S.shadow, G.cap_stream); break;
    case 2: enqueue_post(c, sy, S.shadow, nullptr, S.aold, G.cap_stream, true); break;
    case 3: enqueue_walk(c, sy.n, S.anew, G.cap_stream, false); break;
    default: sim_launch_correct(c, G.cap_stream); break;
  }
  const int lrc = hip_check(hipGetLastError(), "kernel launch");
  rc = hip_check(hipStreamEndCapture(G.cap_stream, &g), "hipStreamEndCapture");
  if (lrc || rc) {
    if (g) (void)hipGraphDestroy(g);
    return lrc ? lrc : rc;
  }
  rc = hip_check(hipGraphInstantiate(out, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  (void)hipGraphDestroy(g);
  return rc;
}

// the segments that do not depend on the group size (predict, tree, correct);
// those that do are captured per group size by capture_groups
static int capture_step(gothic_ctx *c) {
  SimGraphs &G = c->graphs;
  SimState &S = c->sim;
  free_graphs(c);
  int rc;
  if (!G.cap_stream &&
      (rc = hip_check(hipStreamCreateWithFlags(&G.cap_stream, hipStreamNonBlocking),
                      "hipStreamCreateWithFlags")))
    return rc;
  const Systems sy = sim_systems(S);
  if (sy.n > c->cap_n || sy.nsys > c->cap_sys || nodes_wanted(c, sy.n, sy.nsys) > c->cap_nodes ||
      walk_slots(c) != c->walk_waves)
    return set_error(GOTHIC_ECAPTURE, "scratch is not sized for this system; bind again");
  for (int seg : {0, 1, 4}) {
    if ((rc = capture_segment(c, seg, &G.exec[seg]))) {
      free_graphs(c);
      return rc;
    }
  }
  G.generation = c->generation;
  G.valid = true;
  return GOTHIC_OK;
}

// groups + moments and walk segments for group size G = 2^lg
static int capture_groups(gothic_ctx *c, int lg) {
  SimGraphs &G = c->graphs;
  c->cur_G = 1 << lg;
  int rc;
  for (int k = 0; k < 2; ++k)
    if ((rc = capture_segment(c, 2 + k, &G.exec_g[lg][k]))) {
      free_graphs(c);
      return rc;
    }
  return GOTHIC_OK;
}

static int log2_of(int G) {
  int lg = 0;
  while ((1 << lg) < G) ++lg;
  return lg;
}

int gothic_sim_step(gothic_ctx *c, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  SimState &S = c->sim;
  if (!S.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  DeviceGuard guard(c->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TuneState &T = c->tune;
  int rc;
  // class of the coming sub-step: position of the lowest set bit of its index
  const uint64_t snext = (uint64_t)(S.host_s + 1);
  int cls = __builtin_ctzll(snext);
  if (cls > S.kmax) cls = S.kmax;
  float r_crit = c->prm.r_crit;
  // group size of the class: fixed by gothic_sim_set_group_sizes or a
  // finished pick, else (autotune = 2) the candidate being timed
  int gsize = c->prm.group_size;
  bool picking = false;
  if (c->prm.autotune && (rc = meter_prepare(c))) return rc;
  if (T.class_G[cls] > 0) {
    gsize = T.class_G[cls];
  } else if (c->prm.autotune == 2) {
    gsize = T.pick[cls].current();
    picking = true;
  }
  const bool tuning = c->prm.autotune != 0 && !picking;
  if (tuning) r_crit = -(float)std::exp2(T.cls[cls].current());
  if (c->prm.graph && !c->prm.check) {
    if ((rc = ensure_events(c))) return rc;
    if (!c->graphs.valid || c->graphs.generation != c->generation)
      if ((rc = capture_step(c))) return rc;
    const int lg = log2_of(gsize);
    if (!c->graphs.exec_g[lg][0] && (rc = capture_groups(c, lg))) return rc;
    const Systems sy = sim_systems(S);
    const bool meter = metering(c);
    if (meter && ((rc = meter_prepare(c)) || (rc = meter_collect(c, S.kmax)))) return rc;
    // the captured segments were built for these buffers: the reused tree
    // must be one they built
    const bool rebuild = must_rebuild(c, sy);
    c->last_n = S.n;
    c->last_nsys = S.nsys;
    c->last_stream = s;
    c->have_last = true;
    SimGraphs &G = c->graphs;
    enqueue_begin(c, !rebuild, r_crit, s);
    if ((rc = hip_check(hipGraphLaunch(G.exec[0], s), "hipGraphLaunch"))) return rc;
    if (rebuild) {
      if (meter) (void)hipEventRecord(c->tree.mk0, s);
      if ((rc = hip_check(hipGraphLaunch(G.exec[1], s), "hipGraphLaunch"))) return rc;
      if (meter) (void)hipEventRecord(c->tree.mk1, s);
    }
    if ((rc = hip_check(hipGraphLaunch(G.exec_g[lg][0], s), "hipGraphLaunch"))) return rc;
    const bool timed = c->prm.timing && c->ev_used < (int)c->ev_start.size();
    if (meter) (void)hipEventRecord(T.ev0, s);
    if (timed) (void)hipEventRecord(c->ev_start[c->ev_used], s);
    if ((rc = hip_check(hipGraphLaunch(G.exec_g[lg][1], s), "hipGraphLaunch"))) return rc;
    if (timed) (void)hipEventRecord(c->ev_stop[c->ev_used++], s);
    if (meter) (void)hipEventRecord(T.ev1, s);
    if ((rc = hip_check(hipGraphLaunch(G.exec[4], s), "hipGraphLaunch"))) return rc;
    tree_used(c, sy, rebuild);
    if (rebuild) ++S.builds;
    if (meter) meter_mark(c, cls, rebuild, tuning, picking);
  } else {
    sim_launch_predict(c, s);
    EvalOpts o;
    o.meter_class = cls;
    o.tuned = tuning;
    o.picked = picking;
    o.kmax = S.kmax;
    o.group_G = gsize;
    o.sign_active = true;
    rc = run_forces(c, sim_systems(S), S.shadow, nullptr, S.aold, S.anew, s, r_crit, o);
    if (rc) return rc;
    if (c->tree.since == 1) ++S.builds;
    sim_launch_correct(c, s);
    if ((rc = hip_check(hipGetLastError(), "kernel launch"))) return rc;
  }
  ++S.host_s;
  return GOTHIC_OK;
}

int gothic_sim_get_tuning(gothic_ctx *c, int nclass, float *r_crit_best, int *searches,
                          int *group_size) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  if (nclass < 0 || nclass > kTuneClasses)
    return set_error(GOTHIC_EINVAL, "nclass must be in 0..32");
  const TuneState &T = c->tune;
  for (int k = 0; k < nclass; ++k) {
    const bool have = T.ready && T.cls[k].have_best;
    if (r_crit_best) r_crit_best[k] = have ? -(float)std::exp2(T.cls[k].best) : 0.f;
    if (searches) searches[k] = T.ready ? T.cls[k].searches : 0;
    if (group_size) group_size[k] = T.class_G[k] > 0 ? T.class_G[k] : c->prm.group_size;
  }
  return GOTHIC_OK;
}

int gothic_sim_set_group_sizes(gothic_ctx *c, int nclass, const int *group_size) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  if (nclass < 0 || nclass > kTuneClasses)
    return set_error(GOTHIC_EINVAL, "nclass must be in 0..32");
  if (nclass > 0 && !group_size) return set_error(GOTHIC_EINVAL, "group_size must not be NULL");
  for (int k = 0; k < nclass; ++k) {
    const int G = group_size[k];
    if (G != 0 && (G < 1 || G > 64 || (G & (G - 1))))
      return set_error(GOTHIC_EINVAL, "group sizes must be 0 or a power of two in 1..64");
  }
  for (int k = 0; k < nclass; ++k) c->tune.class_G[k] = group_size[k];
  return GOTHIC_OK;
}

// One evaluation with the current tunables and a new tree, timed with the
// tuner's events (enqueued directly: no checks, no user timing).  Flags make
// it invalid.
static int timed_eval(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *act,
                      float4 *o4, hipStream_t s, float r_crit, double *ms) {
  TuneState &T = c->tune;
  int rc;
  if ((rc = ensure(c, sy.n, sy.nsys, nodes_wanted(c, sy.n, sy.nsys), c->spill_per_wave)))
    return rc;
  c->cur_G = c->prm.group_size;
  (void)hipEventRecord(T.ev0, s);
  if ((rc = enqueue_forces(c, sy, x4, act, nullptr, o4, s, r_crit, true))) return rc;
  (void)hipEventRecord(T.ev1, s);
  tree_used(c, sy, true);
  if ((rc = hip_check(hipMemcpyAsync(c->b.ctl_host, c->b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                                     s), "hipMemcpyAsync")) ||
      (rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")))
    return rc;
  float t = 0.f;
  if ((rc = hip_check(hipEventElapsedTime(&t, T.ev0, T.ev1), "hipEventElapsedTime"))) return rc;
  *ms = c->b.ctl_host->flags ? HUGE_VAL : (double)t;
  return GOTHIC_OK;
}

static int autotune_impl(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *act,
                         float4 *o4, hipStream_t s, gothic_tune_result *out) {
  TuneState &T = c->tune;
  int rc;
  if ((rc = meter_prepare(c))) return rc;
  T.pending = -1;  // the events are reused below
  const gothic_params saved = c->prm;
  // a checked evaluation with a new tree and the current tunables sizes the
  // scratch and counts the active particles
  c->prm.autotune = 0;
  c->prm.rebuild_interval = 1;
  rc = run_forces(c, sy, x4, act, nullptr, o4, s, saved.r_crit);
  c->prm = saved;
  if (rc) return rc;
  const int64_t na = c->b.ctl_host->n_active;
  memset(out, 0, sizeof(*out));
  out->group_size = c->prm.group_size;
  out->list_depth = c->prm.list_depth;
  out->r_crit = c->prm.r_crit;
  if (na == 0) return GOTHIC_OK;
  int lg_n = 0, lg_f = 0;
  while ((int64_t)2 << lg_n <= sy.n) ++lg_n;
  while (lg_f < 16 && ((na << (lg_f + 1)) <= sy.n)) ++lg_f;
  const auto key = std::make_tuple(sy.nsys > 1 ? 1 : 0, lg_n, lg_f, c->prm.multipole);
  auto hit = T.cache.find(key);
  if (hit != T.cache.end()) {
    *out = hit->second;
    out->evaluations = 0;
  } else {
    c->prm.check = 0;
    c->prm.timing = 0;
    int evals = 0;
    double best = HUGE_VAL;
    int bestG = saved.group_size, bestD = saved.list_depth;
    const int Gs[4] = {8, 16, 32, 64};
    const int Ds[5] = {128, 256, 384, 512, 768};
    for (int G : Gs)
      for (int D : Ds) {
        c->prm.group_size = G;
        c->prm.list_depth = D;
        double t1, t2;
        if ((rc = timed_eval(c, sy, x4, act, o4, s, saved.r_crit, &t1)) ||
            (rc = timed_eval(c, sy, x4, act, o4, s, saved.r_crit, &t2))) {
          c->prm = saved;
          return rc;
        }
        evals += 2;
        const double t = std::min(t1, t2);
        if (t < best) {
          best = t;
          bestG = G;
          bestD = D;
        }
      }
    c->prm.group_size = bestG;
    c->prm.list_depth = bestD;
    // Brent over log2(r_crit / L), the quantity the paper tunes
    BrentMin bm;
    bm.start(-12.0, 0.0, 0.25, 16);
    double best_u = 0.0, best_rt = HUGE_VAL;
    while (!bm.done()) {
      const double u = bm.ask();
      double t1, t2;
      const float r = -(float)std::exp2(u);
      if ((rc = timed_eval(c, sy, x4, act, o4, s, r, &t1)) ||
          (rc = timed_eval(c, sy, x4, act, o4, s, r, &t2))) {
        c->prm = saved;
        return rc;
      }
      evals += 2;
      const double t = std::min(t1, t2);
      if (t < best_rt) {
        best_rt = t;
        best_u = u;
      }
      bm.tell(t);
    }
    c->prm = saved;
    const float rbest = -(float)std::exp2(best_u);
    const bool r_wins = best_rt < best;
    out->group_size = bestG;
    out->list_depth = bestD;
    out->r_crit = r_wins ? rbest : saved.r_crit;
    out->ms = r_wins ? best_rt : best;
    out->evaluations = evals;
    T.cache[key] = *out;
  }
  gothic_params chosen = c->prm;
  chosen.group_size = out->group_size;
  chosen.list_depth = out->list_depth;
  chosen.r_crit = out->r_crit;
  if ((rc = gothic_set_params(c, &chosen))) return rc;
  // the caller's forces, with the chosen tunables, a new tree and the usual checks
  c->prm.check = 1;
  c->prm.autotune = 0;
  c->prm.rebuild_interval = 1;
  rc = run_forces(c, sy, x4, act, nullptr, o4, s, c->prm.r_crit);
  c->prm.check = chosen.check;
  c->prm.autotune = chosen.autotune;
  c->prm.rebuild_interval = chosen.rebuild_interval;
  return rc;
}

int gothic_autotune(gothic_ctx *c, int nsys, const int64_t *offsets, const float *xyzm,
                    const float *eps, const float *theta, const uint8_t *active,
                    float *acc_pot, gothic_tune_result *out, void *stream) {
  if (!c || !out) return set_error(GOTHIC_EINVAL, "NULL argument");
  Systems sy;
  int rc = make_systems(nsys, offsets, eps, theta, true, &sy);
  if (rc) return rc;
  if (sy.n == 0) return set_error(GOTHIC_EINVAL, "no particles to tune on");
  if (!xyzm || !acc_pot) return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not be NULL");
  if ((const void *)xyzm == (const void *)acc_pot)
    return set_error(GOTHIC_EINVAL, "xyzm and acc_pot must not overlap");
  DeviceGuard guard(c->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (cap != hipStreamCaptureStatusNone)
    return set_error(GOTHIC_ECAPTURE, "gothic_autotune times evaluations and cannot be captured");
  return autotune_impl(c, sy, reinterpret_cast<const float4 *>(xyzm), active,
                       reinterpret_cast<float4 *>(acc_pot), s, out);
}

int gothic_sim_reset_counters(gothic_ctx *c, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (!c->sim.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  DeviceGuard guard(c->device);
  sim_launch_reset(c, reinterpret_cast<hipStream_t>(stream));
  c->sim.builds = 0;
  return hip_check(hipGetLastError(), "kernel launch");
}

static int sim_fetch(gothic_ctx *c) {
  SimState &S = c->sim;
  hipStream_t s = c->last_stream;
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(S.sc_host, S.sc, sizeof(SimCtl), hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync")) ||
      (rc = hip_check(hipMemcpyAsync(S.ss_host, S.ss, sizeof(SimSys) * S.nsys,
                                     hipMemcpyDeviceToHost, s), "hipMemcpyAsync")))
    return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int gothic_sim_get_info(gothic_ctx *c, gothic_sim_info *out) {
  if (!c || !out) return set_error(GOTHIC_EINVAL, "NULL argument");
  SimState &S = c->sim;
  if (!S.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  DeviceGuard guard(c->device);
  sim_launch_hist(c, c->last_stream);
  int rc = sim_fetch(c);
  if (rc) return rc;
  const SimCtl &h = *S.sc_host;
  memset(out, 0, sizeof(*out));
  out->n = S.n;
  out->substep = h.s;
  out->dt_fine = S.ss_host[0].dt_fine;
  out->dt_max = S.ss_host[0].dt_max;
  out->t = (double)h.s * S.ss_host[0].dt_fine;
  out->steps = (int64_t)h.steps;
  out->last_active = (int64_t)h.last_active;
  out->active_total = (int64_t)h.active_total;
  out->interactions_total = (int64_t)h.inter_total;
  out->node_interactions_total = (int64_t)h.node_inter_total;
  out->tree_builds = S.builds;
  for (int k = 0; k < 32; ++k) out->level_count[k] = (int64_t)h.level_count[k];
  return GOTHIC_OK;
}

int gothic_sim_get_steps(gothic_ctx *c, int nsys, double *dt_fine, double *dt_max) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  SimState &S = c->sim;
  if (!S.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  if (nsys != S.nsys) return set_error(GOTHIC_EINVAL, "nsys differs from the bound systems");
  DeviceGuard guard(c->device);
  int rc = sim_fetch(c);
  if (rc) return rc;
  for (int k = 0; k < nsys; ++k) {
    if (dt_fine) dt_fine[k] = S.ss_host[k].dt_fine;
    if (dt_max) dt_max[k] = S.ss_host[k].dt_max;
  }
  return GOTHIC_OK;
}

int gothic_sim_get_state(gothic_ctx *c, float *acc_pot, uint8_t *levels, int64_t *last) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  SimState &S = c->sim;
  if (!S.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  DeviceGuard guard(c->device);
  hipStream_t s = c->last_stream;
  int rc;
  if ((rc = d2d(acc_pot, S.aold, (size_t)S.n * 16, s)) || (rc = d2d(levels, S.lev, (size_t)S.n, s)) ||
      (rc = d2d(last, S.si, (size_t)S.n * 8, s)))
    return rc;
  return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // extern "C"
