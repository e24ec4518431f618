// C ABI of the block-step driver (Section 2.7): binding of the float64
// state, one finest sub-step per call (launched, or replayed as captured HIP
// graphs), counters and state read-back, and the per-class group sizes.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "api_internal.h"

namespace gothic {

static int d2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!dst || !bytes) return GOTHIC_OK;
  return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
}

void free_graphs(gothic_ctx *c) {
  SimGraphs &G = c->graphs;
  for (auto &e : G.exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  for (auto &width : G.exec_g)
    for (auto &pair : width)
      for (auto &e : pair)
        if (e) {
          (void)hipGraphExecDestroy(e);
          e = nullptr;
        }
  G.valid = false;
}

void free_sim(gothic_ctx *c) {
  SimState &S = c->sim;
  void *ptrs[] = {S.shadow, S.aold, S.anew, S.si, S.lev, S.act, S.soff, S.ss, S.sc};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (S.sc_host) (void)hipHostFree(S.sc_host);
  if (S.ss_host) (void)hipHostFree(S.ss_host);
  S = SimState();
  ++c->generation;
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
  for (int &w : c->tune.class_W) w = 0;
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
  sim_launch_reset(c, s, true);
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
  sim_launch_reset(c, s, true);
  sim_launch_predict(c, s);  // the first sub-step; later ones are predicted by the corrector
  if ((rc = hip_check(hipGetLastError(), "kernel launch"))) return rc;
  if ((rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
  S.bound = true;
  return GOTHIC_OK;
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
    case 0: enqueue_upload(c, sy, G.cap_stream); break;
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

// the segments that do not depend on the group shape (system table, tree,
// correct + predict); those that do are captured per shape by capture_groups
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

// groups + moments and walk segments for group size G = 2^lg and walk width
// W = 16 << lw
static int capture_groups(gothic_ctx *c, int lw, int lg) {
  SimGraphs &G = c->graphs;
  c->cur_G = 1 << lg;
  c->cur_W = 16 << lw;
  int rc;
  for (int k = 0; k < 2; ++k)
    if ((rc = capture_segment(c, 2 + k, &G.exec_g[lw][lg][k]))) {
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

}  // namespace gothic

using namespace gothic;

extern "C" {

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
  // group shape of the class: fixed by gothic_sim_set_group_sizes or a
  // finished pick, else (autotune = 2) the candidate being timed
  int gsize = c->prm.group_size, wsize = walk_width_of(c->prm);
  bool picking = false;
  if (c->prm.autotune && (rc = meter_prepare(c))) return rc;
  if (T.class_G[cls] > 0) {
    gsize = T.class_G[cls];
    wsize = T.class_W[cls] > 0 ? T.class_W[cls] : 64;
  } else if (c->prm.autotune == 2) {
    gsize = T.pick[cls].current();
    wsize = T.pick[cls].current_width();
    picking = true;
  }
  const bool tuning = c->prm.autotune != 0 && !picking;
  if (tuning) r_crit = -(float)std::exp2(T.cls[cls].current());
  if (c->prm.graph && !c->prm.check) {
    if ((rc = ensure_events(c))) return rc;
    if (!c->graphs.valid || c->graphs.generation != c->generation)
      if ((rc = capture_step(c))) return rc;
    const int lg = log2_of(gsize), lw = log2_of(wsize) - 4;
    if (!c->graphs.exec_g[lw][lg][0] && (rc = capture_groups(c, lw, lg))) return rc;
    // the shape of this evaluation for read-backs that walk again
    // (gothic_get_lists): a replay does not pass through capture_groups
    c->cur_G = 1 << lg;
    c->cur_W = 16 << lw;
    const Systems sy = sim_systems(S);
    const bool meter = metering(c);
    if (meter && ((rc = meter_prepare(c)) || (rc = meter_collect(c, S.kmax)))) return rc;
    // the captured segments were built for these buffers: the reused tree
    // must be one they built
    const bool rebuild = must_rebuild(c, sy);
    mark_last(c, sy, s, &c->b);
    SimGraphs &G = c->graphs;
    enqueue_begin(c, !rebuild, r_crit, s);
    if ((rc = hip_check(hipGraphLaunch(G.exec[0], s), "hipGraphLaunch"))) return rc;
    if (rebuild) {
      if (meter) (void)hipEventRecord(c->tree.mk0, s);
      if ((rc = hip_check(hipGraphLaunch(G.exec[1], s), "hipGraphLaunch"))) return rc;
      if (meter) (void)hipEventRecord(c->tree.mk1, s);
    }
    if ((rc = hip_check(hipGraphLaunch(G.exec_g[lw][lg][0], s), "hipGraphLaunch"))) return rc;
    const bool timed = c->prm.timing && c->ev_used < (int)c->ev_start.size();
    if (meter) (void)hipEventRecord(T.ev0, s);
    if (timed) (void)hipEventRecord(c->ev_start[c->ev_used], s);
    if ((rc = hip_check(hipGraphLaunch(G.exec_g[lw][lg][1], s), "hipGraphLaunch"))) return rc;
    if (timed) (void)hipEventRecord(c->ev_stop[c->ev_used++], s);
    if (meter) (void)hipEventRecord(T.ev1, s);
    if ((rc = hip_check(hipGraphLaunch(G.exec[4], s), "hipGraphLaunch"))) return rc;
    tree_used(c, sy, rebuild);
    if (rebuild) ++S.builds;
    if (meter) meter_mark(c, cls, rebuild, tuning, picking);
  } else {
    EvalOpts o;
    o.meter_class = cls;
    o.tuned = tuning;
    o.picked = picking;
    o.kmax = S.kmax;
    o.group_G = gsize;
    o.walk_W = wsize;
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
                          int *group_size, int *walk_width) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  if (nclass < 0 || nclass > kTuneClasses)
    return set_error(GOTHIC_EINVAL, "nclass must be in 0..32");
  const TuneState &T = c->tune;
  for (int k = 0; k < nclass; ++k) {
    const bool have = T.ready && T.cls[k].have_best;
    if (r_crit_best) r_crit_best[k] = have ? -(float)std::exp2(T.cls[k].best) : 0.f;
    if (searches) searches[k] = T.ready ? T.cls[k].searches : 0;
    if (group_size) group_size[k] = T.class_G[k] > 0 ? T.class_G[k] : c->prm.group_size;
    if (walk_width)
      walk_width[k] = T.class_G[k] > 0 ? (T.class_W[k] > 0 ? T.class_W[k] : 64)
                                       : walk_width_of(c->prm);
  }
  return GOTHIC_OK;
}

int gothic_sim_set_group_sizes(gothic_ctx *c, int nclass, const int *group_size,
                               const int *walk_width) {
  if (!c) return set_error(GOTHIC_EINVAL, "NULL argument");
  if (nclass < 0 || nclass > kTuneClasses)
    return set_error(GOTHIC_EINVAL, "nclass must be in 0..32");
  if (nclass > 0 && !group_size) return set_error(GOTHIC_EINVAL, "group_size must not be NULL");
  for (int k = 0; k < nclass; ++k) {
    const int G = group_size[k];
    const int W = walk_width ? walk_width[k] : 64;
    if (G != 0 && (G < 1 || G > 64 || (G & (G - 1))))
      return set_error(GOTHIC_EINVAL, "group sizes must be 0 or a power of two in 1..64");
    if (W != 0 && W != 16 && W != 32 && W != 64)
      return set_error(GOTHIC_EINVAL, "walk widths must be 0, 16, 32 or 64");
    if (G > (W ? W : 64)) return set_error(GOTHIC_EINVAL, "a group size exceeds its walk width");
  }
  for (int k = 0; k < nclass; ++k) {
    c->tune.class_G[k] = group_size[k];
    c->tune.class_W[k] = walk_width ? walk_width[k] : 64;
  }
  return GOTHIC_OK;
}

int gothic_sim_reset_counters(gothic_ctx *c, void *stream) {
  if (!c) return set_error(GOTHIC_EINVAL, "context is NULL");
  if (!c->sim.bound) return set_error(GOTHIC_EINVAL, "no system bound (gothic_sim_bind)");
  DeviceGuard guard(c->device);
  sim_launch_reset(c, reinterpret_cast<hipStream_t>(stream), false);
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
