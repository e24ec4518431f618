// Timed search of the tunables of one workload (gothic_autotune): group
// size, walk width and list budget by exhaustive timing, then Brent's method
// on the critical separation r_crit of Section 2.4.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "api_internal.h"

namespace gothic {

static int timed_eval(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *act,
                      float4 *o4, hipStream_t s, float r_crit, double *ms) {
  TuneState &T = c->tune;
  int rc;
  if ((rc = ensure(c, sy.n, sy.nsys, nodes_wanted(c, sy.n, sy.nsys), c->spill_per_wave)))
    return rc;
  c->cur_G = c->prm.group_size;
  c->cur_W = walk_width_of(c->prm);
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
  // a candidate that overflowed is out of the race; its flags are handled here
  const bool bad = c->b.ctl_host->flags != 0u;
  *ms = bad ? HUGE_VAL : (double)t;
  if (bad) enqueue_drop_flags(c, s);
  return hip_check(hipGetLastError(), "drop_flags_k");
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
  out->walk_width = walk_width_of(c->prm);
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
    int bestG = saved.group_size, bestW = walk_width_of(saved), bestD = saved.list_depth;
    // shapes (G, W): one group per wave64, then 64 / W groups side by side
    const int Gs[8] = {8, 16, 32, 64, 4, 8, 8, 16};
    const int Ws[8] = {64, 64, 64, 64, 16, 16, 32, 32};
    const int Ds[5] = {128, 256, 384, 512, 768};
    for (int k = 0; k < 8; ++k)
      for (int D : Ds) {
        const int G = Gs[k], W = Ws[k];
        c->prm.group_size = G;
        c->prm.walk_width = W;
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
          bestW = W;
          bestD = D;
        }
      }
    c->prm.group_size = bestG;
    c->prm.walk_width = bestW;
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
    out->walk_width = bestW;
    out->list_depth = bestD;
    out->r_crit = r_wins ? rbest : saved.r_crit;
    out->ms = r_wins ? best_rt : best;
    out->evaluations = evals;
    T.cache[key] = *out;
  }
  gothic_params chosen = c->prm;
  chosen.group_size = out->group_size;
  chosen.walk_width = out->walk_width;
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


}  // namespace gothic

using namespace gothic;

extern "C" {

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

}  // extern "C"
