// Block (hierarchical) time steps, Section 2.7 of the paper, in float64.
//
// All j-particles are predicted to the current time, the due i-particles get
// tree forces, and they are corrected with the second-order Runge-Kutta
// scheme of the paper:
//   predictor  r = r_j + tau v_j + tau^2/2 a_j          (tau = t - t_j)
//   corrector  r_i += dt v_i + dt^2/2 a_i^old,  v_i += dt/2 (a_i^old + a_i^new)
// With one shared fixed step this is the leap-frog.  The paper gives neither
// the time-step criterion nor the level rules; the readings used here:
//   dt_i = eta sqrt(eps / |a_i|); steps dt_max / 2^k, k = 0..kmax; dt_fine =
//   largest power of two <= min_i dt_i at t = 0, dt_max = dt_fine 2^kmax; a
//   particle takes the coarsest level whose step fits its dt_i (exact
//   comparisons with powers of two); after a correction it may move to any
//   finer level, and one level coarser only when the current sub-step is a
//   multiple of that coarser step.  Time is counted in finest sub-steps s
//   (t = s dt_fine); particle i is due at s when s - s_i = 2^(kmax - k_i).
// The sub-step counter and every count live on the device, so a step needs
// no host round-trip.  The correction of sub-step s and the prediction of
// s + 1 are one pass over the float64 state; the prediction of the first
// sub-step is made when the system is bound.  Several independent systems can be stepped together:
// each has its own dt_fine / dt_max (from its own minimum step) and the
// shared counter s counts every system's own finest sub-steps.
#include "common.h"
#include "primitives.h"

namespace gothic {

__device__ __forceinline__ int level_for(double dt, double dt_max, int kmax) {
  int k = kmax;
  for (int kk = kmax; kk >= 0; --kk)
    if (ldexp(dt_max, -kk) <= dt) k = kk;
  return k;
}

// One coordinate of the predictor, r + tau v + h a with h = tau^2 / 2, rounded
// operation by operation in the written order (no fused multiply-adds), so the
// float32 shadow is the rounding of the value the formula gives in plain
// float64 arithmetic.
__device__ __forceinline__ double predict_coord(double r, double v, double a, double tau,
                                                double h) {
#pragma clang fp contract(off)
  return r + tau * v + h * a;
}

__device__ __forceinline__ double step_of(float4 a, double eps, double eta) {
  const double ax = a.x, ay = a.y, az = a.z;
  const double am = sqrt(ax * ax + ay * ay + az * az);
  return am > 0.0 ? eta * sqrt(eps / am) : HUGE_VAL;
}

__global__ void __launch_bounds__(256)
sim_shadow_k(int64_t n, const double *__restrict__ pos, const float *__restrict__ mass,
             float4 *__restrict__ shadow) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    shadow[i] = make_float4((float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2],
                            mass[i]);
}

// Every kernel below is wave-uniform in its loop control: waves step over
// 64-particle tiles, so the cross-lane reductions never sit under a
// lane-dependent loop condition.  A particle's system (for its clock and
// softening) is found from the offsets; most tiles lie inside one system.

// t = 0: store a as a_old, find each system's min dt (positive doubles order
// like their bits)
__global__ void __launch_bounds__(256)
sim_init_k(int64_t n, unsigned nsys, const uint32_t *__restrict__ soff,
           const float4 *__restrict__ acc, float4 *__restrict__ aold, int64_t *__restrict__ si,
           SimSys *ss, const SimCtl *__restrict__ sc) {
  const double eta = sc->eta;
  const int lane = lane_id();
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = w0 * 64; base < n; base += nw * 64) {
    const int64_t i = base + lane;
    const bool ok = i < n;
    unsigned long long b = ~0ull;
    unsigned sy = 0;
    if (ok) {
      sy = sys_of(soff, nsys, (uint32_t)i);
      const float4 a = acc[i];
      aold[i] = a;
      si[i] = 0;
      b = __double_as_longlong(step_of(a, ss[sy].eps, eta));
    }
    const unsigned s0 = __builtin_amdgcn_readfirstlane(sy);
    if (__ballot(ok && sy != s0) == 0ull) {  // one system in this tile
      for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(b, d, 64);
        b = o < b ? o : b;
      }
      if (lane == 0) atomicMin(&ss[s0].min_dt_bits, b);
    } else if (ok) {
      atomicMin(&ss[sy].min_dt_bits, b);
    }
  }
}

// dt_fine = largest power of two <= min dt of the system, dt_max = dt_fine 2^kmax
__global__ void sim_anchor_k(unsigned nsys, SimSys *ss, SimCtl *sc) {
  for (unsigned k = threadIdx.x; k < nsys; k += blockDim.x) {
    const double m = __longlong_as_double((long long)ss[k].min_dt_bits);
    int e = 0;
    double dtf = 1.0;
    if (m > 0.0 && m < HUGE_VAL) {
      (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
      dtf = ldexp(1.0, e - 1);
    }
    ss[k].dt_fine = dtf;
    ss[k].dt_max = ldexp(dtf, sc->kmax);
  }
  if (threadIdx.x == 0) sc->s = 0;
}

__global__ void __launch_bounds__(256)
sim_levels_k(int64_t n, unsigned nsys, const uint32_t *__restrict__ soff,
             const float4 *__restrict__ aold, uint8_t *__restrict__ lev,
             const SimSys *__restrict__ ss, const SimCtl *__restrict__ sc) {
  const double eta = sc->eta;
  const int kmax = sc->kmax, shared = sc->shared;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const SimSys &r = ss[sys_of(soff, nsys, (uint32_t)i)];
    lev[i] = (uint8_t)(shared ? kmax : level_for(step_of(aold[i], r.eps, eta), r.dt_max, kmax));
  }
}

// sub-step s+1: predict everybody into the float32 shadow, flag the due ones
__global__ void __launch_bounds__(256)
sim_predict_k(int64_t n, unsigned nsys, const uint32_t *__restrict__ soff,
              const double *__restrict__ pos, const double *__restrict__ vel,
              const float *__restrict__ mass, const float4 *__restrict__ aold,
              const int64_t *__restrict__ si, const uint8_t *__restrict__ lev,
              float4 *__restrict__ shadow, uint8_t *__restrict__ act,
              const SimSys *__restrict__ ss, SimCtl *sc) {
  const int64_t s = sc->s + 1;
  const int kmax = sc->kmax;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  unsigned cnt = 0;
  for (int64_t base = w0 * 64; base < n; base += nw * 64) {
    const int64_t i = base + lane_id();
    if (i < n) {
      const double dtf = ss[sys_of(soff, nsys, (uint32_t)i)].dt_fine;
      const int64_t el = s - si[i];
      const double tau = (double)el * dtf;
      const float4 a = aold[i];
      const double h = 0.5 * tau * tau;
      const double x = predict_coord(pos[3 * i], vel[3 * i], (double)a.x, tau, h);
      const double y = predict_coord(pos[3 * i + 1], vel[3 * i + 1], (double)a.y, tau, h);
      const double z = predict_coord(pos[3 * i + 2], vel[3 * i + 2], (double)a.z, tau, h);
      const bool due = el == ((int64_t)1 << (kmax - lev[i]));
      // the sign of the (non-negative) mass carries the due flag to the
      // key-order gather, which then reads one array instead of two
      const float m = mass[i];
      shadow[i] = make_float4((float)x, (float)y, (float)z, due ? -m : m);
      act[i] = due ? 1 : 0;
      cnt += due ? 1u : 0u;
    }
  }
  // one atomic per workgroup instead of one per wave: every count lands on
  // the same counter, and same-address atomics serialise
  __shared__ unsigned wcnt[4];
  cnt = wave_sum(cnt);
  if (lane_id() == 0) wcnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (t) atomicAdd(&sc->n_active, (unsigned long long)t);
  }
}

// End of sub-step s and start of s+1 in one pass over the float64 state: the
// particles due at s are corrected (and take new levels), then every
// particle is predicted to s+1 into the float32 shadow with its due flag.
// The same arithmetic as a correction pass followed by a prediction pass,
// with the state read once.
__global__ void __launch_bounds__(256)
sim_correct_predict_k(int64_t n, unsigned nsys, const uint32_t *__restrict__ soff,
                      double *__restrict__ pos, double *__restrict__ vel,
                      const float *__restrict__ mass, const float4 *__restrict__ anew,
                      float4 *__restrict__ aold, int64_t *__restrict__ si,
                      uint8_t *__restrict__ lev, float4 *__restrict__ shadow,
                      uint8_t *__restrict__ act, const SimSys *__restrict__ ss, SimCtl *sc) {
  const int64_t s = sc->s + 1;  // the sub-step being finished
  const double eta = sc->eta;
  const int kmax = sc->kmax, shared = sc->shared;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  unsigned cnt = 0;
  for (int64_t base = w0 * 64; base < n; base += nw * 64) {
    const int64_t i = base + lane_id();
    if (i < n) {
      const SimSys &r = ss[sys_of(soff, nsys, (uint32_t)i)];
      double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
      double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
      float4 a = aold[i];
      int64_t last = si[i];
      int k = lev[i];
      if (act[i]) {
        const double dt = ldexp(r.dt_fine, kmax - k);
        const float4 an = anew[i];
        const double h = 0.5 * dt * dt;
        x += dt * vx + h * (double)a.x;
        y += dt * vy + h * (double)a.y;
        z += dt * vz + h * (double)a.z;
        vx += 0.5 * dt * ((double)a.x + (double)an.x);
        vy += 0.5 * dt * ((double)a.y + (double)an.y);
        vz += 0.5 * dt * ((double)a.z + (double)an.z);
        pos[3 * i] = x; pos[3 * i + 1] = y; pos[3 * i + 2] = z;
        vel[3 * i] = vx; vel[3 * i + 1] = vy; vel[3 * i + 2] = vz;
        a = an;
        aold[i] = an;
        last = s;
        si[i] = s;
        if (!shared) {
          const int kw = level_for(step_of(an, r.eps, eta), r.dt_max, kmax);
          int kn = k;
          if (kw > k) {
            kn = kw;
          } else if (kw < k && k > 0) {
            const int64_t coarse = (int64_t)1 << (kmax - k + 1);
            if (s % coarse == 0) kn = k - 1;
          }
          k = kn;
          lev[i] = (uint8_t)kn;
        }
      }
      // prediction to s + 1
      const int64_t el = s + 1 - last;
      const double tau = (double)el * r.dt_fine;
      const double h = 0.5 * tau * tau;
      const double px = predict_coord(x, vx, (double)a.x, tau, h);
      const double py = predict_coord(y, vy, (double)a.y, tau, h);
      const double pz = predict_coord(z, vz, (double)a.z, tau, h);
      const bool due = el == ((int64_t)1 << (kmax - k));
      const float m = mass[i];
      shadow[i] = make_float4((float)px, (float)py, (float)pz, due ? -m : m);
      act[i] = due ? 1 : 0;
      cnt += due ? 1u : 0u;
    }
  }
  __shared__ unsigned wcnt[4];
  cnt = wave_sum(cnt);
  if (lane_id() == 0) wcnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (t) atomicAdd(&sc->n_next, (unsigned long long)t);
  }
}

__global__ void sim_advance_k(SimCtl *sc, const Ctl *ctl) {
  if (threadIdx.x == 0) {
    sc->s += 1;
    sc->steps += 1;
    sc->inter_total += ctl->interactions;
    sc->node_inter_total += ctl->node_interactions;
    sc->active_total += sc->n_active;
    sc->last_active = sc->n_active;
    sc->n_active = sc->n_next;  // the next step was predicted with this one's correction
    sc->n_next = 0;
  }
}

__global__ void sim_setup_k(SimCtl *sc, double eta, int kmax, int shared) {
  if (threadIdx.x == 0) {
    sc->eta = eta;
    sc->kmax = kmax;
    sc->shared = shared;
    sc->s = 0;
  }
}

// all = 1 (a new binding): also the due counts of the predicted step
__global__ void sim_reset_k(SimCtl *sc, int all) {
  if (threadIdx.x == 0) {
    if (all) {
      sc->n_active = 0;
      sc->n_next = 0;
    }
    sc->steps = 0;
    sc->inter_total = 0;
    sc->node_inter_total = 0;
    sc->active_total = 0;
    sc->last_active = 0;
  }
}

__global__ void __launch_bounds__(256)
sim_hist_k(int64_t n, const uint8_t *__restrict__ lev, SimCtl *sc) {
  __shared__ unsigned h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[lev[i] & 31], 1u);
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x])
    atomicAdd(&sc->level_count[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void sim_hist_clear_k(SimCtl *sc) {
  if (threadIdx.x < 32) sc->level_count[threadIdx.x] = 0;
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

void sim_launch_setup(gothic_ctx *c, hipStream_t s, double eta, int kmax, int shared) {
  hipLaunchKernelGGL(sim_setup_k, dim3(1), dim3(64), 0, s, c->sim.sc, eta, kmax, shared);
}

void sim_launch_reset(gothic_ctx *c, hipStream_t s, bool all) {
  hipLaunchKernelGGL(sim_reset_k, dim3(1), dim3(64), 0, s, c->sim.sc, all ? 1 : 0);
}

void sim_launch_shadow(gothic_ctx *c, hipStream_t s) {
  SimState &S = c->sim;
  hipLaunchKernelGGL(sim_shadow_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n, S.pos, S.mass,
                     S.shadow);
}

void sim_launch_init(gothic_ctx *c, hipStream_t s) {
  SimState &S = c->sim;
  const unsigned ns = (unsigned)S.nsys;
  hipLaunchKernelGGL(sim_init_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n, ns, S.soff, S.anew,
                     S.aold, S.si, S.ss, S.sc);
  hipLaunchKernelGGL(sim_anchor_k, dim3(1), dim3(256), 0, s, ns, S.ss, S.sc);
  hipLaunchKernelGGL(sim_levels_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n, ns, S.soff, S.aold,
                     S.lev, S.ss, S.sc);
}

void sim_launch_predict(gothic_ctx *c, hipStream_t s) {
  SimState &S = c->sim;
  hipLaunchKernelGGL(sim_predict_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n, (unsigned)S.nsys,
                     S.soff, S.pos, S.vel, S.mass, S.aold, S.si, S.lev, S.shadow, S.act, S.ss,
                     S.sc);
}

// the end of a sub-step: correct the due particles and predict the next
// sub-step, then advance the clock
void sim_launch_correct(gothic_ctx *c, hipStream_t s) {
  SimState &S = c->sim;
  hipLaunchKernelGGL(sim_correct_predict_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n,
                     (unsigned)S.nsys, S.soff, S.pos, S.vel, S.mass, S.anew, S.aold, S.si, S.lev,
                     S.shadow, S.act, S.ss, S.sc);
  hipLaunchKernelGGL(sim_advance_k, dim3(1), dim3(64), 0, s, S.sc, c->b.ctl);
}

void sim_launch_hist(gothic_ctx *c, hipStream_t s) {
  SimState &S = c->sim;
  hipLaunchKernelGGL(sim_hist_clear_k, dim3(1), dim3(64), 0, s, S.sc);
  hipLaunchKernelGGL(sim_hist_k, dim3(grid_for(S.n)), dim3(256), 0, s, S.n, S.lev, S.sc);
}

}  // namespace gothic
