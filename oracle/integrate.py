"""Float64 oracle of the block (hierarchical) time-step integration.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 2.7 of the paper integrates block time steps with a second-order
Runge-Kutta scheme: every j-particle is predicted,
    v^{n+1/2} = v^n + dt/2 a^n,   r^{n+1} = r^n + dt v^{n+1/2},
forces are computed on the i-particles due at the new time, and those are
corrected,  v^{n+1} = v^{n+1/2} + dt/2 a^{n+1}.  With one shared fixed step
the scheme is the leap-frog.  The paper does not give the time-step criterion
nor how levels change; the readings used here (and by the library) are:

  * dt_i = eta sqrt(eps / |a_i|) (eta = 0.1);
  * steps are dt_max / 2^k, k = 0 (coarsest) .. kmax (finest); dt_fine is the
    largest power of two not above min_i dt_i at t = 0 and
    dt_max = dt_fine 2^kmax, so every level time is exact in binary;
  * a particle takes the coarsest level whose step does not exceed its dt_i
    (k = clamp(ceil(log2(dt_max / dt_i)), 0, kmax)), decided by exact
    comparisons with powers of two rather than a rounded logarithm;
  * after a correction a particle may move to any finer level, and to the
    next coarser level only when the current time is a multiple of that
    coarser step;
  * an inactive particle j is predicted to the current time t with its own
    elapsed time tau = t - t_j:  r = r_j + tau v_j + tau^2/2 a_j;
  * time is counted in finest sub-steps s (t = s dt_fine); particle i is due
    at sub-step s when s - s_i = 2^(kmax - k_i).
"""
from __future__ import annotations

import numpy as np


def level_for(dt, dt_max, kmax):
    """Coarsest level k in [0, kmax] with dt_max 2^-k <= dt (kmax if none)."""
    dt = np.asarray(dt, np.float64)
    k = np.full(dt.shape, kmax, np.int64)
    for kk in range(kmax, -1, -1):  # scan from fine to coarse, keep the coarsest fit
        fits = np.ldexp(dt_max, -kk) <= dt
        k = np.where(fits, kk, k)
    return k


def timestep(acc3, eps, eta):
    """dt_i = eta sqrt(eps/|a_i|) (infinite for a_i = 0)."""
    a = np.sqrt((np.asarray(acc3, np.float64) ** 2).sum(1))
    with np.errstate(divide="ignore"):
        return np.where(a > 0, eta * np.sqrt(eps / np.where(a > 0, a, 1.0)), np.inf)


def anchor(dt):
    """dt_fine = largest power of two <= min dt (exact, via the binary exponent)."""
    m, e = np.frexp(np.min(dt))  # min dt = m 2^e, m in [0.5, 1)
    return float(np.ldexp(1.0, int(e) - 1))


def next_level(k_old, k_want, s, kmax):
    """Finer at once; coarser by one level only on a multiple of that step."""
    k_old = np.asarray(k_old, np.int64)
    k_want = np.asarray(k_want, np.int64)
    coarser_ok = (k_old > 0) & (s % (np.int64(1) << np.maximum(kmax - k_old + 1, 0)) == 0)
    return np.where(k_want > k_old, k_want,
                    np.where((k_want < k_old) & coarser_ok, k_old - 1, k_old))


class BlockSim:
    """Block-step state in float64.  force(xyzm_f32, active_u8) -> [n,4]
    (ax, ay, az, phi) supplies the accelerations (tree or direct)."""

    def __init__(self, xyzm, vel, eps, eta, kmax, force, shared=False):
        self.x = np.asarray(xyzm[:, :3], np.float64).copy()
        self.v = np.asarray(vel, np.float64).copy()
        self.m = np.asarray(xyzm[:, 3], np.float32).copy()
        self.eps, self.eta, self.kmax, self.force, self.shared = eps, eta, kmax, force, shared
        n = self.x.shape[0]
        a = force(self._shadow(self.x), None)
        self.a = np.asarray(a[:, :3], np.float64)
        self.phi = np.asarray(a[:, 3], np.float64)
        dt = timestep(self.a, eps, eta)
        self.dt_fine = anchor(dt)
        self.dt_max = float(np.ldexp(self.dt_fine, kmax))
        self.k = np.full(n, kmax, np.int64) if shared else level_for(dt, self.dt_max, kmax)
        self.si = np.zeros(n, np.int64)  # sub-step of each particle's last update
        self.s = 0

    @classmethod
    def from_state(cls, pos, vel, acc3, mass, levels, last, s, dt_fine, eps, eta, kmax,
                   shared=False):
        """The state at the end of sub-step s, given rather than integrated:
        float64 positions and velocities at each particle's last update, the
        accelerations of that update, float32 masses, levels and last-update
        sub-steps, with the finest step dt_fine.  It predicts and selects
        (predict, due) like an integrated one; step() needs a force."""
        self = cls.__new__(cls)
        self.x = np.array(pos, np.float64)
        self.v = np.array(vel, np.float64)
        self.a = np.array(np.asarray(acc3)[:, :3], np.float64)
        self.m = np.array(mass, np.float32)
        self.phi = None
        self.eps, self.eta, self.kmax, self.force, self.shared = eps, eta, kmax, None, shared
        self.dt_fine = float(dt_fine)
        self.dt_max = float(np.ldexp(self.dt_fine, kmax))
        self.k = np.array(levels, np.int64)
        self.si = np.array(last, np.int64)
        self.s = int(s)
        return self

    def _shadow(self, pos):
        out = np.empty((pos.shape[0], 4), np.float32)
        out[:, :3] = pos
        out[:, 3] = self.m
        return out

    def due(self, s):
        return (s - self.si) == (np.int64(1) << (self.kmax - self.k))

    def predict(self, s):
        tau = ((s - self.si) * self.dt_fine)[:, None]
        return self.x + tau * self.v + 0.5 * tau * tau * self.a

    def step(self):
        """Advance one finest sub-step; returns the active mask."""
        s = self.s + 1
        act = self.due(s)
        xp = self.predict(s)
        anew = np.asarray(self.force(self._shadow(xp), act.astype(np.uint8)), np.float64)
        i = np.flatnonzero(act)
        dt = (np.ldexp(1.0, (self.kmax - self.k[i]).astype(np.int64)) * self.dt_fine)[:, None]
        self.x[i] = self.x[i] + dt * self.v[i] + 0.5 * dt * dt * self.a[i]
        self.v[i] = self.v[i] + 0.5 * dt * (self.a[i] + anew[i, :3])
        self.a[i] = anew[i, :3]
        self.phi[i] = anew[i, 3]
        self.si[i] = s
        if not self.shared:
            kw = level_for(timestep(self.a[i], self.eps, self.eta), self.dt_max, self.kmax)
            self.k[i] = next_level(self.k[i], kw, s, self.kmax)
        self.s = s
        return act

    def energy(self):
        """Kinetic + potential energy of the state at the current time (every
        particle predicted to t; potential from the last force evaluation)."""
        m = self.m.astype(np.float64)
        return 0.5 * (m * (self.v ** 2).sum(1)).sum() + 0.5 * (m * self.phi).sum()
