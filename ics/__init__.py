"""Seeded synthetic initial conditions (inputs only; none of the tree method).

The paper draws its particle distributions from an external generator that is
not available here (Section 3.1 names NFW, Plummer, King and Hernquist spheres
and an M31-like three-component galaxy).  These generators stand in for them:
same profiles, equal-mass particles, positions drawn in float64 from the
analytic enclosed-mass distributions, stored as float32 ``xyzm`` rows
(x, y, z, m).  Every array is a pure function of its seed.

Both the oracle-side tests and the GPU-side tests, benchmark and smoke run use
this module; it contains only sampling code (no keys, trees, forces).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "plummer", "nfw", "galaxy", "batched_systems", "random_active",
    "Config", "CONFIGS", "config_system",
]


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Place radii r on random isotropic directions: cos(theta)~U[-1,1], phi~U[0,2pi)."""
    ct = rng.uniform(-1.0, 1.0, r.size)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = rng.uniform(0.0, 2.0 * np.pi, r.size)
    return np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)


def _pack(pos: np.ndarray, m: np.ndarray) -> np.ndarray:
    out = np.empty((pos.shape[0], 4), dtype=np.float32)
    out[:, :3] = pos.astype(np.float32)
    out[:, 3] = m.astype(np.float32)
    return out


def _jeans_sigma_r(r_grid, rho, menc):
    """Isotropic Jeans dispersion sigma_r^2(r) = (1/rho) int_r^rt rho M / r'^2 dr' (G=1)."""
    f = rho * menc / r_grid ** 2
    # cumulative trapezoid from the outer edge inwards
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(r_grid)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    with np.errstate(divide="ignore", invalid="ignore"):
        s2 = np.where(rho > 0, tail / rho, 0.0)
    return np.sqrt(np.maximum(s2, 0.0))


# --------------------------------------------------------------------------
# Plummer sphere (G = M = a = 1), truncated at r_max
# --------------------------------------------------------------------------
def plummer(n: int, seed: int = 101, r_max: float = 20.0, with_vel: bool = False):
    """Truncated Plummer sphere; returns xyzm float32 [n,4] (and float64 vel [n,3]).

    Enclosed mass M(<r) = r^3/(1+r^2)^{3/2}, renormalised to 1 inside r_max and
    inverted in closed form.  Velocities: the Aarseth-Henon-Wielen rejection on
    g(q) = q^2 (1-q^2)^{7/2} with v = q sqrt(2) (1+r^2)^{-1/4}.
    """
    rng = np.random.default_rng(seed)
    mt = r_max ** 3 / (1.0 + r_max ** 2) ** 1.5
    u = rng.uniform(0.0, 1.0, n) * mt
    u = np.clip(u, 1e-300, None)
    r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, r)
    xyzm = _pack(pos, np.full(n, 1.0 / n))
    if not with_vel:
        return xyzm
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.uniform(0.0, 1.0, todo.size)
        x2 = rng.uniform(0.0, 0.1, todo.size)
        ok = x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    v = q * np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = _isotropic(rng, v)
    return xyzm, vel


# --------------------------------------------------------------------------
# NFW sphere (r_s = 1, concentration c, truncated at c r_s, total mass 1)
# --------------------------------------------------------------------------
def _mu(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw(n: int, seed: int = 201, c: float = 10.0, with_vel: bool = False):
    """Truncated NFW sphere; xyzm float32 [n,4] (and float64 vel [n,3]).

    Radius by solving mu(r) = u mu(c), mu(x) = ln(1+x) - x/(1+x), with 60 steps
    of bisection in float64.  Velocities: Gaussian per component with the
    isotropic Jeans dispersion of the truncated profile.
    """
    rng = np.random.default_rng(seed)
    target = rng.uniform(0.0, 1.0, n) * _mu(c)
    lo = np.zeros(n)
    hi = np.full(n, c)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = _mu(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    r = 0.5 * (lo + hi)
    pos = _isotropic(rng, r)
    xyzm = _pack(pos, np.full(n, 1.0 / n))
    if not with_vel:
        return xyzm
    grid = np.geomspace(1e-4, c, 4096)
    rho = 1.0 / (grid * (1.0 + grid) ** 2) / (4.0 * np.pi * _mu(c))
    menc = _mu(grid) / _mu(c)
    sig = np.interp(r, grid, _jeans_sigma_r(grid, rho, menc))
    vel = rng.normal(0.0, 1.0, (n, 3)) * sig[:, None]
    return xyzm, vel


# --------------------------------------------------------------------------
# M31-like galaxy stand-in: NFW halo + Hernquist bulge + exponential disk
# --------------------------------------------------------------------------
def galaxy(n: int = 1 << 22, seeds=(301, 302, 303)):
    """Three-component galaxy: NFW halo (c=10, 80 %), Hernquist bulge (a=0.1, 5 %),
    exponential disk (h=0.5, sech^2 height 0.05, 15 %); equal-mass particles.

    Bulge: M(<r) ~ r^2/(r+a)^2 truncated at r=10, inverted in closed form.
    Disk: R from 1-(1+R/h)e^{-R/h} truncated at 10h (bisection), z = z0 atanh(2u-1)
    with |z| <= 10 z0.  Counts are rounded so they sum to n exactly.
    """
    n_halo = int(round(0.80 * n))
    n_bulge = int(round(0.05 * n))
    n_disk = n - n_halo - n_bulge
    m = 1.0 / n
    halo = nfw(n_halo, seed=seeds[0])[:, :3].astype(np.float64)

    rng = np.random.default_rng(seeds[1])
    a, rt = 0.1, 10.0
    mt = rt ** 2 / (rt + a) ** 2
    s = np.sqrt(rng.uniform(0.0, 1.0, n_bulge) * mt)
    rb = a * s / (1.0 - s)
    bulge = _isotropic(rng, rb)

    rng = np.random.default_rng(seeds[2])
    h, z0 = 0.5, 0.05
    cdf = lambda x: 1.0 - (1.0 + x) * np.exp(-x)
    target = rng.uniform(0.0, 1.0, n_disk) * cdf(10.0)
    lo, hi = np.zeros(n_disk), np.full(n_disk, 10.0)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = cdf(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    R = h * 0.5 * (lo + hi)
    ph = rng.uniform(0.0, 2.0 * np.pi, n_disk)
    umax = np.tanh(10.0)
    z = z0 * np.arctanh(rng.uniform(-umax, umax, n_disk))
    disk = np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)

    pos = np.concatenate([halo, bulge, disk], axis=0)
    return _pack(pos, np.full(n, m))


# --------------------------------------------------------------------------
# batched systems: 64 independent spheres, log-uniform sizes
# --------------------------------------------------------------------------
def batched_systems(nsys: int = 64, seed: int = 401, lg_min: int = 12, lg_max: int = 18,
                    with_vel: bool = False):
    """nsys systems, N_s = floor(2^(lg_min + (lg_max-lg_min) u_s)); even s Plummer
    (eps 1/64), odd s NFW (eps 1/128); system s seeded with 410+s.

    Returns (xyzm concatenated, offsets int64 [nsys+1], eps float32 [nsys]
    [, vel float64]).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, nsys)
    sizes = np.floor(2.0 ** (lg_min + (lg_max - lg_min) * u)).astype(np.int64)
    parts, vels, eps = [], [], []
    for s in range(nsys):
        if s % 2 == 0:
            res = plummer(int(sizes[s]), seed=410 + s, with_vel=with_vel)
            eps.append(1.0 / 64)
        else:
            res = nfw(int(sizes[s]), seed=410 + s, with_vel=with_vel)
            eps.append(1.0 / 128)
        if with_vel:
            parts.append(res[0]); vels.append(res[1])
        else:
            parts.append(res)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    out = (np.concatenate(parts, axis=0), offsets, np.array(eps, dtype=np.float32))
    if with_vel:
        out = out + (np.concatenate(vels, axis=0),)
    return out


def random_active(n: int, frac: float, seed: int) -> np.ndarray:
    """A seeded 0/1 uint8 mask with about frac*n ones (block-step stand-in)."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.0, 1.0, n) < frac).astype(np.uint8)


# --------------------------------------------------------------------------
# the five measured workloads
# --------------------------------------------------------------------------
class Config(dict):
    pass


CONFIGS = {
    "plummer8k": Config(kind="plummer", n=8192, seed=101, eps=1.0 / 64, theta=0.5,
                        multipole=1, kmax=0),
    "nfw1m": Config(kind="nfw", n=1 << 20, seed=201, eps=1.0 / 128, theta=0.5,
                    multipole=2, kmax=8),
    "galaxy4m": Config(kind="galaxy", n=1 << 22, seed=301, eps=1.0 / 256, theta=0.5,
                       multipole=1, kmax=0),
    "batched64": Config(kind="batched", n=None, seed=401, eps=None, theta=0.5,
                        multipole=1, kmax=6),
    "nfw16m": Config(kind="nfw", n=1 << 24, seed=501, eps=1.0 / 512, theta=0.5,
                     multipole=2, kmax=8),
}


def config_system(name: str, n: int | None = None, with_vel: bool = False):
    """Build the named workload (optionally at a reduced particle count n)."""
    cfg = CONFIGS[name]
    nn = cfg["n"] if n is None else n
    if cfg["kind"] == "plummer":
        return plummer(nn, seed=cfg["seed"], with_vel=with_vel)
    if cfg["kind"] == "nfw":
        return nfw(nn, seed=cfg["seed"], with_vel=with_vel)
    if cfg["kind"] == "galaxy":
        return galaxy(nn)
    raise ValueError(name)
