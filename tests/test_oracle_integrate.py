"""Pins for the float64 block-step integrator oracle (CPU only).

Level assignment against hand values and the logarithm away from level
boundaries; anchoring on the finest power of two; the level-change rule; the
paper's statement that with one fixed shared step the RK2 scheme is the
leap-frog (checked against an independent kick-drift-kick loop); second-order
convergence of the energy error on a two-body orbit; and the bookkeeping of a
block cycle (a level-k particle is active every 2^(kmax-k) sub-steps and all
particles are synchronised after 2^kmax sub-steps).
"""
import numpy as np
import pytest

import ics
import oracle
from oracle import integrate as I


def test_level_for_hand_values():
    dt = np.array([2.0, 1.0, 0.75, 0.5, 0.49, 1 / 256, 1 / 1000, np.inf])
    k = I.level_for(dt, 1.0, 8)
    assert list(k) == [0, 0, 1, 1, 2, 8, 8, 0]


def test_level_for_matches_log2_away_from_boundaries():
    rng = np.random.default_rng(1)
    dt = 2.0 ** rng.uniform(-10, 2, 5000)
    frac = np.log2(1.0 / dt) % 1.0
    ok = (frac > 1e-6) & (frac < 1 - 1e-6)
    k = I.level_for(dt[ok], 1.0, 8)
    assert np.array_equal(k, np.clip(np.ceil(np.log2(1.0 / dt[ok])), 0, 8).astype(np.int64))


def test_anchor_power_of_two():
    assert I.anchor(np.array([0.3, 0.7])) == 0.25
    assert I.anchor(np.array([0.25, 4.0])) == 0.25
    assert I.anchor(np.array([1.0])) == 1.0
    assert I.anchor(np.array([3e-5])) == 2.0 ** -16


def test_next_level_rule():
    kmax = 4
    # finer at once, whatever the time
    assert I.next_level([1], [3], 5, kmax)[0] == 3
    # coarser by one only when s is a multiple of the coarser step 2^(kmax-k+1)
    assert I.next_level([3], [0], 4, kmax)[0] == 2   # step of level 2 = 4 sub-steps
    assert I.next_level([3], [0], 6, kmax)[0] == 3   # 6 is not a multiple of 4
    assert I.next_level([2], [2], 8, kmax)[0] == 2
    assert I.next_level([0], [0], 16, kmax)[0] == 0


def _direct_force(eps):
    def f(xyzm, active):
        return oracle.direct(xyzm, eps)
    return f


def test_rk2_shared_equals_leapfrog():
    x, v = ics.plummer(64, seed=3, with_vel=True)
    eps = 0.05
    sim = I.BlockSim(x, v, eps, 0.1, 3, _direct_force(eps), shared=True)
    dt = sim.dt_fine
    for _ in range(40):
        sim.step()
    # independent kick-drift-kick leap-frog with the same float32 force input
    xr = x[:, :3].astype(np.float64).copy()
    vr = v.astype(np.float64).copy()

    def acc(p):
        s = np.empty((p.shape[0], 4), np.float32)
        s[:, :3] = p
        s[:, 3] = x[:, 3]
        return oracle.direct(s, eps)[:, :3]

    a = acc(xr)
    for _ in range(40):
        vr += 0.5 * dt * a
        xr += dt * vr
        a = acc(xr)
        vr += 0.5 * dt * a
    assert np.abs(sim.x - xr).max() < 1e-12 * np.abs(xr).max()
    assert np.abs(sim.v - vr).max() < 1e-12 * np.abs(vr).max()


def _two_body(e=0.5):
    # bodies of mass 0.5 on an orbit of semi-major axis 1 and eccentricity e,
    # started at apocentre
    m = 0.5
    ra = 1.0 + e
    vrel = np.sqrt((1.0) * (1 - e) / ra)  # G M_tot = 1, vis-viva at apocentre
    x = np.array([[-ra / 2, 0, 0, m], [ra / 2, 0, 0, m]], np.float32)
    v = np.array([[0, -vrel / 2, 0], [0, vrel / 2, 0]], np.float64)
    return x, v


def test_two_body_energy_second_order():
    # largest energy error over the first half orbit (apocentre to pericentre)
    # at two step sizes: a second-order scheme gives a ratio near 4
    errs = []
    period = 2 * np.pi
    for nsteps in (200, 400):
        x, v = _two_body()
        eps = 1e-4
        sim = I.BlockSim(x, v, eps, 0.1, 0, _direct_force(eps), shared=True)
        sim.dt_fine = period / nsteps
        e0 = sim.energy()
        worst = 0.0
        for _ in range(nsteps // 2):
            sim.step()
            worst = max(worst, abs(sim.energy() - e0) / abs(e0))
        errs.append(worst)
    ratio = errs[0] / errs[1]
    assert errs[1] > 1e-6  # well above the float32 force-input floor
    assert 3.0 < ratio < 5.0, errs


def test_block_cycle_bookkeeping():
    x, v = ics.nfw(300, seed=4, with_vel=True)
    eps, kmax = 1 / 32, 4
    sim = I.BlockSim(x, v, eps, 0.1, kmax, _direct_force(eps))
    k0 = sim.k.copy()
    assert k0.min() >= 0 and k0.max() <= kmax and k0.max() == kmax  # anchored at the finest
    counts = np.zeros(300, np.int64)
    for _ in range(1 << kmax):
        act = sim.step()
        counts += act
    # every particle was active, and all are synchronised after a full cycle
    assert np.all(counts >= 1)
    assert np.all(sim.si == sim.s)
    # no particle is active more often than the finest level allows
    assert counts.max() <= 1 << kmax


def test_state_taken_mid_cycle_predicts_like_the_integrated_one():
    x, v = ics.nfw(300, seed=5, with_vel=True)
    eps, kmax = 1 / 32, 4
    sim = I.BlockSim(x, v, eps, 0.1, kmax, _direct_force(eps))
    for _ in range(3):
        sim.step()
    got = I.BlockSim.from_state(sim.x, sim.v, sim.a, sim.m, sim.k, sim.si, sim.s, sim.dt_fine,
                                eps, 0.1, kmax)
    s = sim.s + 1
    assert np.array_equal(got.due(s), sim.due(s)) and got.due(s).any()
    assert np.array_equal(got.predict(s), sim.predict(s))
    assert got.dt_max == sim.dt_max
    # the copy does not alias the integrated state
    sim.step()
    assert not np.array_equal(got.si, sim.si)
