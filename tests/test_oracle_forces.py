"""Pins for the oracle's direct sum and tree forces (CPU only).

Each pin is fixed by physics or mathematics, not by the oracle itself:
closed forms (two bodies, a symmetric cube of masses, the Plummer sphere's
enclosed mass), Newton's third law (momentum), the tree reducing to the direct
sum when the opening angle is zero, mass closure of every interaction list,
the truncation error falling with theta, the multipole orders of the
monopole and quadrupole terms (error ~ (b/d)^2 and (b/d)^3, in the
acceleration and in the potential), and the binomial series of a symmetric
pair of masses, whose b^4 term is the quadrupole node's residual.
"""
import numpy as np
import pytest

import ics
import oracle


def _rel_rms(a, b):
    return np.sqrt(((a[:, :3] - b[:, :3]) ** 2).sum() / (b[:, :3] ** 2).sum())


def test_two_body_closed_form():
    eps = 0.05
    xyzm = np.array([[0.0, 0.0, 0.0, 2.0], [1.5, 0.0, 0.0, 3.0]], np.float32)
    d = oracle.direct(xyzm, eps)
    R = np.sqrt(1.5 ** 2 + eps ** 2)
    assert np.isclose(d[0, 0], 3.0 * 1.5 / R ** 3, rtol=1e-14)  # pulled towards +x
    assert np.isclose(d[1, 0], -2.0 * 1.5 / R ** 3, rtol=1e-14)
    assert np.isclose(d[0, 3], -3.0 / R, rtol=1e-14) and np.isclose(d[1, 3], -2.0 / R, rtol=1e-14)
    assert d[0, 1] == 0 and d[0, 2] == 0
    t = oracle.tree_forces(xyzm, eps, 0.5, n_leaf=1, group_size=1)["acc_pot"]
    assert np.allclose(t, d, rtol=1e-14, atol=0)


def test_single_particle_self_term_removed():
    xyzm = np.array([[0.3, -0.2, 0.1, 1.0]], np.float32)
    t = oracle.tree_forces(xyzm, 0.01, 0.5)["acc_pot"]
    assert np.abs(t).max() <= 1e-12
    assert np.abs(oracle.direct(xyzm, 0.01)).max() == 0


def test_symmetric_cube_centre():
    s, m, eps = 0.5, 0.125, 0.02
    pts = [(x, y, z) for x in (-s, s) for y in (-s, s) for z in (-s, s)] + [(0.0, 0.0, 0.0)]
    xyzm = np.zeros((9, 4), np.float32)
    xyzm[:, :3] = pts
    xyzm[:8, 3] = m
    xyzm[8, 3] = 1.0
    d = oracle.direct(xyzm, eps)
    assert np.abs(d[8, :3]).max() < 1e-15
    assert np.isclose(d[8, 3], -8 * m / np.sqrt(3 * s * s + eps * eps), rtol=1e-14)
    t = oracle.tree_forces(xyzm, eps, 0.0, n_leaf=1, group_size=4)["acc_pot"]
    assert np.allclose(t, d, rtol=1e-13, atol=1e-15)


def test_momentum_conservation_direct():
    xyzm = ics.plummer(2048, seed=12)
    xyzm[:, 3] *= np.random.default_rng(2).uniform(0.2, 2.0, 2048).astype(np.float32)
    d = oracle.direct(xyzm, 1.0 / 64)
    m = xyzm[:, 3].astype(np.float64)
    net = np.abs((m[:, None] * d[:, :3]).sum(0)).max()
    assert net / (m[:, None] * np.abs(d[:, :3])).sum() < 1e-14


def test_plummer_shell_profile():
    # shell-averaged radial acceleration against -M(<r)/r^2 with the truncated
    # Plummer enclosed mass; discreteness noise ~ N_shell^-1/2
    n = 8192
    xyzm = ics.plummer(n, seed=101)
    d = oracle.direct(xyzm, 1.0 / 256)
    r = np.linalg.norm(xyzm[:, :3].astype(np.float64), axis=1)
    ar = (d[:, :3] * xyzm[:, :3].astype(np.float64)).sum(1) / r
    mt = 20.0 ** 3 / 401.0 ** 1.5
    edges = np.quantile(r, np.linspace(0.05, 0.9, 9))
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        rr = r[sel]
        menc = rr ** 3 / (rr ** 2 + 1) ** 1.5 / mt
        expect = -(menc / rr ** 2).mean()
        assert abs(ar[sel].mean() / expect - 1) < 0.06, (lo, hi)


def test_theta_zero_equals_direct_and_mass_closure():
    xyzm = ics.nfw(3000, seed=21)
    xyzm[:, 3] *= np.random.default_rng(3).uniform(0.5, 1.5, 3000).astype(np.float32)
    d = oracle.direct(xyzm, 1.0 / 128)
    r = oracle.tree_forces(xyzm, 1.0 / 128, 0.0, group_size=32)
    assert _rel_rms(r["acc_pot"], d) < 1e-13
    assert np.abs(r["acc_pot"][:, 3] - d[:, 3]).max() < 1e-13 * np.abs(d[:, 3]).max()
    M = xyzm[:, 3].astype(np.float64).sum()
    assert np.allclose(r["mass"], M, rtol=1e-13)


@pytest.mark.parametrize("multipole", [1, 2])
def test_mass_closure_and_error_falls_with_theta(multipole):
    xyzm = ics.plummer(8192, seed=101)
    d = oracle.direct(xyzm, 1.0 / 64)
    errs = []
    for th in (0.7, 0.5, 0.3):
        r = oracle.tree_forces(xyzm, 1.0 / 64, th, group_size=32, multipole=multipole)
        assert np.allclose(r["mass"], xyzm[:, 3].astype(np.float64).sum(), rtol=1e-12)
        errs.append(_rel_rms(r["acc_pot"], d))
    assert errs[0] > errs[1] > errs[2]
    if multipole == 1:
        # the paper's typical galactic accuracy, ~1e-3, sits at theta 0.5-0.7
        assert 3e-4 < errs[1] < 5e-3


def test_quadrupole_beats_monopole():
    xyzm = ics.nfw(8192, seed=31)
    d = oracle.direct(xyzm, 1.0 / 128)
    e1 = _rel_rms(oracle.tree_forces(xyzm, 1.0 / 128, 0.5, multipole=1)["acc_pot"], d)
    e2 = _rel_rms(oracle.tree_forces(xyzm, 1.0 / 128, 0.5, multipole=2)["acc_pot"], d)
    assert e2 < 0.6 * e1


def _far_cluster(D, seed=5):
    rng = np.random.default_rng(seed)
    k = 24
    pts = rng.uniform(-1.0, 1.0, (k, 3)) * [1.0, 0.6, 0.8]
    pts[:, 0] += D
    xyzm = np.zeros((k + 1, 4), np.float32)
    xyzm[1:, :3] = pts
    xyzm[1:, 3] = rng.uniform(0.5, 1.5, k)
    xyzm[0, 3] = 1.0
    act = np.zeros(k + 1, np.uint8)
    act[0] = 1
    return xyzm, act


@pytest.mark.parametrize("multipole,order", [(1, 2), (2, 3)])
def test_multipole_error_order(multipole, order):
    # one i-particle and a far cluster accepted as one node: the relative error
    # of the node term falls as (b/d)^order
    eps = 1e-3
    errs = []
    Ds = (20.0, 40.0, 80.0)  # the cluster stays inside one level-1 cell
    for D in Ds:
        xyzm, act = _far_cluster(D)
        r = oracle.tree_forces(xyzm, eps, 0.9, active=act, n_leaf=1, group_size=1,
                               multipole=multipole)
        # two node entries: the cluster's cell and the i-particle's own
        # one-particle leaf (b_J = 0, accepted; its self term is removed)
        assert r["counts"][0, 0] == 2 and r["counts"][0, 1] == 0
        d = oracle.direct(xyzm, eps, idx=np.array([0]))
        errs.append(np.linalg.norm(r["acc_pot"][0, :3] - d[0, :3]) / np.linalg.norm(d[0, :3]))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(Ds))
    assert np.all(np.abs(slopes + order) < 0.35), slopes


def test_group_subset_matches_full():
    xyzm = ics.plummer(3000, seed=44)
    full = oracle.tree_forces(xyzm, 1.0 / 64, 0.5)
    ng = full["groups"]["first"].size
    sel = np.array([0, 5, ng - 1])
    part = oracle.tree_forces(xyzm, 1.0 / 64, 0.5, gsel=sel)
    rows = np.isfinite(part["acc_pot"][:, 0])
    assert rows.sum() == full["groups"]["count"][sel].sum()
    assert np.array_equal(part["acc_pot"][rows], full["acc_pot"][rows])
    assert np.array_equal(part["counts"][sel], full["counts"][sel])


def test_inactive_rows_untouched_and_active_subset():
    xyzm = ics.plummer(2000, seed=45)
    act = ics.random_active(2000, 0.1, seed=46)
    r = oracle.tree_forces(xyzm, 1.0 / 64, 0.0, active=act)
    a = r["acc_pot"]
    assert np.isnan(a[act == 0]).all() and np.isfinite(a[act == 1]).all()
    d = oracle.direct(xyzm, 1.0 / 64, idx=np.flatnonzero(act))
    assert _rel_rms(a[act == 1], d) < 1e-13


# ---------------------------------------------------------------- other MACs (Section 2.2)
@pytest.mark.parametrize("mac", [1, 2])
def test_mac_tiny_delta_is_the_direct_sum(mac):
    x = ics.plummer(2000, seed=41)
    d = oracle.direct(x, 1 / 64)
    r = oracle.tree_forces(x, 1 / 64, 0.5, mac=mac, delta=1e-14, acc_old=d)
    assert np.abs(r["acc_pot"] - d).max() <= 1e-12 * np.abs(d).max()


@pytest.mark.parametrize("mac", [1, 2])
def test_mac_huge_delta_is_the_unit_opening_angle(mac):
    # with Delta -> infinity only the guard (b_J = 0 or b_J < d) is left: the
    # opening-angle MAC just below theta = 1, list for list (Warren-Salmon:
    # b/2 + sqrt(b^2/4) is b only to rounding, so nodes with d within an ulp
    # of b may differ)
    x = ics.nfw(3000, seed=42)
    d = oracle.direct(x, 1 / 128)
    r = oracle.tree_forces(x, 1 / 128, 0.5, mac=mac, delta=1e30, acc_old=d)
    r1 = oracle.tree_forces(x, 1 / 128, float(np.nextafter(1.0, 0.0)), mac=0)
    same = (r["counts"][:, :2] == r1["counts"][:, :2]).all(1)
    if mac == 1:
        assert same.all()
        assert np.array_equal(r["acc_pot"], r1["acc_pot"])
    else:
        assert same.mean() >= 0.99
        a, b = r["acc_pot"], r1["acc_pot"]
        assert np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()) < 1e-4


def test_acceleration_mac_error_scales_with_delta():
    # each accepted node's monopole error is at most about Delta |a_old| (Springel's
    # criterion); the median relative error is below Delta and falls with it
    x = ics.plummer(3000, seed=43)
    d = oracle.direct(x, 1 / 64)
    prev = np.inf
    for delta in (1e-1, 1e-2, 1e-3, 1e-4):
        a = oracle.tree_forces(x, 1 / 64, 0.5, mac=1, delta=delta, acc_old=d)["acc_pot"]
        err = np.linalg.norm(a[:, :3] - d[:, :3], axis=1) / np.linalg.norm(d[:, :3], axis=1)
        assert np.median(err) <= delta
        assert np.median(err) < prev
        prev = np.median(err)


def test_multipole_mac_error_scales_with_delta():
    # Warren-Salmon bound each node's truncation error by about Delta (an
    # absolute acceleration): the median absolute error stays below Delta
    x = ics.plummer(3000, seed=44)
    d = oracle.direct(x, 1 / 64)
    prev = np.inf
    for delta in (1e-1, 1e-2, 1e-3, 1e-4):
        a = oracle.tree_forces(x, 1 / 64, 0.5, mac=2, delta=delta)["acc_pot"]
        err = np.linalg.norm(a[:, :3] - d[:, :3], axis=1)
        assert np.median(err) <= delta
        assert np.median(err) < prev
        prev = np.median(err)


# ---------------------------------------------------------------- quadrupole closed forms
def _pair_node(D, b, along):
    """An i-particle at (D, 0, 0) and two masses m = 1/2 at -b and +b along
    `along` (0 = x, the line of sight; 2 = z, across it), far enough that the
    pair is one level-1 node accepted whole (theta 0.9, groups of one)."""
    xyzm = np.zeros((3, 4), np.float32)
    xyzm[0] = (D, 0.0, 0.0, 1.0)
    xyzm[1, along] = -b
    xyzm[2, along] = b
    xyzm[1:, 3] = 0.5
    act = np.array([1, 0, 0], np.uint8)
    return xyzm, act


def _tree_and_direct(xyzm, act, eps, multipole):
    r = oracle.tree_forces(xyzm, eps, 0.9, active=act, n_leaf=1, group_size=1,
                           multipole=multipole)
    # the pair's node and the i-particle's own one-particle leaf
    assert r["counts"][0, 0] == 2 and r["counts"][0, 1] == 0
    d = oracle.direct(xyzm, eps, idx=np.array([0]))
    return r["acc_pot"][0], d[0]


@pytest.mark.parametrize("D", [8.0, 16.0, 32.0])
def test_quadrupole_pair_across_the_line_of_sight_closed_form(D):
    # Two masses m at (0, 0, +-b) seen from (D, 0, 0) with softening eps:
    # exactly  phi = -2m (R^2 + b^2)^(-1/2),  a_x = -2m D (R^2 + b^2)^(-3/2),
    # R^2 = D^2 + eps^2.  The second-order expansion of the softened kernel
    # about the centre of mass keeps the b^2 terms, so the tree's residual is
    # the b^4 term of the binomial series:
    #   phi_exact - phi_tree = -(3/4) m b^4 / R^5,
    #   a_exact  - a_tree    = -(15/4) m b^4 D / R^7   (each + O(b^6)).
    # A wrong sign or factor of the trace term leaves a b^2 residual instead.
    m, b, eps = 0.5, 0.25, 1.0 / 64
    xyzm, act = _pair_node(D, b, along=2)
    t, d = _tree_and_direct(xyzm, act, eps, multipole=2)
    R = np.sqrt(D * D + eps * eps)
    assert np.isclose(d[3], -2 * m / np.sqrt(R * R + b * b), rtol=1e-14)
    assert np.isclose(d[0], -2 * m * D / (R * R + b * b) ** 1.5, rtol=1e-14)
    next_phi = 15.0 / 16 * m * b ** 6 / R ** 7   # size of the b^6 term
    next_acc = 105.0 / 16 * m * b ** 6 * D / R ** 9
    assert abs((d[3] - t[3]) - (-0.75 * m * b ** 4 / R ** 5)) <= 2 * next_phi
    assert abs((d[0] - t[0]) - (-3.75 * m * b ** 4 * D / R ** 7)) <= 2 * next_acc
    assert t[1] == 0.0 and t[2] == 0.0


def test_quadrupole_pair_along_the_line_of_sight_error_order():
    # Two masses on the line of sight (the y.S.y term is nonzero): the pair
    # has no dipole (centre of mass) and no octupole (symmetric), so the
    # quadrupole node's error in a and phi falls as (b/D)^4; the monopole's
    # as (b/D)^2.
    b, eps = 0.25, 1.0 / 64
    Ds = (8.0, 16.0, 32.0)
    for multipole, order in ((1, 2), (2, 4)):
        ea, ep = [], []
        for D in Ds:
            xyzm, act = _pair_node(D, b, along=0)
            t, d = _tree_and_direct(xyzm, act, eps, multipole)
            ea.append(abs(t[0] - d[0]) / abs(d[0]))
            ep.append(abs(t[3] - d[3]) / abs(d[3]))
        for errs in (ea, ep):
            slopes = np.diff(np.log(errs)) / np.diff(np.log(Ds))
            assert np.all(np.abs(slopes + order) < 0.2), (multipole, slopes)


@pytest.mark.parametrize("multipole,order", [(1, 2), (2, 3)])
def test_multipole_potential_error_order(multipole, order):
    # An unequal pair on the line of sight: 3/4 at x = -s and 1/4 at x = +3s
    # (centre of mass at 0) seen from (D, 0, 0).  Its multipole series along
    # that line is -(1/D)(1 + 3 (s/D)^2 + 6 (s/D)^3 + ...): the octupole term
    # is nonzero, so the relative potential error of a monopole node falls as
    # (s/D)^2 and that of a quadrupole node as (s/D)^3.
    s, eps = 0.25, 1.0 / 64
    Ds = (8.0, 16.0, 32.0)
    errs = []
    for D in Ds:
        xyzm = np.array([[D, 0, 0, 1.0], [-s, 0, 0, 0.75], [3 * s, 0, 0, 0.25]], np.float32)
        act = np.array([1, 0, 0], np.uint8)
        t, d = _tree_and_direct(xyzm, act, eps, multipole)
        errs.append(abs(t[3] - d[3]) / abs(d[3]))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(Ds))
    assert np.all(np.abs(slopes + order) < 0.2), slopes


def test_quadrupole_potential_beats_monopole():
    xyzm = ics.nfw(8192, seed=31)
    xyzm[:, 3] *= np.random.default_rng(32).uniform(0.5, 1.5, 8192).astype(np.float32)
    d = oracle.direct(xyzm, 1.0 / 128)

    def phi_err(mp):
        p = oracle.tree_forces(xyzm, 1.0 / 128, 0.5, multipole=mp)["acc_pot"][:, 3]
        return np.sqrt(((p - d[:, 3]) ** 2).sum() / (d[:, 3] ** 2).sum())

    assert phi_err(2) < 0.5 * phi_err(1)
