"""Pins for the oracle's keys, quantisation and sort (CPU only).

Morton (Appendix A): fixed bit positions, de-interleave round trip, order
equals the level-by-level octant order.  Peano-Hilbert (Appendix A): keys
traced by hand through the printed encoder (tests/golden), face adjacency of
consecutive cells (the defining property of a Hilbert curve), the hierarchical
block property, and an encode/decode round trip.  Sort: against numpy's
stable argsort.
"""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ph_keys_nlev2.txt")


def _deinterleave(key):
    x = y = z = 0
    for b in range(21):
        x |= ((key >> (3 * b + 2)) & 1) << b
        y |= ((key >> (3 * b + 1)) & 1) << b
        z |= ((key >> (3 * b)) & 1) << b
    return x, y, z


def test_morton_bit_positions():
    assert oracle.morton(1, 0, 0) == 4
    assert oracle.morton(0, 1, 0) == 2
    assert oracle.morton(0, 0, 1) == 1
    full = (1 << 21) - 1
    assert oracle.morton(full, full, full) == (1 << 63) - 1
    assert oracle.morton(1 << 20, 0, 0) == 1 << 62
    assert oracle.morton(0, 0, 1 << 20) == 1 << 60


def test_morton_roundtrip_random():
    rng = np.random.default_rng(7)
    for x, y, z in rng.integers(0, 1 << 21, size=(2000, 3)):
        k = oracle.morton(int(x), int(y), int(z))
        assert _deinterleave(k) == (x, y, z)


def test_morton_order_is_octant_order():
    # sorting a 4^3 grid by Morton key equals sorting by (octant digit level 1,
    # level 2) computed from the coordinates' bits
    pts = [(x, y, z) for x in range(4) for y in range(4) for z in range(4)]
    by_key = sorted(pts, key=lambda p: oracle.morton(*p))
    by_oct = sorted(pts, key=lambda p: (
        (p[0] >> 1) * 4 + (p[1] >> 1) * 2 + (p[2] >> 1), (p[0] & 1) * 4 + (p[1] & 1) * 2 + (p[2] & 1)))
    assert by_key == by_oct


def _gold():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tag, x, y, z, k = line.split()
        rows.append((1 if tag == "nlev1" else 2, int(x), int(y), int(z), int(k)))
    return rows


def test_ph_golden_hand_traced():
    rows = _gold()
    assert len(rows) >= 12
    for nlev, x, y, z, k in rows:
        assert oracle.ph_encode(x, y, z, nlev) == k, (nlev, x, y, z)


@pytest.mark.parametrize("nlev", [1, 2, 3, 4])
def test_ph_face_adjacent_and_bijective(nlev):
    side = 1 << nlev
    cells = {}
    for x in range(side):
        for y in range(side):
            for z in range(side):
                k = oracle.ph_encode(x, y, z, nlev)
                assert k not in cells
                cells[k] = (x, y, z)
    assert sorted(cells) == list(range(side ** 3))
    for k in range(side ** 3 - 1):
        a, b = np.array(cells[k]), np.array(cells[k + 1])
        assert np.abs(a - b).sum() == 1, (k, cells[k], cells[k + 1])
    assert cells[0] == (0, 0, 0)


@pytest.mark.parametrize("nlev", [2, 3])
def test_ph_hierarchical_blocks(nlev):
    # every aligned run of 8^l keys fills one aligned cube of side 2^l
    side = 1 << nlev
    inv = {}
    for x in range(side):
        for y in range(side):
            for z in range(side):
                inv[oracle.ph_encode(x, y, z, nlev)] = (x, y, z)
    for l in range(1, nlev + 1):
        run = 8 ** l
        for s in range(0, side ** 3, run):
            pts = np.array([inv[k] for k in range(s, s + run)])
            lo = pts.min(axis=0)
            assert (pts.max(axis=0) - lo == (1 << l) - 1).all()
            assert (lo % (1 << l) == 0).all()


def test_ph_roundtrip_random_21bit():
    rng = np.random.default_rng(11)
    for x, y, z in rng.integers(0, 1 << 21, size=(3000, 3)):
        k = oracle.ph_encode(int(x), int(y), int(z))
        assert k < (1 << 63)
        assert oracle.ph_decode(k) == (x, y, z)


def test_cube_and_quantisation():
    rng = np.random.default_rng(3)
    xyzm = rng.uniform(-3.0, 5.0, (1000, 4)).astype(np.float32)
    cb = oracle.cube(xyzm)
    ext = (xyzm[:, :3].max(0).astype(np.float64) - xyzm[:, :3].min(0)).max()
    L = cb[3]
    assert L >= ext and L / 2 < ext
    assert np.log2(L) == np.round(np.log2(L))
    assert np.array_equal(cb[:3], xyzm[:, :3].min(0).astype(np.float64))
    k, _ = oracle.keys(xyzm, 0)
    q = np.array([_deinterleave(int(v)) for v in k])
    # the minimum particle on each axis quantises to 0; all codes are in range
    assert (q.min(0) == 0).all() and (q.max(0) < (1 << 21)).all()
    # brute-force the quantisation of a few particles
    for i in range(0, 1000, 97):
        for a in range(3):
            t = np.floor((np.float64(xyzm[i, a]) - cb[a]) * (2.0 ** 21 / L))
            assert q[i, a] == min(int(t), (1 << 21) - 1)


def test_cube_power_of_two_extent_and_degenerate():
    xyzm = np.zeros((3, 4), np.float32)
    xyzm[:, 0] = [0.0, 2.0, 1.0]  # extent exactly 2 -> L = 2; x=2 clamps
    cb = oracle.cube(xyzm)
    assert cb[3] == 2.0
    k, _ = oracle.keys(xyzm, 0)
    assert _deinterleave(int(k[1]))[0] == (1 << 21) - 1
    assert _deinterleave(int(k[2]))[0] == 1 << 20
    one = np.zeros((1, 4), np.float32)
    assert oracle.cube(one)[3] == 1.0


def test_sort_stable_against_numpy():
    rng = np.random.default_rng(5)
    k = rng.integers(0, 50, 5000).astype(np.uint64)  # many equal keys
    ks, perm = oracle.sort(k)
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(perm, ref.astype(np.uint32))
    assert np.array_equal(ks, k[ref])
