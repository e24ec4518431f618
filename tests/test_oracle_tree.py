"""Pins for the oracle's octree, pseudo j-particles and groups (CPU only).

Tree: a hand-placed example whose shape is known, brute-force enumeration of
the cells from key prefixes, and the structural invariants.  Moments: the
parallel-axis identity (children's moments combine into the parent's),
containment and tightness of b_J, root mass and centre of mass.  Groups:
chunking and the geometric-centre ball.
"""
import numpy as np
import pytest

import ics
import oracle


def _tree_for(xyzm, n_leaf, key_kind=0):
    k, _ = oracle.keys(xyzm, key_kind)
    ks, perm = oracle.sort(k)
    return ks, perm, oracle.build(ks, n_leaf)


def test_hand_placed_tree():
    # 8 particles near the corners of the unit cube plus 2 more in the (+,+,+)
    # octant and two pinning the cube to [0,1]; n_leaf = 2: the root splits
    # into 8 children and only the (+,+,+) child (4 particles) splits again,
    # into octant 110 (1 particle) and 111 (3 particles, split once more).
    c = []
    for x in (0.1, 0.9):
        for y in (0.1, 0.9):
            for z in (0.1, 0.9):
                c.append((x, y, z))
    c += [(0.95, 0.95, 0.95), (0.99, 0.99, 0.6)]
    pts = np.array(c)
    pts = np.vstack([pts, [[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]])  # pin the cube to [0,1]
    xyzm = np.zeros((pts.shape[0], 4), np.float32)
    xyzm[:, :3] = pts
    xyzm[:, 3] = 1.0
    ks, perm, t = _tree_for(xyzm, 2)
    assert t["n_child"][0] == 8
    assert list(t["level"][1:9]) == [1] * 8
    assert list(t["count"][1:9]) == [2, 1, 1, 1, 1, 1, 1, 4]
    split = [k for k in range(1, 9) if t["n_child"][k] > 0]
    assert split == [8]  # (-,-,-) holds 2 = n_leaf (a leaf); (+,+,+) holds 4
    assert t["child_first"][8] == 9
    assert t["n_child"][8] == 2 and list(t["count"][9:11]) == [1, 3]
    assert t["n_child"][9] == 0 and t["n_child"][10] > 0 and t["level"][10] == 2


def _brute_cells(ks, n_leaf):
    """All (level, prefix) cells whose parent cell holds more than n_leaf keys."""
    n = ks.size
    cells = {(0, 0): (0, n)}
    out = [(0, 0, 0, n)]
    for l in range(1, 22):
        pref = ks >> np.uint64(3 * (21 - l))
        ppref = ks >> np.uint64(3 * (21 - l + 1))
        starts = np.flatnonzero(np.r_[True, pref[1:] != pref[:-1]])
        ends = np.r_[starts[1:], n]
        for s, e in zip(starts, ends):
            par = (l - 1, int(ppref[s]))
            ps, pe = cells[par] if par in cells else (None, None)
            if ps is not None and pe - ps > n_leaf:
                cells[(l, int(pref[s]))] = (s, e)
                out.append((l, int(pref[s]), s, e - s))
    return out


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n,n_leaf", [(3000, 16), (2000, 4), (777, 1)])
def test_tree_matches_brute_force_cells(kind, n, n_leaf):
    xyzm = ics.nfw(n, seed=n + kind)
    ks, perm, t = _tree_for(xyzm, n_leaf, kind)
    brute = _brute_cells(ks, n_leaf)
    # brute list is in (level, key) order = BFS order of the oracle's tree
    assert len(brute) == t["first"].size
    for k, (l, _, s, c) in enumerate(brute):
        assert t["level"][k] == l and t["first"][k] == s and t["count"][k] == c


@pytest.mark.parametrize("kind", [0, 1])
def test_tree_invariants(kind):
    xyzm = ics.plummer(5000, seed=9)
    xyzm[100:140, :3] = xyzm[99, :3]  # coincident keys force level-21 leaves
    ks, perm, t = _tree_for(xyzm, 8, kind)
    nn = t["first"].size
    covered = np.zeros(ks.size, np.int32)
    for k in range(nn):
        f, c, nc, l = int(t["first"][k]), int(t["count"][k]), int(t["n_child"][k]), int(t["level"][k])
        if nc == 0:
            assert c <= 8 or l == 21
            covered[f:f + c] += 1
            assert t["child_first"][k] == 0
        else:
            ch = range(int(t["child_first"][k]), int(t["child_first"][k]) + nc)
            assert sum(int(t["count"][j]) for j in ch) == c
            s = f
            for j in ch:
                assert t["first"][j] == s and t["level"][j] == l + 1
                s += int(t["count"][j])
        if l > 0:
            pre = ks[f:f + c] >> np.uint64(3 * (21 - l))
            assert (pre == pre[0]).all()
    assert (covered == 1).all()
    assert (np.diff(t["level"].astype(int)) >= 0).all()
    assert (t["level"] == 21).any()


def test_empty_and_single():
    t = oracle.build(np.zeros(0, np.uint64), 16)
    assert t["first"].size == 0
    t = oracle.build(np.zeros(1, np.uint64), 16)
    assert t["first"].size == 1 and t["count"][0] == 1 and t["n_child"][0] == 0


def test_moments_parallel_axis_and_ball():
    xyzm = ics.nfw(4000, seed=2)
    xyzm[:, 3] *= np.random.default_rng(1).uniform(0.5, 1.5, 4000).astype(np.float32)
    ks, perm, t = _tree_for(xyzm, 8)
    ps = xyzm[perm].astype(np.float64)
    com, b, S = oracle.moments(t, ps)
    M = ps[:, 3].sum()
    assert abs(com[0, 3] - M) <= 1e-13 * M
    gc = (ps[:, :3] * ps[:, 3:4]).sum(0) / M
    assert np.allclose(com[0, :3], gc, rtol=0, atol=1e-13)
    for k in range(t["first"].size):
        f, c = int(t["first"][k]), int(t["count"][k])
        d = np.linalg.norm(ps[f:f + c, :3] - com[k, :3], axis=1)
        assert d.max() <= b[k] * (1 + 1e-14) + 1e-300  # contains every member
        assert d.max() >= b[k] * (1 - 1e-14)  # and is tight
        nc = int(t["n_child"][k])
        if nc:
            ch = np.arange(int(t["child_first"][k]), int(t["child_first"][k]) + nc)
            Mc = com[ch, 3]
            assert abs(Mc.sum() - com[k, 3]) <= 1e-14 * com[k, 3]
            rc = (com[ch, :3] * Mc[:, None]).sum(0) / Mc.sum()
            assert np.allclose(rc, com[k, :3], rtol=0, atol=1e-13)
            # parallel-axis: S_parent = sum_c [S_c + M_c d_c d_c^T]
            dd = com[ch, :3] - com[k, :3]
            Sp = S[ch].sum(0).copy()
            Sp[0] += (Mc * dd[:, 0] ** 2).sum(); Sp[1] += (Mc * dd[:, 1] ** 2).sum()
            Sp[2] += (Mc * dd[:, 2] ** 2).sum(); Sp[3] += (Mc * dd[:, 0] * dd[:, 1]).sum()
            Sp[4] += (Mc * dd[:, 0] * dd[:, 2]).sum(); Sp[5] += (Mc * dd[:, 1] * dd[:, 2]).sum()
            scale = com[k, 3] * max(b[k], 1e-300) ** 2
            assert np.abs(Sp - S[k]).max() <= 1e-12 * scale


@pytest.mark.parametrize("r_crit", [0.05, 0.3])
def test_groups_split_at_critical_separation(r_crit):
    xyzm = ics.nfw(3000, seed=6)
    act = ics.random_active(3000, 0.5, seed=7)
    k, _ = oracle.keys(xyzm, 0)
    ks, perm = oracle.sort(k)
    ps = xyzm[perm].astype(np.float64)
    g = oracle.groups(act[perm], ps, 16, r_crit)
    al = g["alist"]
    gap = np.r_[np.inf, np.sqrt((np.diff(ps[al, :3], axis=0) ** 2).sum(1))]
    starts = np.zeros(al.size, bool)
    starts[g["first"]] = True
    # a group never spans a gap above r_crit ...
    assert np.all(starts[gap > r_crit])
    # ... and inside a run of small gaps groups are cut exactly every G
    run = np.maximum.accumulate(np.where(gap > r_crit, np.arange(al.size), 0))
    assert np.array_equal(starts, (np.arange(al.size) - run) % 16 == 0)
    assert g["count"].sum() == al.size and g["count"].max() <= 16
    assert np.array_equal(g["first"][1:], (g["first"] + g["count"])[:-1])
    # no split at all without r_crit
    g0 = oracle.groups(act[perm], ps, 16, 0.0)
    assert g0["first"].size == (al.size + 15) // 16


def test_groups_chunks_and_geo_ball():
    xyzm = ics.plummer(1000, seed=4)
    act = ics.random_active(1000, 0.3, seed=8)
    k, _ = oracle.keys(xyzm, 0)
    ks, perm = oracle.sort(k)
    ps = xyzm[perm].astype(np.float64)
    g = oracle.groups(act[perm], ps, 32)
    na = int(act.sum())
    assert np.array_equal(g["alist"], np.flatnonzero(act[perm]).astype(np.uint32))
    assert g["first"].size == (na + 31) // 32
    assert (g["count"][:-1] == 32).all() and g["count"].sum() == na
    for q in range(g["first"].size):
        mem = ps[g["alist"][g["first"][q]:g["first"][q] + g["count"][q]], :3]
        c = 0.5 * (mem.min(0) + mem.max(0))
        assert np.array_equal(g["ball"][q, :3], c)
        assert np.isclose(g["ball"][q, 3], np.linalg.norm(mem - c, axis=1).max(), rtol=1e-15)


# ---------------------------------------------------------------- enclosing balls (Appendix B)
def _brute_seb(P):
    """Smallest enclosing ball by enumerating every ball through 1-4 points."""
    import itertools
    best = None
    for k in (1, 2, 3, 4):
        for S in itertools.combinations(range(len(P)), k):
            pts = P[list(S)]
            if k == 1:
                c = pts[0]
            elif k == 2:
                c = pts.mean(0)
            elif k == 3:
                a, b, cc = pts
                u, v = b - a, cc - a
                w = np.cross(u, v)
                if w @ w < 1e-20:
                    continue
                c = a + np.cross((u @ u) * v - (v @ v) * u, w) / (2 * (w @ w))
            else:
                M = 2 * (pts[1:] - pts[0])
                if abs(np.linalg.det(M)) < 1e-14:
                    continue
                c = np.linalg.solve(M, (pts[1:] ** 2).sum(1) - pts[0] @ pts[0])
            r = np.sqrt(((P - c) ** 2).sum(1).max())
            if best is None or r < best[1]:
                best = (c, r)
    return best


def test_smallest_enclosing_ball_is_the_brute_force_minimum():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 9))
        P = rng.normal(size=(n, 3)) * rng.uniform(0.01, 10)
        c, r = oracle.seb(P)
        cb, rb = _brute_seb(P)
        assert abs(r - rb) <= 1e-9 * max(rb, 1e-300)
        assert np.all(np.sqrt(((P - c) ** 2).sum(1)) <= r * (1 + 1e-12))


def test_smallest_enclosing_ball_special_cases():
    # regular tetrahedron: the circumsphere; square: its circumcircle; a
    # segment with interior points: half its length; repeated points
    tet = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    c, r = oracle.seb(tet)
    assert np.allclose(c, 0, atol=1e-12) and abs(r - np.sqrt(3)) < 1e-12
    sq = np.array([[1, 0, 5], [0, 1, 5], [-1, 0, 5], [0, -1, 5], [0.2, 0.1, 5]], float)
    c, r = oracle.seb(sq)
    assert np.allclose(c, [0, 0, 5], atol=1e-12) and abs(r - 1) < 1e-12
    seg = np.array([[0, 0, 0], [0.3, 0, 0], [2, 0, 0], [1.1, 0, 0]], float)
    c, r = oracle.seb(seg)
    assert np.allclose(c, [1, 0, 0], atol=1e-12) and abs(r - 1) < 1e-12
    rep = np.array([[0.5, 0.5, 0.5]] * 5 + [[1.5, 0.5, 0.5]], float)
    c, r = oracle.seb(rep)
    assert abs(r - 0.5) < 1e-12


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_group_balls_contain_their_members(kind):
    x = ics.nfw(6000, seed=12)
    k, _ = oracle.keys(x)
    ks, perm = oracle.sort(k)
    ps = x[perm].astype(np.float64)
    act = ics.random_active(6000, 0.5, seed=13)[perm]
    grp = oracle.groups(act, ps, 32, 0.0, kind)
    seb_r = []
    for q in range(grp["first"].size):
        mem = ps[grp["alist"][grp["first"][q]:grp["first"][q] + grp["count"][q]], :3]
        c, r = grp["ball"][q, :3], grp["ball"][q, 3]
        dist = np.sqrt(((mem - c) ** 2).sum(1))
        assert r == dist.max()  # the radius is the largest member distance
        _, rs = oracle.seb(mem)
        seb_r.append((r, rs))
        if kind == 1:
            assert abs(r - rs) <= 1e-12 * rs
    ratio = np.array([r / rs for r, rs in seb_r if rs > 0])
    assert np.all(ratio >= 1 - 1e-12)
    if kind == 2:   # Ritter: a few per cent above the minimum
        assert np.median(ratio) < 1.05 and ratio.max() < 1.3
    if kind == 0:   # bounding-box centre: at most sqrt(3) x the minimum
        assert ratio.max() <= np.sqrt(3) + 1e-12


def test_cmp_ball_is_the_smaller_of_geo_and_com():
    x = ics.plummer(5000, seed=14)
    k, _ = oracle.keys(x)
    ks, perm = oracle.sort(k)
    ps = x[perm].astype(np.float64)
    act = np.ones(5000, np.uint8)
    geo = oracle.groups(act, ps, 16, 0.0, 0)["ball"]
    com = oracle.groups(act, ps, 16, 0.0, 3)["ball"]
    cmp_ = oracle.groups(act, ps, 16, 0.0, 4)["ball"]
    use_com = com[:, 3] < geo[:, 3] * (1 - 1e-5)
    assert np.array_equal(cmp_[use_com], com[use_com])
    assert np.array_equal(cmp_[~use_com], geo[~use_com])
    assert 0 < use_com.mean() < 1


# ---------------------------------------------------------------- balls worked by hand
def _one_group(pts, masses):
    """All points active, one group, in the given order (they are passed as
    already key-sorted positions)."""
    ps = np.zeros((len(pts), 4))
    ps[:, :3] = pts
    ps[:, 3] = masses
    return ps, np.ones(len(pts), np.uint8)


def test_com_ball_is_mass_weighted():
    # masses 1 and 3 at x = 0 and x = 4: the centre of mass is x = 3 (not the
    # plain mean 2), radius 3
    ps, act = _one_group([[0, 0, 0], [4, 0, 0]], [1.0, 3.0])
    b = oracle.groups(act, ps, 2, 0.0, oracle.BALL_COM)["ball"][0]
    assert np.allclose(b, [3, 0, 0, 3], rtol=0, atol=1e-15)
    # 3-D: masses 1, 1, 2 at (0,0,0), (2,0,0), (0,2,0): centre (1/2, 1, 0),
    # farthest member (2,0,0) at sqrt(9/4 + 1)
    ps, act = _one_group([[0, 0, 0], [2, 0, 0], [0, 2, 0]], [1.0, 1.0, 2.0])
    b = oracle.groups(act, ps, 4, 0.0, oracle.BALL_COM)["ball"][0]
    assert np.allclose(b, [0.5, 1.0, 0.0, np.sqrt(3.25)], rtol=0, atol=1e-15)
    # CMP keeps GEO here: the bounding-box ball (centre (1, 1, 0), radius
    # sqrt 2) is smaller than the COM ball
    c = oracle.groups(act, ps, 4, 0.0, oracle.BALL_CMP)["ball"][0]
    assert np.allclose(c, [1, 1, 0, np.sqrt(2)], rtol=0, atol=1e-15)
    # and takes COM when that is smaller: equal masses at (0,0,0), (4,0,0),
    # (2,3,0): COM (2, 1, 0) radius sqrt 5 < GEO (2, 1.5, 0) radius 2.5
    ps, act = _one_group([[0, 0, 0], [4, 0, 0], [2, 3, 0]], [1.0, 1.0, 1.0])
    c = oracle.groups(act, ps, 4, 0.0, oracle.BALL_CMP)["ball"][0]
    assert np.allclose(c, [2, 1, 0, np.sqrt(5)], rtol=0, atol=1e-15)


def test_ebs_ball_worked_by_hand():
    # Ritter's sphere.  Members in order: P0 (0,0,0), P1 (6,0,0), P2 (3,4,0),
    # P3 (3,0.5,-5).  Farthest from P0 is P1 (36 against 25 and 34.25);
    # farthest from P1 is P0.  Start: centre (3,0,0), radius 3.
    # P2 lies 4 > 3 out: the grown sphere is the smallest one holding the old
    # sphere and P2, i.e. tangent to the old one on the far side and passing
    # through P2: radius (3 + 4)/2 = 3.5, centre P2 + (c - P2) 3.5/4 =
    # (3, 0.5, 0).  P3 then lies 5 > 3.5 out: radius (3.5 + 5)/2 = 4.25,
    # centre P3 + (c - P3) 4.25/5 = (3, 0.5, -0.75).  The ball's radius is the
    # largest member distance from that centre, P3's 4.25.
    pts = [[0, 0, 0], [6, 0, 0], [3, 4, 0], [3, 0.5, -5]]
    ps, act = _one_group(pts, [1.0] * 4)
    b = oracle.groups(act, ps, 4, 0.0, oracle.BALL_EBS)["ball"][0]
    assert np.allclose(b, [3, 0.5, -0.75, 4.25], rtol=0, atol=1e-12)
    # without P3 the sphere stops after the first growth
    ps, act = _one_group(pts[:3], [1.0] * 3)
    b = oracle.groups(act, ps, 4, 0.0, oracle.BALL_EBS)["ball"][0]
    assert np.allclose(b, [3, 0.5, 0, 3.5], rtol=0, atol=1e-12)
