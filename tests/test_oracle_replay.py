"""Pins for the oracle's check of another walk's decisions (walk_replay).

The replay walks the tree again following GIVEN accept/open decisions and
compares each with the float64 MAC.  Fed the oracle's own lists it must find
no disagreement and reproduce the oracle's forces bit for bit (same lists,
same summation order); fed the theta = 0 lists (every leaf, no multipole
term) it must give the direct sum; fed a list with one planted mistake it
must report it.
"""
import numpy as np
import pytest

import ics
import oracle


def _ref(x, eps, theta, **kw):
    return oracle.tree_forces(x, eps, theta, **kw)


def _own_lists(ref, eps, theta, multipole=1, mac=0, delta=0.0, amag=None):
    gsel = np.arange(ref["groups"]["first"].size)
    out, cnt, mass, lists = oracle.walk(ref["tree"], (ref["com"], ref["b"], ref["S"]), ref["ps"],
                                        ref["groups"], eps, theta, multipole, gsel=gsel,
                                        mac=mac, delta=delta, amag=amag, lists_cap=1 << 16)
    return gsel, lists, out


@pytest.mark.parametrize("multipole", [1, 2])
def test_replay_of_the_oracles_own_lists(multipole):
    x = ics.nfw(3000, seed=61)
    x[:, 3] *= np.random.default_rng(62).uniform(0.5, 1.5, 3000).astype(np.float32)
    eps, theta = 1 / 128, 0.5
    ref = _ref(x, eps, theta, multipole=multipole)
    gsel, lists, _ = _own_lists(ref, eps, theta, multipole)
    acc, info, mass = oracle.walk_replay(ref, gsel, lists, eps, theta, multipole)
    assert (info[:, 1:5] == 0).all()
    assert np.array_equal(acc, ref["acc_pot"])  # same lists, same order: identical sums
    assert np.allclose(mass, x[:, 3].astype(np.float64).sum(), rtol=1e-12)
    # the lists' sizes are the oracle's per-group counts
    sizes = np.array([[a.size, ref["tree"]["count"][b].sum()] for a, b in lists])
    assert np.array_equal(sizes, ref["counts"][:, :2])


@pytest.mark.parametrize("mac", [1, 2])
def test_replay_with_the_other_macs(mac):
    x = ics.plummer(2500, seed=63)
    eps = 1 / 64
    d = oracle.direct(x, eps)
    ref = oracle.tree_forces(x, eps, 0.5, mac=mac, delta=1e-3, acc_old=d)
    a3 = d[:, :3]
    amag = np.sqrt((a3 * a3).sum(1))[ref["perm"]] if mac == 1 else None
    gsel, lists, _ = _own_lists(ref, eps, 0.5, 1, mac=mac, delta=1e-3, amag=amag)
    acc, info, _ = oracle.walk_replay(ref, gsel, lists, eps, 0.5, 1, mac=mac, delta=1e-3,
                                      acc_old=d)
    assert (info[:, 1:5] == 0).all()
    assert np.array_equal(acc, ref["acc_pot"])


def test_replay_of_theta_zero_lists_is_the_direct_sum():
    # theta = 0: a node is accepted only when b_J = 0; every other leaf is opened
    x = ics.plummer(1500, seed=64)
    eps = 1 / 64
    ref = _ref(x, eps, 0.0)
    t = ref["tree"]
    leaves = np.flatnonzero(t["n_child"] == 0).astype(np.uint32)
    pts = ref["b"][leaves] == 0
    ng = ref["groups"]["first"].size
    lists = [(leaves[pts], leaves[~pts])] * ng
    acc, info, mass = oracle.walk_replay(ref, np.arange(ng), lists, eps, 0.0)
    assert (info[:, 1:5] == 0).all()
    d = oracle.direct(x, eps)
    assert np.abs(acc - d).max() <= 1e-13 * np.abs(d).max()


def test_replay_reports_planted_mistakes():
    x = ics.nfw(3000, seed=65)
    eps, theta = 1 / 128, 0.5
    ref = _ref(x, eps, theta)
    gsel, lists, _ = _own_lists(ref, eps, theta)
    g = int(np.argmax([a.size for a, _ in lists]))
    nodes, leaves = lists[g]
    assert leaves.size > 1 and nodes.size > 1
    one = np.array([g])
    # a dropped leaf: the walk reaches a leaf that is neither accepted nor opened
    _, info, mass = oracle.walk_replay(ref, one, [(nodes, leaves[1:])], eps, theta)
    assert info[0, 4] == 1 and info[0, 2] == 0
    assert mass[0] < x[:, 3].astype(np.float64).sum() * (1 - 1e-9)
    # a duplicated entry
    _, info, _ = oracle.walk_replay(ref, one, [(np.append(nodes, nodes[0]), leaves)], eps, theta)
    assert info[0, 4] == 1
    # the root accepted: a decision the float64 MAC contradicts, and every
    # other entry is never reached
    _, info, _ = oracle.walk_replay(ref, one, [(np.array([0], np.uint32), leaves)], eps, theta)
    assert info[0, 2] == 1 and info[0, 3] == leaves.size
    # an accepted node given as opened: its children are visited unlisted
    t = ref["tree"]
    inner = [J for J in nodes if t["n_child"][J] > 0]
    assert inner
    J = inner[0]
    _, info, _ = oracle.walk_replay(ref, one, [(nodes[nodes != J], leaves)], eps, theta)
    assert info[0, 2] >= 1
