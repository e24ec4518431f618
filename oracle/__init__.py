"""Python face of the float64 CPU oracle (oracle/gothic_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check the HIP library.  It shares no code with the
library and the library never imports it.

``tree_forces`` runs the whole method step by step (keys, stable sort,
breadth-first tree, pseudo j-particles, groups with pseudo i-particles, walk
with the opening-angle MAC) and returns every intermediate array so that
integer results can be compared bit for bit and floating results within a
tolerance.  ``direct`` is the softened direct sum (the plain definition the
tree approximates).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NLEV = 21


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_lib
        build_lib.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    i64, f64, i32 = C.c_int64, C.c_double, C.c_int
    lib.orc_num_threads.restype = i32
    lib.orc_direct.argtypes = [i64, P, f64, i64, P, P]
    lib.orc_morton.restype = C.c_uint64
    lib.orc_morton.argtypes = [C.c_uint64] * 3
    lib.orc_ph_encode.restype = C.c_uint64
    lib.orc_ph_encode.argtypes = [i32, C.c_uint64, C.c_uint64, C.c_uint64]
    lib.orc_ph_decode.argtypes = [i32, C.c_uint64, P, P, P]
    lib.orc_cube.argtypes = [i64, P, P]
    lib.orc_keys.argtypes = [i64, P, i32, P, P]
    lib.orc_sort.argtypes = [i64, P, P, P]
    lib.orc_build.restype = i64
    lib.orc_build.argtypes = [i64, P, i32, i64, P, P, P, P, P]
    lib.orc_moments.argtypes = [i64, P, P, P, P, P, P]
    lib.orc_groups.restype = i64
    lib.orc_groups.argtypes = [i64, P, P, i32, f64, P, P, P, P, i32]
    lib.orc_seb.argtypes = [i32, P, P]
    lib.orc_walk.argtypes = [i64, P, P, P, P, P, P, P, P, P, i64, P, P, P,
                             f64, f64, i32, f64, f64, P, i64, P, P, P, i32, f64, P, P, i64, P]
    lib.orc_walk_replay.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, f64, f64, i32, f64,
                                    f64, i32, f64, P, i64, P, P, i64, P, P, P, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ---------------------------------------------------------------- keys
def morton(x: int, y: int, z: int) -> int:
    return int(_load().orc_morton(x, y, z))


def ph_encode(x: int, y: int, z: int, nlev: int = NLEV) -> int:
    return int(_load().orc_ph_encode(nlev, x, y, z))


def ph_decode(key: int, nlev: int = NLEV):
    a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _load().orc_ph_decode(nlev, key, C.byref(a), C.byref(b), C.byref(c))
    return int(a.value), int(b.value), int(c.value)


def cube(xyzm: np.ndarray) -> np.ndarray:
    xyzm = np.ascontiguousarray(xyzm, dtype=np.float32)
    out = np.zeros(4, dtype=np.float64)
    _load().orc_cube(xyzm.shape[0], _p(xyzm), _p(out))
    return out


def keys(xyzm: np.ndarray, key_kind: int = 0):
    xyzm = np.ascontiguousarray(xyzm, dtype=np.float32)
    cb = cube(xyzm)
    k = np.zeros(xyzm.shape[0], dtype=np.uint64)
    _load().orc_keys(xyzm.shape[0], _p(xyzm), key_kind, _p(cb), _p(k))
    return k, cb


def sort(k: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.uint64)
    ks = np.zeros_like(k)
    perm = np.zeros(k.size, dtype=np.uint32)
    _load().orc_sort(k.size, _p(k), _p(ks), _p(perm))
    return ks, perm


def build(ks: np.ndarray, n_leaf: int = 16):
    n = ks.size
    cap = max(1, 2 * n + 64)
    while True:
        first = np.zeros(cap, np.uint32)
        count = np.zeros(cap, np.uint32)
        cf = np.zeros(cap, np.uint32)
        nc = np.zeros(cap, np.uint8)
        lv = np.zeros(cap, np.uint8)
        nn = _load().orc_build(n, _p(ks), n_leaf, cap, _p(first), _p(count), _p(cf),
                               _p(nc), _p(lv))
        if nn >= 0:
            break
        cap *= 2
    return dict(first=first[:nn].copy(), count=count[:nn].copy(), child_first=cf[:nn].copy(),
                n_child=nc[:nn].copy(), level=lv[:nn].copy())


def moments(tree, ps: np.ndarray):
    nn = tree["first"].size
    com = np.zeros((nn, 4), np.float64)
    b = np.zeros(nn, np.float64)
    S = np.zeros((nn, 6), np.float64)
    ps = np.ascontiguousarray(ps, dtype=np.float64)
    _load().orc_moments(nn, _p(tree["first"]), _p(tree["count"]), _p(ps), _p(com), _p(b), _p(S))
    return com, b, S


BALL_GEO, BALL_SEB, BALL_EBS, BALL_COM, BALL_CMP = 0, 1, 2, 3, 4


def groups(act_sorted: np.ndarray, ps: np.ndarray, G: int, r_crit: float = 0.0,
           ball: int = BALL_GEO):
    """r_crit: critical separation (Section 2.4); pass the float32 value the
    library uses, e.g. float(np.float32(r)); <= 0 disables the gap split.
    ball: the enclosing-ball kind of the pseudo i-particles (Appendix B)."""
    n = act_sorted.size
    act_sorted = np.ascontiguousarray(act_sorted, dtype=np.uint8)
    alist = np.zeros(max(n, 1), np.uint32)
    gmax = max(1, n)
    gfirst = np.zeros(gmax, np.uint32)
    gcount = np.zeros(gmax, np.uint32)
    balls = np.zeros((gmax, 4), np.float64)
    ng = _load().orc_groups(n, _p(act_sorted), _p(ps), G, float(r_crit), _p(alist), _p(gfirst),
                            _p(gcount), _p(balls), int(ball))
    na = int(act_sorted.sum())
    return dict(alist=alist[:na].copy(), first=gfirst[:ng].copy(), count=gcount[:ng].copy(),
                ball=balls[:ng].copy())


def seb(pts: np.ndarray):
    """Smallest enclosing ball of pts [n,3] (Welzl): (centre [3], radius)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.zeros(4, np.float64)
    _load().orc_seb(pts.shape[0], _p(pts), _p(out))
    return out[:3], float(out[3])


def walk(tree, mom, ps, grp, eps, theta, multipole=1, tie_rel=1e-5, tie_abs=0.0,
         gsel=None, mac=0, delta=0.0, amag=None, lists_cap=0):
    """mac 0: opening angle theta; 1: acceleration MAC with accuracy delta and
    amag = |a_old| of every particle in key order; 2: Warren-Salmon with delta.
    lists_cap > 0 (with gsel) also returns each selected group's list as
    (accepted node indices, opened leaf indices)."""
    com, b, S = mom
    if mac == 1:
        amag = np.ascontiguousarray(amag, dtype=np.float64)
    n = ps.shape[0]
    ng = grp["first"].size
    out = np.full((n, 4), np.nan, np.float64)
    cnt = np.zeros((max(ng, 1), 3), np.int64)
    mass = np.zeros(max(ng, 1), np.float64)
    if gsel is not None:
        gsel = np.ascontiguousarray(gsel, dtype=np.int64)
    want_lists = lists_cap > 0 and gsel is not None
    lists = np.zeros((gsel.size if want_lists else 1, max(lists_cap, 1)), np.uint32)
    lcount = np.zeros((gsel.size if want_lists else 1, 2), np.uint32)
    _load().orc_walk(tree["first"].size, _p(tree["first"]), _p(tree["count"]),
                     _p(tree["child_first"]), _p(tree["n_child"]), _p(com), _p(b), _p(S),
                     _p(ps), _p(grp["alist"]), ng, _p(grp["first"]), _p(grp["count"]),
                     _p(grp["ball"]), float(eps), float(theta), int(multipole),
                     float(tie_rel), float(tie_abs),
                     _p(gsel) if gsel is not None else None,
                     0 if gsel is None else gsel.size, _p(out), _p(cnt), _p(mass),
                     int(mac), float(delta), _p(amag) if mac == 1 else None,
                     _p(lists) if want_lists else None, int(lists_cap), _p(lcount))
    if want_lists:
        got = []
        for q in range(gsel.size):
            nl, nf = int(lcount[q, 0]), int(lcount[q, 1])
            if nl + nf > lists_cap:
                raise ValueError("lists_cap too small")
            got.append((lists[q, :nl].copy(), lists[q, nl:nl + nf] & 0x7fffffff))
        return out, cnt[:ng], mass[:ng], got
    return out, cnt[:ng], mass[:ng]


def tree_forces(xyzm, eps, theta, active=None, n_leaf=16, group_size=32, multipole=1,
                key_kind=0, tie_rel=1e-5, tie_abs=0.0, gsel=None, r_crit=-0.0625, mac=0,
                delta=0.0, acc_old=None, ball=BALL_GEO):
    """All steps of the method in float64; acc_pot is [n,4] in the caller's
    order (NaN rows for inactive particles).  r_crit < 0 is a fraction of the
    key-cube side (the library's convention); 0 disables the gap split.
    mac / delta: the acceptance criterion (see walk); acc_old [n,>=3] in the
    caller's order for the acceleration MAC."""
    xyzm = np.ascontiguousarray(xyzm, dtype=np.float32)
    n = xyzm.shape[0]
    k, cb = keys(xyzm, key_kind)
    ks, perm = sort(k)
    tree = build(ks, n_leaf)
    ps = xyzm[perm].astype(np.float64)
    mom = moments(tree, ps)
    act = np.ones(n, np.uint8) if active is None else np.asarray(active, np.uint8)
    rc = float(np.float32(r_crit))
    if rc < 0:
        rc = -rc * float(cb[3])
    grp = groups(act[perm], ps, group_size, rc, ball)
    amag = None
    if mac == 1:
        a3 = np.asarray(acc_old, np.float64)[:, :3]
        amag = np.sqrt((a3 * a3).sum(1))[perm]
    out_sorted, cnt, mass = walk(tree, mom, ps, grp, eps, theta, multipole, tie_rel, tie_abs,
                                 gsel, mac=mac, delta=delta, amag=amag)
    acc = np.full((n, 4), np.nan, np.float64)
    acc[perm] = out_sorted
    return dict(keys=k, cube=cb, keys_sorted=ks, perm=perm, tree=tree, com=mom[0], b=mom[1],
                S=mom[2], groups=grp, acc_pot=acc, counts=cnt, mass=mass, ps=ps)


def direct(xyzm, eps, idx=None):
    """Softened direct sum in float64 for the particles idx (default all);
    returns [len(idx),4] = ax, ay, az, phi."""
    xyzm = np.ascontiguousarray(xyzm, dtype=np.float32)
    n = xyzm.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, np.int64)
    out = np.zeros((idx.size, 4), np.float64)
    _load().orc_direct(n, _p(xyzm), float(eps), idx.size, _p(idx), _p(out))
    return out


def walk_replay(ref, gsel, lists, eps, theta, multipole=1, tie_rel=1e-5, tie_abs=0.0, mac=0,
                delta=0.0, acc_old=None):
    """Check another walk's interaction lists for the groups gsel of the
    float64 evaluation `ref` (the dict of tree_forces): lists[k] = (accepted
    node indices, opened leaf indices) of group gsel[k].  The tree is walked
    again following those decisions and each is compared with the float64
    MAC.  Returns (out [n,4] float64 forces of the listed groups' particles
    from the given lists, in the caller's order, NaN elsewhere; info [k,6]:
    visited, decisions differing inside the near-tie window, differing
    outside it, entries never reached, inconsistent entries, list entries;
    mass [k] summed mass of each list)."""
    t = ref["tree"]
    grp = ref["groups"]
    ps = ref["ps"]
    n = ps.shape[0]
    gsel = np.ascontiguousarray(gsel, dtype=np.int64)
    k = gsel.size
    cap = max([a.size + b.size for a, b in lists] + [1])
    ent = np.zeros((max(k, 1), cap), np.uint32)
    nent = np.zeros((max(k, 1), 2), np.uint32)
    for q, (acc_nodes, leaves) in enumerate(lists):
        ent[q, :acc_nodes.size] = acc_nodes
        ent[q, acc_nodes.size:acc_nodes.size + leaves.size] = leaves.astype(np.uint32) | 0x80000000
        nent[q] = (acc_nodes.size, leaves.size)
    amag = np.zeros(1)
    if mac == 1:
        a3 = np.asarray(acc_old, np.float64)[:, :3]
        amag = np.ascontiguousarray(np.sqrt((a3 * a3).sum(1))[ref["perm"]])
    out = np.full((n, 4), np.nan, np.float64)
    info = np.zeros((max(k, 1), 6), np.int64)
    mass = np.zeros(max(k, 1), np.float64)
    _load().orc_walk_replay(t["first"].size, _p(t["first"]), _p(t["count"]), _p(t["child_first"]),
                            _p(t["n_child"]), _p(ref["com"]), _p(ref["b"]), _p(ref["S"]), _p(ps),
                            _p(grp["alist"]), _p(grp["first"]), _p(grp["count"]), _p(grp["ball"]),
                            float(eps), float(theta), int(multipole), float(tie_rel),
                            float(tie_abs), int(mac), float(delta), _p(amag), k, _p(gsel), None,
                            cap, _p(ent), _p(nent), _p(out), _p(info), _p(mass))
    acc = np.full((n, 4), np.nan, np.float64)
    acc[ref["perm"]] = out
    return acc, info[:k], mass[:k]
