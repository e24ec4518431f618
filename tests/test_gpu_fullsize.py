"""Parity at the workloads' full sizes, on outputs the oracle can afford.

* NFW 2^24, eps 1/512, theta 0.5, quadrupole, in the launch configuration the
  benchmark times (G = 32, r_crit = 0.25, list depth 384, EBS balls): bit-exact
  keys, permutation, octree and groups; forces of 48 sampled groups against
  the float64 tree.
* The benchmark's block sub-steps on that system (kmax 8, eta 0.1, captured
  sub-steps, groups of one in sub-step class 0, trees rebuilt when the growth
  models say so): sub-steps of both group sizes on a reused tree and the first
  sub-step on a rebuilt one, each against the oracle's own prediction, tree,
  groups and forces of sampled groups.
* Galaxy-like model 2^22 (NFW halo + Hernquist bulge + exponential disk),
  eps 1/256, theta 0.5, monopole: plain FP32 and compensated accumulation
  against the float64 tree and the float64 direct sum on 4096 random
  particles (seed 304).
* NFW 2^20, eps 1/128, quadrupole, block levels (kmax = 8): t = 0 forces on
  sampled groups, anchored steps exact, levels exact away from boundaries.
"""
import functools

import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, oracle_parts, rel_rms, say, tie_params
from oracle import integrate as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _oracle_prep(x, n_leaf, G, r_crit, key_kind=0):
    k, cb = oracle.keys(x, key_kind)
    ks, perm = oracle.sort(k)
    tree = oracle.build(ks, n_leaf)
    ps = x[perm].astype(np.float64)
    mom = oracle.moments(tree, ps)
    rc = float(np.float32(r_crit))
    rc = -rc * cb[3] if rc < 0 else rc
    return ks, perm, tree, ps, mom, rc


@functools.lru_cache(maxsize=1)
def _nfw16m():
    """The benchmark's system (NFW 2^24, seed 501) with velocities, and the
    oracle's keys, permutation, tree and moments of its float32 positions."""
    x, v = ics.nfw(1 << 24, seed=501, with_vel=True)
    say("  oracle tree at 2^24")
    return (x, v) + _oracle_prep(x, 16, 32, 0.25)


def test_nfw16m_bench_configuration():
    n, eps, theta = 1 << 24, 1 / 512, 0.5
    say("[gpu] NFW 2^24 quadrupole, G=32, r_crit=0.25, list depth 384, EBS balls")
    x, _, ks_o, perm_o, tree, ps, mom, rc = _nfw16m()
    ctx = g.Context(device=0, multipole=2, group_size=32, r_crit=0.25, list_depth=384,
                    ball=oracle.BALL_EBS)
    out = ctx.tree_forces(torch.from_numpy(x).cuda(), eps, theta).cpu().numpy()
    ks, perm, cube = ctx.keys()
    t = ctx.tree()
    gg = ctx.groups()
    assert np.array_equal(ks, ks_o) and np.array_equal(perm, perm_o)
    for f in ("first", "count", "child_first", "n_child", "level"):
        assert np.array_equal(t[f], tree[f]), f
    grp = oracle.groups(np.ones(n, np.uint8), ps, 32, rc, oracle.BALL_EBS)
    assert np.array_equal(gg["first"], grp["first"]) and np.array_equal(gg["count"], grp["count"])
    # EBS centres: float64 on both sides, rounded to float32 by the library
    scale = np.abs(grp["ball"][:, :3]).max(1) + grp["ball"][:, 3]
    close = np.abs(gg["ball"][:, :3] - grp["ball"][:, :3]).max(1) <= 1e-6 * scale
    assert close.mean() >= 0.999
    rng = np.random.default_rng(5)
    ng = grp["first"].size
    sel = np.unique(np.r_[rng.choice(ng, 40, replace=False), np.argsort(-grp["ball"][:, 3])[:8]])
    gate_forces(ctx, oracle_parts(tree, mom, ps, grp, perm), out, np.ones(n, bool), eps, theta,
                2, sel=sel, label=f"sampled {sel.size} groups: ")
    assert ctx.stats()["sticky_flags"] == 0


def test_nfw16m_bench_block_substeps():
    """Sub-steps as the benchmark times them.  Before every sub-step the float64
    state is read back; the oracle predicts every particle from it to the new
    sub-step (float64, rounded to float32: the library's key-ordered positions
    must be these, bit for bit), selects the due ones, and, on the sub-step
    that builds a new tree, builds its own from those positions (keys,
    permutation and octree must be the library's, bit for bit).  On the checked
    sub-steps it computes node moments on the tree in use, groups of the
    class's size and the forces of sampled groups, which the library's must
    match.  The first sub-step is checked and the rest captured, as in the
    benchmark's warm-up."""
    n, eps, theta, eta, kmax = 1 << 24, 1 / 512, 0.5, 0.1, 8
    say("[gpu] NFW 2^24 block sub-steps, captured, groups of 1 in class 0 and 32 above, "
        "growth-model rebuilds")
    x, v, _, perm_t, tree_t, _, _, rc = _nfw16m()
    ctx = g.Context(device=0, multipole=2, group_size=32, r_crit=0.25, list_depth=384,
                    ball=oracle.BALL_EBS, graph=1, rebuild_interval=0)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    m32 = np.ascontiguousarray(x[:, 3])
    ctx.sim_bind(pos, vel, torch.from_numpy(m32).cuda(), eps, theta, eta=eta, kmax=kmax)
    table = [1] + [32] * kmax  # group size per sub-step class
    ctx.sim_set_group_sizes(table)
    info = ctx.sim_info()
    dt_fine, builds = info["dt_fine"], info["tree_builds"]
    rng = np.random.default_rng(9)
    checked = []
    for s in range(1, 25):
        acc, lev, last = ctx.sim_state()
        st = I.BlockSim.from_state(pos.cpu().numpy(), vel.cpu().numpy(), acc, m32, lev, last,
                                   s - 1, dt_fine, eps, eta, kmax)
        del acc, lev, last
        ctx.set_params(check=1 if s == 1 else 0)
        ctx.sim_step()
        torch.cuda.synchronize()
        info = ctx.sim_info()
        assert info["substep"] == s
        rebuilt = info["tree_builds"] > builds
        builds = info["tree_builds"]
        if not (rebuilt or s in (5, 6)):
            continue
        shadow = st._shadow(st.predict(s))
        if rebuilt:
            say(f"  sub-step {s}: new tree")
            k, _ = oracle.keys(shadow, 0)
            ks_t, perm_t = oracle.sort(k)
            tree_t = oracle.build(ks_t, 16)
            ks, perm, _ = ctx.keys()
            assert np.array_equal(ks, ks_t) and np.array_equal(perm, perm_t)
            t = ctx.tree()
            for f in ("first", "count", "child_first", "n_child", "level"):
                assert np.array_equal(t[f], tree_t[f]), f
        # the float32 prediction in key order, bit for bit (Section 2.7's
        # predictor, masses carried unchanged)
        assert np.array_equal(ctx.positions(), shadow[perm_t])
        act = st.due(s)
        G = table[min((s & -s).bit_length() - 1, kmax)]
        ps = shadow[perm_t].astype(np.float64)
        mom = oracle.moments(tree_t, ps)
        grp = oracle.groups(act[perm_t].astype(np.uint8), ps, G, rc, oracle.BALL_EBS)
        ng = grp["first"].size
        assert ng == ctx.stats()["n_groups"] and act.sum() == ctx.stats()["n_active"]
        sel = np.unique(np.r_[rng.choice(ng, min(40, ng), replace=False),
                              np.argsort(-grp["ball"][:, 3])[:8]])
        out, _, last_gpu = ctx.sim_state()
        assert np.array_equal(last_gpu == s, act)
        gate_forces(ctx, oracle_parts(tree_t, mom, ps, grp, perm_t), out, act, eps, theta, 2,
                    sel=sel, label=f"sub-step {s} ({'new' if rebuilt else 'reused'} tree, "
                                   f"{int(act.sum())} due, groups of <= {G}): ")
        checked.append((s, rebuilt))
        if s >= 6 and any(r for _, r in checked):
            break
    say(f"  checked sub-steps (sub-step, new tree): {checked}")
    assert ctx.stats()["sticky_flags"] == 0
    assert {5, 6} <= {c[0] for c in checked}
    assert any(r for _, r in checked), "no tree built in 24 sub-steps"


@functools.lru_cache(maxsize=1)
def _galaxy_reference():
    n, eps = 1 << 22, 1 / 256
    x = ics.galaxy(n)
    rng = np.random.default_rng(304)
    sub = rng.choice(n, 4096, replace=False)
    say("  oracle direct sum on 4096 particles")
    d = oracle.direct(x, eps, idx=sub)
    say("  oracle tree on the groups of the sample")
    ks_o, perm_o, tree, ps, mom, rc = _oracle_prep(x, 16, 32, -0.0625)
    grp = oracle.groups(np.ones(n, np.uint8), ps, 32, rc)
    inv = np.empty(n, np.int64)
    inv[perm_o] = np.arange(n)
    sel = np.unique(np.searchsorted(grp["first"], inv[sub], side="right") - 1)
    return x, sub, d, oracle_parts(tree, mom, ps, grp, perm_o), sel


@pytest.mark.parametrize("compensated", [0, 1])
def test_galaxy4m_fp32_and_compensated(compensated):
    eps, theta = 1 / 256, 0.5
    say(f"[gpu] galaxy 2^22 monopole compensated={compensated}")
    x, sub, d, parts, sel = _galaxy_reference()
    ctx = g.Context(device=0, multipole=1, compensated=compensated)
    out = ctx.tree_forces(torch.from_numpy(x).cuda(), eps, theta).cpu().numpy()
    err_direct = np.linalg.norm(out[sub, :3] - d[:, :3], axis=1) / np.linalg.norm(d[:, :3], axis=1)
    r = gate_forces(ctx, parts, out, np.ones(x.shape[0], bool), eps, theta, 1, sel=sel,
                    label=f"vs float64 tree ({sel.size} groups): ")
    say(f"  compensated={compensated}: vs float64 tree rms acc {r['e_acc']:.2e} pot "
        f"{r['e_pot']:.2e}; vs float64 direct sum on 4096 particles: "
        f"p50 {np.median(err_direct):.2e} p99 {np.percentile(err_direct, 99):.2e} "
        f"rms {rel_rms(out[sub], d):.2e}")
    # truncation error of theta = 0.5 monopoles (about 1e-3 typical)
    assert np.median(err_direct) < 3e-3 and rel_rms(out[sub], d) < 1e-2


def test_nfw1m_block_levels():
    n, eps, theta, eta, kmax = 1 << 20, 1 / 128, 0.5, 0.1, 8
    say("[gpu] NFW 2^20 quadrupole block levels")
    x, v = ics.nfw(n, seed=201, with_vel=True)
    ctx = g.Context(device=0, multipole=2, r_crit=0.5)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=eta, kmax=kmax)
    info = ctx.sim_info()
    acc, lev, _ = ctx.sim_state()
    ks_o, perm_o, tree, ps, mom, rc = _oracle_prep(x, 16, 32, 0.5)
    grp = oracle.groups(np.ones(n, np.uint8), ps, 32, rc)
    rng = np.random.default_rng(6)
    sel = rng.choice(grp["first"].size, 64, replace=False)
    # the t = 0 forces (the bind's evaluation is the context's last one)
    r = gate_forces(ctx, oracle_parts(tree, mom, ps, grp, perm_o), acc, np.ones(n, bool), eps,
                    theta, 2, sel=sel, label="t = 0 forces, 64 sampled groups: ")
    e_acc = r["e_acc"]
    ref_sorted, cnt, _ = oracle.walk(tree, mom, ps, grp, eps, theta, 2, gsel=sel, **tie_params())
    clean = cnt[sel, 2] == 0
    rows = np.concatenate([grp["alist"][grp["first"][q]:grp["first"][q] + grp["count"][q]]
                           for q in sel[clean]])
    # levels from the oracle's accelerations on the sampled rows
    dt_o = I.timestep(ref_sorted[rows, :3], eps, eta)
    dt_all_gpu = I.timestep(acc[:, :3].astype(np.float64), eps, eta)
    assert info["dt_fine"] == I.anchor(dt_all_gpu)
    k_o = I.level_for(dt_o, info["dt_max"], kmax)
    r = np.log2(info["dt_max"] / dt_o)
    away = np.abs(r - np.round(r)) > 1e-4
    lv = lev[perm_o[rows]]
    say(f"  rms acc {e_acc:.2e}; levels agree {np.mean(lv[away] == k_o[away]):.5f}; histogram "
        f"{[c for c in info['level_count'] if c]}")
    assert e_acc <= 1e-5
    assert np.array_equal(lv[away], k_o[away])
    assert sum(info["level_count"]) == n
