"""Tuning (Section 2.4: r_crit by Brent's method on the measured time, kept
perturbed; plus the group size and list budget) through the C ABI.

Tuning chooses among configurations that are all exact evaluations of the
method, so the checks are: the choice is one of the candidates, the forces
of the chosen configuration match the float64 oracle run with the same
configuration, the cache answers a repeated bucket without timing, the
online tuner finishes searches while the block steps stay valid, and a
captured sub-step reads r_crit from device memory.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, rel_rms, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _oracle_gate(ctx, x, eps, theta, out, active, multipole=1, **kw):
    ref = oracle.tree_forces(x, eps, theta, active=active, multipole=multipole, **kw,
                             **tie_params())
    act = np.ones(x.shape[0], bool) if active is None else active.astype(bool)
    return gate_forces(ctx, ref, out, act, eps, theta, multipole)


def test_autotune_choice_cache_and_parity():
    n, eps, theta = 30000, 1 / 128, 0.5
    x = ics.nfw(n, seed=81)
    act = ics.random_active(n, 0.25, seed=82)
    xt = torch.from_numpy(x).cuda()
    at = torch.from_numpy(act).cuda()
    ctx = g.Context(device=0, multipole=2)
    out = torch.full((n, 4), float("nan"), device="cuda")
    say("[gpu] autotune NFW 30000, 25% active")
    res = ctx.autotune(xt, eps, theta, active=at, out=out)
    say(f"  {res}")
    shapes = {(8, 64), (16, 64), (32, 64), (64, 64), (4, 16), (8, 16), (8, 32), (16, 32)}
    assert (res["group_size"], res["walk_width"]) in shapes
    assert res["list_depth"] in (128, 256, 384, 512, 768)
    assert res["r_crit"] < 0 and res["evaluations"] > 80 and res["ms"] > 0
    p = ctx.params
    assert (p["group_size"], p["walk_width"], p["list_depth"]) == \
        (res["group_size"], res["walk_width"], res["list_depth"])
    assert p["r_crit"] == pytest.approx(res["r_crit"])
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[act == 0])) and np.all(np.isfinite(o[act == 1]))
    _oracle_gate(ctx, x, eps, theta, o, act, multipole=2, group_size=res["group_size"],
                 r_crit=res["r_crit"])
    # same bucket: from the cache, identical choice
    res2 = ctx.autotune(xt, eps, theta, active=at, out=out)
    assert res2["evaluations"] == 0
    assert (res2["group_size"], res2["walk_width"], res2["list_depth"], res2["r_crit"]) == \
        (res["group_size"], res["walk_width"], res["list_depth"], res["r_crit"])
    # another active fraction is another bucket
    res3 = ctx.autotune(xt, eps, theta, out=out)
    assert res3["evaluations"] > 0


@pytest.mark.parametrize("graph", [0, 1])
def test_online_rcrit_tuning_in_block_steps(graph):
    kmax = 3
    x, v = ics.nfw(20000, seed=83, with_vel=True)
    say(f"[gpu] online r_crit tuning, graph={graph}")
    runs = []
    for tune in (0, 1):
        ctx = g.Context(device=0, multipole=2, graph=graph, autotune=tune)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        ctx.sim_bind(pos, vel, mass, 1 / 128, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_step(16 << kmax)
        torch.cuda.synchronize()
        assert ctx.stats()["sticky_flags"] == 0
        runs.append((ctx, pos.cpu().numpy(), vel.cpu().numpy()))
    (c0, p0, _), (c1, p1, _) = runs
    r, k = c1.sim_tuning(kmax + 1)
    say(f"  searches per class {k.tolist()}, best r_crit {r.tolist()}")
    assert k[0] >= 2 and k[1] >= 1
    assert np.all(r[k > 0] < 0)
    # the tuned run follows the untuned one (different groups only change the
    # truncation error of the tree force)
    dx = np.abs(p1 - p0).max(1) / (np.abs(p0).max(1) + 1e-3)
    say(f"  position difference to the untuned run: p99 {np.percentile(dx, 99):.2e}")
    assert np.percentile(dx, 99) < 1e-3
    i0, i1 = c0.sim_info(), c1.sim_info()
    assert i0["substep"] == i1["substep"] == 16 << kmax


def test_captured_step_reads_rcrit_from_device():
    kmax = 3
    x, v = ics.plummer(5000, seed=84, with_vel=True)
    say("[gpu] r_crit changed between replays without re-capture")
    runs = []
    for graph in (0, 1):
        ctx = g.Context(device=0, graph=graph, r_crit=-0.0625)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        ctx.sim_bind(pos, vel, mass, 1 / 64, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        runs.append((ctx, pos, vel))
    groups = []
    for phase, rc in enumerate((-0.0625, 0.02, -0.0625)):
        for ctx, _, _ in runs:
            ctx.set_params(r_crit=rc)
        for step in range(1 << kmax):
            for ctx, _, _ in runs:
                ctx.sim_step()
            torch.cuda.synchronize()
            (c0, p0, v0), (c1, p1, v1) = runs
            assert torch.equal(p0, p1) and torch.equal(v0, v1), (phase, step)
        groups.append(runs[1][0].stats()["n_groups"])
    say(f"  groups at the last sub-step of each phase {groups}")
    assert groups[1] != groups[0] and groups[2] == groups[0]


def _bound(x, v, eps, **kw):
    ctx = g.Context(device=0, multipole=2, **kw)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    return ctx, pos, vel, mass


def _rewalk_reproduces(ctx, k=8):
    """The forces the list read-back's walk writes for k groups of the last
    evaluation are that evaluation's, bit for bit."""
    gg = ctx.groups()
    _, perm, _ = ctx.keys()
    acc, _, _ = ctx.sim_state()
    pick = np.unique(np.linspace(0, gg["first"].size - 1, k).astype(np.int64))
    _, rewalk = ctx.lists(pick)
    for q in pick:
        rows = perm[gg["alist"][gg["first"][q]:gg["first"][q] + gg["count"][q]]]
        assert rows.size and np.array_equal(rewalk[rows], acc[rows]), q


def test_group_size_per_class_replays_equal_launches():
    """A group shape per sub-step class (G i-particles walked by W lanes, S =
    W / G lanes per i-particle): captured sub-steps with one groups + walk
    graph per shape give the launched sub-steps bit for bit, and the table is
    what the classes use."""
    kmax = 3
    x, v = ics.plummer(6000, seed=85, with_vel=True)
    table = [8, 64, 16, 8]
    widths = [16, 64, 32, 64]
    say(f"[gpu] group sizes per class {table}, walk widths {widths}, graph vs launched")
    runs = []
    for graph in (0, 1):
        ctx, pos, vel, mass = _bound(x, v, 1 / 64, graph=graph)
        ctx.sim_bind(pos, vel, mass, 1 / 64, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_set_group_sizes(table, widths)
        runs.append((ctx, pos, vel))
    _, _, gs, ws = runs[1][0].sim_tuning(kmax + 2, with_groups=True)
    assert gs.tolist() == table + [32] and ws.tolist() == widths + [64]
    for step in range(3 << kmax):
        for ctx, _, _ in runs:
            ctx.sim_step()
        torch.cuda.synchronize()
        (c0, p0, v0), (c1, p1, v1) = runs
        assert torch.equal(p0, p1) and torch.equal(v0, v1), step
        assert c0.stats()["n_groups"] == c1.stats()["n_groups"], step
    assert runs[1][0].stats()["sticky_flags"] == 0
    # a read-back that walks the groups again (gothic_get_lists) takes the
    # shape of the last evaluation, also when that was a replay: class 1 (G 64)
    # after the last capture (class 3, G 8)
    for _ in range(2):
        for ctx, _, _ in runs:
            ctx.sim_step()
    for ctx, _, _ in runs:
        _rewalk_reproduces(ctx)
    # the last sub-step of a cycle (every particle due) walks groups of the
    # size its class is given
    n_groups = []
    for size in (8, 64):
        ctx, pos, vel, mass = _bound(x, v, 1 / 64, graph=1)
        ctx.sim_bind(pos, vel, mass, 1 / 64, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_set_group_sizes([size] * (kmax + 1))
        ctx.sim_step(1 << kmax)
        st = ctx.stats()
        n_groups.append((st["n_groups"], st["n_active"]))
    say(f"  all-active sub-step with G = 8 / 64: (groups, active) {n_groups}")
    (g8, a8), (g64, a64) = n_groups
    assert a8 == a64 == x.shape[0] and g8 >= a8 // 8 and g64 < g8
    with pytest.raises(g.GothicError):
        runs[0][0].sim_set_group_sizes([12])
    with pytest.raises(g.GothicError):
        runs[0][0].sim_set_group_sizes([32], [16])  # more i-particles than lanes
    with pytest.raises(g.GothicError):
        runs[0][0].sim_set_group_sizes([8], [8])  # not a walk width


@pytest.mark.parametrize("graph", [0, 1])
def test_autotune_picks_group_size_per_class(graph):
    kmax = 3
    x, v = ics.nfw(20000, seed=86, with_vel=True)
    say(f"[gpu] autotune = 2 (group size per class, then r_crit), graph={graph}")
    runs = []
    for tune in (0, 2):
        ctx, pos, vel, mass = _bound(x, v, 1 / 128, graph=graph, autotune=tune)
        ctx.sim_bind(pos, vel, mass, 1 / 128, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_step(16 << kmax)
        torch.cuda.synchronize()
        assert ctx.stats()["sticky_flags"] == 0
        runs.append((ctx, pos.cpu().numpy()))
    (c0, p0), (c1, p1) = runs
    r, k, gs, ws = c1.sim_tuning(kmax + 1, with_groups=True)
    say(f"  group size per class {gs.tolist()}, walk width {ws.tolist()}, r_crit searches "
        f"{k.tolist()}")
    shapes = {(8, 64), (16, 64), (32, 64), (64, 64), (4, 16), (8, 16), (8, 32), (16, 32)}
    assert set(zip(gs.tolist(), ws.tolist())) <= shapes
    assert k[0] >= 1 and np.all(r[k > 0] < 0)
    dx = np.abs(p1 - p0).max(1) / (np.abs(p0).max(1) + 1e-3)
    say(f"  position difference to the untuned run: p99 {np.percentile(dx, 99):.2e}")
    assert np.percentile(dx, 99) < 1e-3


def test_group_sizes_with_batched_systems_and_errors():
    """Per-class group sizes and their picking also drive a batched block-step
    run (every system's groups use the class's size); bad arguments are
    refused without changing anything."""
    kmax = 3
    x, offs, eps, v = ics.batched_systems(5, seed=87, lg_min=10, lg_max=13, with_vel=True)
    say(f"[gpu] batched systems n={x.shape[0]}: autotune = 2, graph vs launched with one table")
    runs = []
    for graph in (0, 1):
        ctx = g.Context(device=0, graph=graph)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v.astype(np.float64)).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        ctx.sim_bind_batched(pos, vel, mass, offs, eps, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_set_group_sizes([16, 64, 8, 32])
        runs.append((ctx, pos, vel))
    for step in range(2 << kmax):
        for ctx, _, _ in runs:
            ctx.sim_step()
        torch.cuda.synchronize()
        (_, p0, v0), (_, p1, v1) = runs
        assert torch.equal(p0, p1) and torch.equal(v0, v1), step
    ctx = runs[1][0]
    assert ctx.stats()["sticky_flags"] == 0
    with pytest.raises(g.GothicError):
        ctx.sim_set_group_sizes([0] * 33)  # more classes than there are
    with pytest.raises(g.GothicError):
        ctx.sim_set_group_sizes([32, 128])  # not a size the walk has
    _, _, gs, ws = ctx.sim_tuning(4, with_groups=True)
    assert gs.tolist() == [16, 64, 8, 32]  # unchanged by the refused calls
    assert ws.tolist() == [64] * 4
    with pytest.raises(g.GothicError):
        ctx.sim_tuning(33)
    # autotune = 2 on the batched run: sizes picked from the candidates
    ctx2 = g.Context(device=0, graph=1, autotune=2)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v.astype(np.float64)).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    ctx2.sim_bind_batched(pos, vel, mass, offs, eps, 0.5, eta=0.1, kmax=kmax)
    ctx2.set_params(check=0)
    ctx2.sim_step(16 << kmax)
    torch.cuda.synchronize()
    assert ctx2.stats()["sticky_flags"] == 0
    _, _, gs2, ws2 = ctx2.sim_tuning(kmax + 1, with_groups=True)
    say(f"  picked group sizes per class {gs2.tolist()}, walk widths {ws2.tolist()}")
    assert set(gs2.tolist()) <= {4, 8, 16, 32, 64} and set(ws2.tolist()) <= {16, 32, 64}
