"""Batched evaluation of many systems and captured sub-steps (through the C ABI).

A batched evaluation must give every system exactly what a call on that
system alone gives: the same keys, permutation (offset by the system's first
row), key cube, tree and groups, hence bit-identical forces; and those match
the float64 oracle run on each system separately.  A block-step driver over
several systems must follow each system's own oracle integrator.  A captured
sub-step (params.graph) must reproduce the launched one bit for bit on every
replay.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, rel_rms, say, tie_params
from oracle import integrate as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _mixed_batch():
    """Seven systems: sizes from one particle to a few thousand, one empty,
    Plummer and NFW, different softenings and opening angles."""
    parts = [ics.plummer(3000, seed=51), ics.nfw(1, seed=52), np.zeros((0, 4), np.float32),
             ics.nfw(4097, seed=53), ics.plummer(2, seed=54), ics.plummer(17, seed=55),
             ics.nfw(2500, seed=56)]
    eps = np.array([1 / 64, 1 / 128, 0.1, 1 / 128, 1 / 64, 1 / 32, 1 / 100], np.float32)
    theta = np.array([0.5, 0.5, 0.5, 0.6, 0.3, 0.5, 0.7], np.float32)
    offs = np.zeros(len(parts) + 1, np.int64)
    offs[1:] = np.cumsum([p.shape[0] for p in parts])
    return np.concatenate(parts), offs, eps, theta


def _tree_of_system(t, lo, hi):
    """The nodes of the system owning rows [lo, hi) in their combined
    breadth-first order, with child indices renumbered to the system."""
    sel = np.flatnonzero((t["first"] >= lo) & (t["first"] < hi) & (t["count"] > 0))
    local = np.full(t["first"].size, -1, np.int64)
    local[sel] = np.arange(sel.size)
    cf = t["child_first"][sel].astype(np.int64)
    has = t["n_child"][sel] > 0
    cf[has] = local[cf[has]]
    return dict(first=t["first"][sel] - lo, count=t["count"][sel], child_first=cf,
                n_child=t["n_child"][sel], level=t["level"][sel])


@pytest.mark.parametrize("multipole", [1, 2])
def test_batched_equals_single_system_calls(multipole):
    x, offs, eps, theta = _mixed_batch()
    n = x.shape[0]
    act = ics.random_active(n, 0.4, seed=57)
    act[offs[3]] = 1
    say(f"[gpu] batched 7 systems n={n} multipole={multipole}")
    ctx = g.Context(device=0, multipole=multipole)
    xt = torch.from_numpy(x).cuda()
    at = torch.from_numpy(act).cuda()
    out = torch.full((n, 4), float("nan"), device="cuda")
    ctx.tree_forces_batched(xt, offs, eps, theta, active=at, out=out)
    ob = out.cpu().numpy()
    st = ctx.stats()
    ks, perm, cubes = ctx.keys()
    t = ctx.tree()
    assert st["n_systems"] == 6 and cubes.shape == (6, 4)
    single = g.Context(device=0, multipole=multipole)
    k = 0
    for s in range(len(offs) - 1):
        lo, hi = int(offs[s]), int(offs[s + 1])
        if hi == lo:
            continue
        xs = x[lo:hi]
        # bit-exact keys, permutation, cube and tree against the oracle
        k_o, cube_o = oracle.keys(xs, 0)
        ks_o, perm_o = oracle.sort(k_o)
        assert np.array_equal(ks[lo:hi], ks_o), s
        assert np.array_equal(perm[lo:hi].astype(np.int64) - lo, perm_o), s
        assert np.array_equal(cubes[k], cube_o), s
        t_o = oracle.build(ks_o, 16)
        ts = _tree_of_system(t, lo, hi)
        for f in ("first", "count", "child_first", "n_child", "level"):
            assert np.array_equal(ts[f], t_o[f]), (s, f)
        k += 1
        # the same system alone: identical forces, bit for bit
        o1 = torch.full((hi - lo, 4), float("nan"), device="cuda")
        single.tree_forces(xt[lo:hi].contiguous(), float(eps[s]), float(theta[s]),
                           active=at[lo:hi].contiguous(), out=o1)
        o1 = o1.cpu().numpy()
        assert np.array_equal(np.isnan(o1), np.isnan(ob[lo:hi])), s
        assert np.array_equal(o1[~np.isnan(o1)], ob[lo:hi][~np.isnan(o1)]), s
        # and the float64 oracle on the system alone
        ref = oracle.tree_forces(xs, float(eps[s]), float(theta[s]), active=act[lo:hi],
                                 multipole=multipole, **tie_params())
        a = act[lo:hi].astype(bool)
        if a.any():  # the single call (identical to the batched one) against the oracle
            gate_forces(single, ref, o1, a, float(eps[s]), float(theta[s]), multipole,
                        label=f"system {s}: n={hi - lo} active={a.sum()} ")
    assert np.all(np.isnan(ob[~act.astype(bool)]))


def test_batched64_configuration():
    x, offs, eps = ics.batched_systems(64, seed=401)
    n = x.shape[0]
    say(f"[gpu] 64 systems, n={n}")
    ctx = g.Context(device=0)
    xt = torch.from_numpy(x).cuda()
    ob = ctx.tree_forces_batched(xt, offs, eps, 0.5).cpu().numpy()
    assert ctx.stats()["n_systems"] == 64
    single = g.Context(device=0)
    for s in range(64):
        lo, hi = int(offs[s]), int(offs[s + 1])
        o1 = single.tree_forces(xt[lo:hi].contiguous(), float(eps[s]), 0.5).cpu().numpy()
        assert np.array_equal(o1, ob[lo:hi]), s
    # oracle parity on the smallest, a middle and the largest system
    sizes = np.diff(offs)
    for s in (int(np.argmin(sizes)), int(np.argsort(sizes)[32]), int(np.argmax(sizes))):
        lo, hi = int(offs[s]), int(offs[s + 1])
        # the single call on the system (bit-identical to the batched rows, as
        # checked above) against the oracle, every row
        o1 = single.tree_forces(xt[lo:hi].contiguous(), float(eps[s]), 0.5).cpu().numpy()
        assert np.array_equal(o1, ob[lo:hi]), s
        ref = oracle.tree_forces(x[lo:hi], float(eps[s]), 0.5, **tie_params())
        gate_forces(single, ref, o1, np.ones(hi - lo, bool), float(eps[s]), 0.5, 1,
                    label=f"system {s}: n={hi - lo} ")


def _tree_force(eps, theta):
    def f(xyzm, active):
        return oracle.tree_forces(xyzm, eps, theta, active=active)["acc_pot"]
    return f


def test_batched_block_steps_follow_each_system():
    kmax, eta, theta = 4, 0.1, 0.5
    sys = [(ics.plummer(2048, seed=61, with_vel=True), 1 / 64),
           (ics.nfw(3000, seed=62, with_vel=True), 1 / 128),
           (ics.plummer(700, seed=63, with_vel=True), 1 / 32)]
    xs = [s[0][0] for s in sys]
    vs = [s[0][1] for s in sys]
    eps = np.array([s[1] for s in sys], np.float32)
    offs = np.zeros(4, np.int64)
    offs[1:] = np.cumsum([x.shape[0] for x in xs])
    x = np.concatenate(xs)
    v = np.concatenate(vs)
    say(f"[gpu] batched block steps, 3 systems n={x.shape[0]}")
    ctx = g.Context(device=0)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v.astype(np.float64)).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    ctx.sim_bind_batched(pos, vel, mass, offs, eps, theta, eta=eta, kmax=kmax)
    sims = [I.BlockSim(xs[k], vs[k], float(eps[k]), eta, kmax, _tree_force(float(eps[k]), theta))
            for k in range(3)]
    dtf, dtm = ctx.sim_steps()
    for k in range(3):
        assert dtf[k] == sims[k].dt_fine and dtm[k] == sims[k].dt_max, k
    active_o = 0
    for _ in range(1 << kmax):
        for sim in sims:
            active_o += int(sim.step().sum())
    ctx.sim_step(1 << kmax)
    info = ctx.sim_info()
    _, lev, last = ctx.sim_state()
    p = pos.cpu().numpy()
    q = vel.cpu().numpy()
    assert info["substep"] == 1 << kmax
    assert abs(info["active_total"] - active_o) <= 0.01 * active_o + 5
    for k in range(3):
        lo, hi = int(offs[k]), int(offs[k + 1])
        same = lev[lo:hi] == sims[k].k
        dx = np.abs(p[lo:hi] - sims[k].x).max(1) / (np.abs(sims[k].x).max(1) + 1e-3)
        dv = np.abs(q[lo:hi] - sims[k].v).max(1) / (np.abs(sims[k].v).max(1) + 1e-3)
        say(f"  system {k}: levels agree {same.mean():.5f}, dpos p99 {np.percentile(dx, 99):.2e}")
        assert same.mean() > 0.995
        assert np.all(last[lo:hi] == 1 << kmax)
        assert np.percentile(dx, 99) < 1e-5 and np.percentile(dv, 99) < 1e-4


@pytest.mark.parametrize("batched", [False, True])
def test_captured_substeps_replay_the_launched_ones(batched):
    kmax, eta = 3, 0.1
    if batched:
        x, offs, eps, v = ics.batched_systems(5, seed=71, lg_min=10, lg_max=13, with_vel=True)
    else:
        x, v = ics.plummer(6000, seed=73, with_vel=True)
    say(f"[gpu] graph vs launched sub-steps, batched={batched}, n={x.shape[0]}")
    runs = []
    for graph in (0, 1):
        ctx = g.Context(device=0, graph=graph, multipole=2, timing=1)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v.astype(np.float64)).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        if batched:
            ctx.sim_bind_batched(pos, vel, mass, offs, eps, 0.5, eta=eta, kmax=kmax)
        else:
            ctx.sim_bind(pos, vel, mass, 1 / 64, 0.5, eta=eta, kmax=kmax)
        ctx.set_params(check=0)
        ctx.walk_time()  # drop the bind's evaluation
        runs.append((ctx, pos, vel))
    (c0, p0, v0), (c1, p1, v1) = runs
    for step in range(3 << kmax):
        c0.sim_step()
        c1.sim_step()
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.equal(p0, p1) and torch.equal(v0, v1), step
        assert float(junk) == float(junk)
    s0, s1 = c0.sim_state(), c1.sim_state()
    for a, b in zip(s0, s1):
        assert np.array_equal(a, b)
    i0, i1 = c0.sim_info(), c1.sim_info()
    assert i0["interactions_total"] == i1["interactions_total"] > 0
    assert i0["active_total"] == i1["active_total"]
    assert c1.stats()["sticky_flags"] == 0
    ms, k = c1.walk_time()
    assert k == 3 << kmax and ms > 0


def test_tree_forces_inside_a_user_graph_capture():
    """A caller captures one evaluation into its own HIP graph (after one
    uncaptured call of the same size sized the scratch) and replays it on new
    positions: every replay, with unrelated eager work and a synchronisation
    in between, equals an eager evaluation of the same input bit for bit."""
    n, eps, theta = 6000, 1 / 64, 0.5
    xs = [ics.plummer(n, seed=s) for s in (91, 92, 93)]
    say(f"[gpu] tree_forces captured by the caller, n={n}, 3 replays")
    ctx = g.Context(device=0, multipole=2, check=0)
    xt = torch.from_numpy(xs[0]).cuda()
    out = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    ctx.tree_forces(xt, eps, theta, out=out)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=side):
        ctx.tree_forces(xt, eps, theta, out=out)
    ref_ctx = g.Context(device=0, multipole=2)
    for k, x in enumerate(xs + xs[:1]):
        xt.copy_(torch.from_numpy(x).cuda())
        out.fill_(float("nan"))
        graph.replay()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        ref = ref_ctx.tree_forces(torch.from_numpy(x).cuda(), eps, theta)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
        assert float(junk) == float(junk)
