"""Tree reuse between rebuilds (Section 2.6) through the C ABI.

An evaluation on a reused tree walks the tree of the last build with the
current positions: the permutation and node membership are the old ones, and
moments, radii, groups and forces are recomputed.  The oracle does the same
from its own float64 tree of the old positions, so parity is checked at the
usual 1e-5.  A fixed interval rebuilds exactly every k evaluations; the
automatic interval (the paper's growth models) rebuilds sometimes, and the
block steps stay close to those with a new tree every sub-step.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, oracle_parts, rel_rms, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _oracle_on_old_tree(x_old, x_new, eps, theta, act, multipole, G=32, r_crit=-0.0625):
    k, cube = oracle.keys(x_old, 0)
    ks, perm = oracle.sort(k)
    tree = oracle.build(ks, 16)
    ps = x_new[perm].astype(np.float64)
    mom = oracle.moments(tree, ps)
    rc = float(np.float32(r_crit))
    rc = -rc * cube[3] if rc < 0 else rc
    grp = oracle.groups(act[perm], ps, G, rc)
    return oracle_parts(tree, mom, ps, grp, perm), ks, tree, mom


@pytest.mark.parametrize("multipole", [1, 2])
def test_reused_tree_matches_the_oracle(multipole):
    n, eps, theta = 20000, 1 / 128, 0.5
    x0, v = ics.nfw(n, seed=91, with_vel=True)
    act = ics.random_active(n, 0.5, seed=92)
    say(f"[gpu] reused tree, multipole={multipole}")
    ctx = g.Context(device=0, multipole=multipole, rebuild_interval=3)
    at = torch.from_numpy(act).cuda()
    xs = [x0]
    for step in range(1, 4):  # drift: a few per cent of the local spacing and more
        x = xs[-1].copy()
        x[:, :3] = (x[:, :3].astype(np.float64) + 0.02 * step * v).astype(np.float32)
        xs.append(x)
    keys = []
    for i, x in enumerate(xs):
        out = torch.full((n, 4), float("nan"), device="cuda")
        ctx.tree_forces(torch.from_numpy(x).cuda(), eps, theta, active=at, out=out)
        o = out.cpu().numpy()
        ks, perm, _ = ctx.keys()
        keys.append(ks.copy())
        built_from = xs[0] if i < 3 else xs[3]
        parts, ks_o, tree_o, mom_o = _oracle_on_old_tree(built_from, x, eps, theta, act,
                                                         multipole)
        assert np.array_equal(ks, ks_o) and np.array_equal(perm, parts["perm"]), i
        t = ctx.tree()
        assert np.array_equal(t["first"], tree_o["first"]), i
        # node radii of the (reused) tree at the current positions
        _, b, _ = ctx.nodes()
        scale = np.abs(mom_o[0][:, :3]).sum(1) + mom_o[1]
        assert np.all(np.abs(b - mom_o[1]) <= 1e-5 * mom_o[1] + 2e-6 * scale), i
        gate_forces(ctx, parts, o, act.astype(bool), eps, theta, multipole,
                    sel=np.arange(parts["groups"]["first"].size),
                    label=f"evaluation {i} ({'new' if i in (0, 3) else 'reused'} tree): ")
        assert np.all(np.isnan(o[act == 0]))
    assert np.array_equal(keys[0], keys[1]) and np.array_equal(keys[0], keys[2])
    assert not np.array_equal(keys[2], keys[3])


@pytest.mark.parametrize("graph", [0, 1])
def test_fixed_interval_in_block_steps(graph):
    kmax, k = 3, 4
    x, v = ics.plummer(8000, seed=93, with_vel=True)
    say(f"[gpu] block steps, rebuild every {k}, graph={graph}")
    res = []
    for interval in (1, k):
        ctx = g.Context(device=0, graph=graph, rebuild_interval=interval)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        ctx.sim_bind(pos, vel, mass, 1 / 64, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        ctx.sim_step(4 << kmax)
        info = ctx.sim_info()
        assert ctx.stats()["sticky_flags"] == 0
        res.append((info, pos.cpu().numpy()))
    (i1, p1), (ik, pk) = res
    assert i1["tree_builds"] == 4 << kmax
    # the bind built the first tree; then a new one every k sub-steps
    assert ik["tree_builds"] == (4 << kmax) // k
    dx = np.abs(pk - p1).max(1) / (np.abs(p1).max(1) + 1e-3)
    say(f"  builds {ik['tree_builds']} of {4 << kmax}; position difference p99 "
        f"{np.percentile(dx, 99):.2e}")
    assert np.percentile(dx, 99) < 1e-3


def test_graph_and_launched_steps_agree_with_reuse():
    kmax = 3
    x, v = ics.nfw(6000, seed=94, with_vel=True)
    say("[gpu] captured vs launched sub-steps with rebuild every 3")
    runs = []
    for graph in (0, 1):
        ctx = g.Context(device=0, graph=graph, multipole=2, rebuild_interval=3)
        pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
        vel = torch.from_numpy(v).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
        ctx.sim_bind(pos, vel, mass, 1 / 128, 0.5, eta=0.1, kmax=kmax)
        ctx.set_params(check=0)
        runs.append((ctx, pos, vel))
    for step in range(2 << kmax):
        for ctx, _, _ in runs:
            ctx.sim_step()
        torch.cuda.synchronize()
        assert torch.equal(runs[0][1], runs[1][1]) and torch.equal(runs[0][2], runs[1][2]), step


def test_automatic_interval():
    kmax = 3
    x, v = ics.nfw(30000, seed=95, with_vel=True)
    say("[gpu] automatic rebuild interval")
    ctx = g.Context(device=0, multipole=2, rebuild_interval=0)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    ctx.sim_bind(pos, vel, mass, 1 / 128, 0.5, eta=0.1, kmax=kmax)
    ctx.set_params(check=0)
    steps = 16 << kmax
    ctx.sim_step(steps)
    info = ctx.sim_info()
    say(f"  {info['tree_builds']} builds in {steps} sub-steps")
    assert ctx.stats()["sticky_flags"] == 0
    assert 1 <= info["tree_builds"] < steps
