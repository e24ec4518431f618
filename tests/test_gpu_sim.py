"""GPU block-step driver against the float64 oracle integrator (through the C ABI).

Both sides start from the same float32/float64 state; the oracle takes its
forces from its own float64 tree, the library from its float32 tree, so the
trajectories agree to single-precision force accuracy.  Integer results
(anchored steps, levels, last-update sub-steps) must agree exactly except for
particles whose step sits within a relative 1e-4 of a level boundary.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import say
from oracle import integrate as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def _tree_force(eps, theta, **kw):
    def f(xyzm, active):
        return oracle.tree_forces(xyzm, eps, theta, active=active, **kw)["acc_pot"]
    return f


def _near_boundary(sim_o, a3):
    dt = I.timestep(a3, sim_o.eps, sim_o.eta)
    r = np.log2(sim_o.dt_max / dt)
    return np.abs(r - np.round(r)) < 2e-4


def _gpu_sim(x, v, eps, theta, eta, kmax, shared, **params):
    import paper_1610_07279_amd as g
    ctx = g.Context(device=0, **params)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda().contiguous()
    vel = torch.from_numpy(v.astype(np.float64)).cuda().contiguous()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    say(f"[gpu] sim n={x.shape[0]} eps={eps} theta={theta} kmax={kmax} shared={shared} {params}")
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=eta, kmax=kmax, shared=shared)
    return ctx, pos, vel


@pytest.mark.parametrize("shared", [False, True])
def test_block_steps_match_oracle(shared):
    n, eps, theta, eta, kmax = 4096, 1 / 64, 0.5, 0.1, 4
    x, v = ics.plummer(n, seed=31, with_vel=True)
    sim_o = I.BlockSim(x, v, eps, eta, kmax, _tree_force(eps, theta), shared=shared)
    ctx, pos, vel = _gpu_sim(x, v, eps, theta, eta, kmax, shared)
    info = ctx.sim_info()
    assert info["dt_fine"] == sim_o.dt_fine and info["dt_max"] == sim_o.dt_max
    _, lev0, _ = ctx.sim_state()
    nb0 = _near_boundary(sim_o, sim_o.a)
    assert np.array_equal(lev0[~nb0], sim_o.k[~nb0])
    active_o = 0
    for _ in range(1 << kmax):
        active_o += int(sim_o.step().sum())
    ctx.sim_step(1 << kmax)
    info = ctx.sim_info()
    acc, lev, last = ctx.sim_state()
    assert info["substep"] == sim_o.s == 1 << kmax
    same = lev == sim_o.k
    say(f"  levels agree {same.mean():.5f}; active {info['active_total']} vs {active_o}")
    assert same.mean() > 0.995
    # after a full cycle every particle is synchronised on both sides
    assert np.all(last == sim_o.s) and np.all(sim_o.si == sim_o.s)
    p = pos.cpu().numpy()
    q = vel.cpu().numpy()
    dx = np.abs(p - sim_o.x).max(1) / (np.abs(sim_o.x).max(1) + 1e-3)
    dv = np.abs(q - sim_o.v).max(1) / (np.abs(sim_o.v).max(1) + 1e-3)
    say(f"  max rel dpos {dx.max():.2e} dvel {dv.max():.2e}")
    assert np.percentile(dx, 99) < 1e-5 and np.percentile(dv, 99) < 1e-4
    assert abs(info["active_total"] - active_o) <= 0.01 * active_o + 5
    if shared:
        assert info["active_total"] == n << kmax


def test_sim_energy_and_counts():
    n, eps, theta, eta, kmax = 8192, 1 / 64, 0.5, 0.1, 3
    x, v = ics.plummer(n, seed=32, with_vel=True)
    ctx, pos, vel = _gpu_sim(x, v, eps, theta, eta, kmax, False, timing=1)
    ctx.sim_reset_counters()
    ctx.walk_time()
    ctx.sim_step(1 << kmax)
    info = ctx.sim_info()
    ms, k = ctx.walk_time()
    assert k == 1 << kmax and ms > 0
    assert info["steps"] == 1 << kmax
    assert info["interactions_total"] > 0 and info["active_total"] >= n
    assert sum(info["level_count"]) == n


def test_sim_argument_errors():
    import paper_1610_07279_amd as g
    ctx = g.Context(device=0)
    with pytest.raises(g.GothicError):
        ctx._sim_keep = (torch.zeros((1, 3), dtype=torch.float64, device="cuda"),)
        ctx.sim_step()
    x, v = ics.plummer(100, seed=33, with_vel=True)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    for kw in (dict(eta=0.0), dict(kmax=31), dict(kmax=-1)):
        with pytest.raises(g.GothicError) as e:
            ctx.sim_bind(pos, vel, mass, 0.01, 0.5, **kw)
        assert e.value.code == g.EINVAL
