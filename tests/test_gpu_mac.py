"""The acceleration and multipole MACs of Section 2.2 (params.mac) against the
float64 oracle, through the C ABI.

The acceleration MAC reads the previous accelerations; both sides get the
same float32 array (here the forces of an opening-angle evaluation).  Lists
are compared for groups without a near tie (a decision that changes within
single-precision rounding of the distance); the lists of groups with one are
read back and each decision checked by the oracle; forces of every active
particle at the usual 1e-5 (gpu_util.gate_forces).
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, rel_rms, run_gpu, say, tie_params
from oracle import integrate as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _mac_parity(x, eps, mac, delta, multipole=1, active=None, G=32):
    n = x.shape[0]
    _, a_old = run_gpu(x, eps, 0.5, multipole=multipole)  # previous accelerations
    a_old = np.ascontiguousarray(a_old, np.float32)
    say(f"[gpu] mac={mac} delta={delta} multipole={multipole} n={n}")
    ctx = g.Context(device=0, mac=mac, mac_delta=delta, multipole=multipole, group_size=G)
    xt = torch.from_numpy(x).cuda()
    at = None if active is None else torch.from_numpy(active).cuda()
    out = torch.full((n, 4), float("nan"), device="cuda")
    ctx.tree_forces(xt, eps, 0.5, active=at, out=out,
                    acc_old=torch.from_numpy(a_old).cuda() if mac == 1 else None)
    o = out.cpu().numpy()
    ref = oracle.tree_forces(x, eps, 0.5, active=active, multipole=multipole, group_size=G,
                             mac=mac, delta=delta, acc_old=a_old, **tie_params())
    act = np.ones(n, bool) if active is None else active.astype(bool)
    gate_forces(ctx, ref, o, act, eps, 0.5, multipole, mac=mac, delta=delta, acc_old=a_old,
                label=f"mac {mac}: ")
    return o, ref


@pytest.mark.parametrize("multipole", [1, 2])
@pytest.mark.parametrize("delta", [2.0 ** -7, 1e-4])
def test_acceleration_mac(delta, multipole):
    x = ics.nfw(20000, seed=101)
    act = ics.random_active(20000, 0.4, seed=102)
    _mac_parity(x, 1 / 128, 1, delta, multipole, active=act)


@pytest.mark.parametrize("multipole", [1, 2])
@pytest.mark.parametrize("delta", [1e-2, 1e-4])
def test_multipole_mac(delta, multipole):
    x = ics.plummer(20000, seed=103)
    _mac_parity(x, 1 / 64, 2, delta, multipole)


@pytest.mark.parametrize("mac", [1, 2])
def test_tiny_delta_is_the_direct_sum(mac):
    x = ics.plummer(4096, seed=104)
    d = oracle.direct(x, 1 / 64)
    o, _ = _mac_parity(x, 1 / 64, mac, 1e-20, 1, G=8)
    assert rel_rms(o, d) <= 1e-5 and rel_rms(o, d, cols=slice(3, 4)) <= 1e-5


def test_acceleration_mac_block_steps():
    n, eps, theta, eta, kmax, delta = 4096, 1 / 64, 0.5, 0.1, 4, 2.0 ** -7
    x, v = ics.plummer(n, seed=105, with_vel=True)
    holder = {}

    def force(xyzm, active):
        sim = holder.get("sim")
        if sim is None:  # t = 0: no previous accelerations yet, the opening angle
            return oracle.tree_forces(xyzm, eps, theta, active=active)["acc_pot"]
        return oracle.tree_forces(xyzm, eps, theta, active=active, mac=1, delta=delta,
                                  acc_old=sim.a.astype(np.float32))["acc_pot"]
    sim_o = I.BlockSim(x, v, eps, eta, kmax, force)
    holder["sim"] = sim_o
    say("[gpu] acceleration MAC in block steps")
    ctx = g.Context(device=0, mac=1, mac_delta=delta)
    pos = torch.from_numpy(x[:, :3].astype(np.float64)).cuda()
    vel = torch.from_numpy(v).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).cuda()
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=eta, kmax=kmax)
    for _ in range(1 << kmax):
        sim_o.step()
    ctx.sim_step(1 << kmax)
    _, lev, last = ctx.sim_state()
    p = pos.cpu().numpy()
    dx = np.abs(p - sim_o.x).max(1) / (np.abs(sim_o.x).max(1) + 1e-3)
    say(f"  levels agree {(lev == sim_o.k).mean():.5f}, dpos p99 {np.percentile(dx, 99):.2e}")
    assert (lev == sim_o.k).mean() > 0.99
    assert np.percentile(dx, 99) < 1e-5


def test_mac_argument_errors():
    for bad in (dict(mac=3), dict(mac=1, mac_delta=0.0), dict(mac=2, mac_delta=float("nan"))):
        with pytest.raises(g.GothicError) as e:
            g.Context(device=0, **bad)
        assert e.value.code == g.EINVAL
    ctx = g.Context(device=0, mac=1)
    x = torch.from_numpy(ics.plummer(100, seed=106)).cuda()
    with pytest.raises(g.GothicError) as e:
        ctx.tree_forces(x, 0.01, 0.5)   # no previous accelerations
    assert e.value.code == g.EINVAL
