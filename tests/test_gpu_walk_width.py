"""Walk width W < 64 (the paper's T_sub of Table 2, the threads that share one
traversal): a wave64 walks 64 / W groups side by side, each with W lanes and
S = W / G lanes per i-particle.  Every shape is held to the same bar as the
one-group-per-wave walk: per-group list lengths bit-exact for groups without a
MAC near tie, the lists themselves for a sample, and forces within 1e-5 of a
float64 evaluation of the same lists (gpu_util.gate_forces, which also reads
the lists of near-tie groups back through the same kernel)."""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import diagnose_forces, gate_forces, run_gpu, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402


def _check(x, eps, theta, active=None, **params):
    ctx, out = run_gpu(x, eps, theta, active=active, **params)
    multipole = params.get("multipole", 1)
    ref = oracle.tree_forces(x, eps, theta, active=active, n_leaf=params.get("n_leaf", 16),
                             group_size=params.get("group_size", 32), multipole=multipole,
                             r_crit=params.get("r_crit", -0.0625), **tie_params())
    act = np.ones(x.shape[0], bool) if active is None else active.astype(bool)
    assert np.all(np.isnan(out[~act])), "inactive rows must stay untouched"
    assert np.all(np.isfinite(out[act]))
    try:
        errs = gate_forces(ctx, ref, out, act, eps, theta, multipole)
    except AssertionError:
        diagnose_forces(ctx, x, ref, out, act)
        raise
    st = ctx.stats()
    cnt = ref["counts"]
    if (cnt[:, 2] == 0).all():
        gg = ctx.groups()
        assert st["interactions"] == int(((cnt[:, 0] + cnt[:, 1]) * gg["count"]).sum())
    assert st["sticky_flags"] == 0
    say(f"  errors {errs}")
    return ctx, out


# (W, G): S = W / G in 1, 2, 4 (compile-time) and 16 (run-time)
SHAPES = [(16, 16), (16, 8), (16, 4), (16, 1), (32, 32), (32, 16), (32, 8), (32, 2)]


@pytest.mark.parametrize("W,G", SHAPES)
def test_walk_width_monopole(W, G):
    _check(ics.plummer(6000, seed=31), 1 / 64, 0.5, group_size=G, walk_width=W)


@pytest.mark.parametrize("W,G", [(16, 8), (32, 16), (32, 8)])
def test_walk_width_quadrupole(W, G):
    _check(ics.nfw(20000, seed=32), 1 / 128, 0.5, multipole=2, group_size=G, walk_width=W)


@pytest.mark.parametrize("W", [16, 32])
@pytest.mark.parametrize("depth", [64, 1024])
def test_walk_width_list_depths(W, depth):
    # depth 64: a walk of W lanes gets the smallest lists (one batch), so it
    # flushes after nearly every batch
    _check(ics.nfw(7000, seed=33), 1 / 128, 0.5, multipole=2, group_size=8, walk_width=W,
           list_depth=depth)


@pytest.mark.parametrize("W", [16, 32])
def test_walk_width_sparse_active_and_split_groups(W):
    x = ics.nfw(30000, seed=34)
    _check(x, 1 / 128, 0.5, active=ics.random_active(30000, 0.01, seed=35), group_size=8,
           walk_width=W, r_crit=0.05)


@pytest.mark.parametrize("name", ["one", "two", "coincident"])
def test_walk_width_edge_systems(name):
    if name == "coincident":
        x = ics.plummer(300, seed=3)
        x[10:60, :3] = x[9, :3]
    else:
        x = ics.plummer(1 if name == "one" else 2, seed=1)
    for W in (16, 32):
        _check(x, 1 / 64, 0.5, group_size=8, walk_width=W)


@pytest.mark.parametrize("W", [16, 32])
def test_walk_width_spill_overflow_grows_and_repeats(W):
    """The smallest pending stacks (256 entries per wave, 256 / (64 / W) per
    walk) on groups that span a whole uniform cube (1 particle in 64 active,
    no r_crit split): with check = 0 the walks overflow their global stacks
    and the sticky flag shows it; with check = 1 the stacks grow and the
    evaluation repeats, matching the oracle."""
    n = 1 << 16
    rng = np.random.default_rng(305)
    x = np.empty((n, 4), np.float32)
    x[:, :3] = rng.uniform(-1, 1, (n, 3))
    x[:, 3] = 1.0 / n
    act = np.zeros(n, np.uint8)
    act[rng.choice(n, n // 64, replace=False)] = 1
    eps, theta = 1 / 64, 0.3
    xt = torch.from_numpy(x).cuda()
    at = torch.from_numpy(act).cuda()
    say(f"[gpu] W={W}, spill_per_wave = 256, check = 0: the walks' stacks overflow")
    ctx = g.Context(device=0, group_size=W, walk_width=W, r_crit=0.0, spill_per_wave=256,
                    check=0)
    out = torch.full((n, 4), float("nan"), device="cuda")
    ctx.tree_forces(xt, eps, theta, active=at, out=out)
    st = ctx._stats_raw()
    say(f"  flags {st['flags']} sticky {st['sticky_flags']}")
    assert st["flags"] & 4 and st["sticky_flags"] & 4
    ctx.clear_flags()
    ctx.set_params(check=1)
    held0, _ = ctx.scratch()
    out.fill_(float("nan"))
    ctx.tree_forces(xt, eps, theta, active=at, out=out)
    st = ctx.stats()
    held1, _ = ctx.scratch()
    say(f"  check mode: flags {st['flags']} sticky {st['sticky_flags']}, scratch {held0} -> {held1}")
    assert st["flags"] == 0 and st["sticky_flags"] == 0 and held1 > held0
    ref = oracle.tree_forces(x, eps, theta, active=act, group_size=W, r_crit=0.0,
                             **tie_params())
    gate_forces(ctx, ref, out.cpu().numpy(), act.astype(bool), eps, theta, 1,
                label=f"W={W} grown stack: ")


def test_walk_width_argument_errors():
    with pytest.raises(g.GothicError):
        g.Context(device=0, group_size=32, walk_width=16)
    with pytest.raises(g.GothicError):
        g.Context(device=0, walk_width=8)
    ctx = g.Context(device=0, group_size=16, walk_width=16)
    with pytest.raises(g.GothicError):
        ctx.set_params(group_size=64)
    assert ctx.params["group_size"] == 16 and ctx.params["walk_width"] == 16
