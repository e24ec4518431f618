"""The boundary's failure handling on the GPU, through the C ABI: the scratch
cap and the size a refused call needed, the node count read back with the
tree, host tensors refused before any library call, and the walk's pending-
node stack (Section 2.3 keeps a walk's pending nodes in small buffers) forced
past its global part: with check = 0 the overflow shows in the sticky flags
of a later evaluation; with check = 1 the stack grows and the evaluation is
repeated, matching the oracle."""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, run_gpu, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402

FLAG_SPILL = 4


def test_scratch_cap_and_required_size():
    x = torch.from_numpy(ics.plummer(20000, seed=301)).cuda()
    say("[gpu] max_scratch_bytes = 1 MiB, n = 20000")
    ctx = g.Context(device=0, max_scratch_bytes=1 << 20)
    with pytest.raises(g.GothicError) as e:
        ctx.tree_forces(x, 1 / 64, 0.5)
    assert e.value.code == g.ENOMEM
    held, req = ctx.scratch()
    assert held == 0 and req > 1 << 20
    ctx.set_params(max_scratch_bytes=req)
    ctx.tree_forces(x, 1 / 64, 0.5)
    held2, req2 = ctx.scratch()
    assert held2 >= req - 4096 and req2 == 0
    say(f"  needed {req} bytes; holds {held2}")


def test_capture_reports_the_required_size():
    n = 12000
    x = torch.from_numpy(ics.plummer(n, seed=302)).cuda()
    out = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    ctx = g.Context(device=0, check=0)
    say("[gpu] first call inside a capture: ECAPTURE with the size")
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(g.GothicError) as e:
        with torch.cuda.graph(graph, stream=side):
            ctx.tree_forces(x, 1 / 64, 0.5, out=out)
    assert e.value.code == g.ECAPTURE
    held, req = ctx.scratch()
    assert held == 0 and req > 0
    torch.cuda.synchronize()
    ctx.tree_forces(x, 1 / 64, 0.5, out=out)  # uncaptured: sizes the scratch
    torch.cuda.synchronize()
    held2, _ = ctx.scratch()
    assert held2 >= req - 4096


def test_tree_read_back_names_its_node_count():
    ctx, _ = run_gpu(ics.nfw(5000, seed=303), 1 / 128, 0.5)
    t = ctx.tree()
    assert t["first"].size == ctx.stats()["n_nodes"] > 0
    gg = ctx.groups()
    st = ctx.stats()
    assert gg["first"].size == st["n_groups"] and gg["alist"].size == st["n_active"]


def test_host_tensors_are_refused():
    ctx = g.Context(device=0)
    x = torch.from_numpy(ics.plummer(1000, seed=304)).cuda()
    with pytest.raises(ValueError):
        ctx.tree_forces(x, 1 / 64, 0.5, out=torch.zeros((1000, 4), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.tree_forces(x, 1 / 64, 0.5, active=torch.ones(1000, dtype=torch.uint8))
    with pytest.raises(ValueError):
        ctx.tree_forces(x.cpu(), 1 / 64, 0.5)


def _spread_groups():
    """A uniform cube with 1 particle in 64 active and no r_crit split: each
    group of 64 spans the whole system, so its walk opens most of the tree
    and its pending-node stack runs deep."""
    n = 1 << 16
    rng = np.random.default_rng(305)
    x = np.empty((n, 4), np.float32)
    x[:, :3] = rng.uniform(-1, 1, (n, 3))
    x[:, 3] = 1.0 / n
    act = np.zeros(n, np.uint8)
    act[rng.choice(n, n // 64, replace=False)] = 1
    return x, act


def test_spill_overflow_is_sticky_then_grown_and_repeated():
    x, act = _spread_groups()
    n = x.shape[0]
    eps, theta = 1 / 64, 0.3
    xt = torch.from_numpy(x).cuda()
    at = torch.from_numpy(act).cuda()
    say("[gpu] spill_per_wave = 256, check = 0: the walk's stack overflows")
    ctx = g.Context(device=0, group_size=64, r_crit=0.0, spill_per_wave=256, check=0)
    out = torch.full((n, 4), float("nan"), device="cuda")
    ctx.tree_forces(xt, eps, theta, active=at, out=out)
    st = ctx._stats_raw()
    say(f"  flags {st['flags']} sticky {st['sticky_flags']}")
    assert st["flags"] & FLAG_SPILL and st["sticky_flags"] & FLAG_SPILL
    # a later evaluation that does not overflow: the flag stays sticky
    small = torch.from_numpy(ics.plummer(2000, seed=306)).cuda()
    ctx.tree_forces(small, 1 / 64, 0.5)
    st = ctx._stats_raw()
    assert st["flags"] == 0 and st["sticky_flags"] & FLAG_SPILL
    ctx.clear_flags()
    assert ctx._stats_raw()["sticky_flags"] == 0
    # check mode: the stack grows and the evaluation repeats
    ctx.set_params(check=1)
    held0, _ = ctx.scratch()
    out.fill_(float("nan"))
    ctx.tree_forces(xt, eps, theta, active=at, out=out)
    st = ctx.stats()
    held1, _ = ctx.scratch()
    say(f"  check mode: flags {st['flags']} sticky {st['sticky_flags']}, scratch {held0} -> {held1}")
    assert st["flags"] == 0 and st["sticky_flags"] == 0 and held1 > held0
    o = out.cpu().numpy()
    ref = oracle.tree_forces(x, eps, theta, active=act, group_size=64, r_crit=0.0,
                             **tie_params())
    gate_forces(ctx, ref, o, act.astype(bool), eps, theta, 1, label="grown stack: ")
