"""The scratch-free entry point (gothic_tree_forces_noalloc), through the C
ABI: two calls in a row on one context, the second on a smaller system with
an active subset, each bit-identical to gothic_tree_forces on the same input
(whose forces are held to 1e-5 against the float64 oracle on the same
interaction lists) and with keys and permutation read back from the static
array bit-exact against the oracle; the context's own scratch stays empty, and
a system too large for the array is refused before any launch."""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402

PARAMS = dict(multipole=2, group_size=32, list_depth=384, r_crit=-0.0625)


def _one(ctx_na, ctx_ref, x, eps, theta, active, label):
    n = x.shape[0]
    say(f"[gpu] {label}: n={n} eps={eps} theta={theta} "
        f"active={'all' if active is None else int(active.sum())} {PARAMS}")
    xd = torch.from_numpy(x).cuda()
    ad = None if active is None else torch.from_numpy(active).cuda()
    out_na = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    out_ref = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    ctx_na.tree_forces_noalloc(xd, eps, theta, active=ad, out=out_na)
    torch.cuda.synchronize()
    st = ctx_na.stats()
    assert st["flags"] == 0 and st["sticky_flags"] == 0, st
    ks, perm, _ = ctx_na.keys()
    ctx_ref.tree_forces(xd, eps, theta, active=ad, out=out_ref)
    torch.cuda.synchronize()
    a_na, a_ref = out_na.cpu().numpy(), out_ref.cpu().numpy()
    act = np.ones(n, bool) if active is None else active.astype(bool)
    assert np.isnan(a_na[~act]).all(), "an inactive row was written"
    assert np.array_equal(a_na[act], a_ref[act]), "scratch-free result differs"
    ref = oracle.tree_forces(x, eps, theta, active=active, multipole=PARAMS["multipole"],
                             group_size=PARAMS["group_size"], r_crit=PARAMS["r_crit"],
                             **tie_params())
    assert np.array_equal(ks, ref["keys_sorted"]) and np.array_equal(perm, ref["perm"])
    errs = gate_forces(ctx_ref, ref, a_ref, act, eps, theta, multipole=PARAMS["multipole"],
                       label=label)
    say(f"  {label}: bit-identical to gothic_tree_forces; against the oracle {errs}")


def test_noalloc_two_calls_match_the_allocating_entry_point():
    ctx_na = g.Context(device=0, **PARAMS)
    ctx_ref = g.Context(device=0, **PARAMS)
    x1 = ics.nfw(60000, seed=611)
    _one(ctx_na, ctx_ref, x1, 1 / 128, 0.5, None, "first call, NFW 60000")
    x2 = ics.plummer(9000, seed=612)
    act = (np.random.default_rng(613).random(9000) < 0.3).astype(np.uint8)
    _one(ctx_na, ctx_ref, x2, 1 / 64, 0.5, act, "second call, Plummer 9000, 30% active")
    held, req = ctx_na.scratch()
    assert held == 0 and req == 0, (held, req)


def test_noalloc_refuses_a_system_beyond_the_array():
    n = 1 << 21
    ctx = g.Context(device=0, **PARAMS)
    xd = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    out = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    say(f"[gpu] scratch-free call with n={n}: refused on the host")
    with pytest.raises(g.GothicError) as e:
        ctx.tree_forces_noalloc(xd, 1 / 64, 0.5, out=out)
    assert e.value.code == g.ENOMEM
    held, req = ctx.scratch()
    assert held == 0 and req > 256 << 20, (held, req)
