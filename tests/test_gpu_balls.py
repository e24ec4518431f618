"""Enclosing balls of the pseudo i-particles (Appendix B: GEO, SEB, EBS,
COM, CMP) against the float64 oracle, through the C ABI.

The library computes the SEB / EBS / COM centres in float64 and the radius
(largest member distance) in float32 widened by 4 ulp; so centres agree to
single-precision rounding and radii to a few ulp, and forces at the usual
1e-5 for every active particle (gpu_util.gate_forces).  Masses are unequal, so
the COM and CMP centres depend on the mass weighting.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import gate_forces, rel_rms, run_gpu, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

KINDS = {"GEO": 0, "SEB": 1, "EBS": 2, "COM": 3, "CMP": 4}


def _unequal(x, seed):
    """Masses spread over a factor 16, so the COM and CMP centres depend on the
    mass weighting (Appendix B)."""
    x = x.copy()
    x[:, 3] *= np.random.default_rng(seed).uniform(0.25, 4.0, x.shape[0]).astype(np.float32)
    return x


@pytest.mark.parametrize("name", list(KINDS))
@pytest.mark.parametrize("G", [64, 32, 8])
def test_balls_match(name, G):
    kind = KINDS[name]
    x = _unequal(ics.nfw(12000, seed=121), 131)
    act = ics.random_active(12000, 0.5, seed=122)
    ctx, _ = run_gpu(x, 1 / 128, 0.5, active=act, group_size=G, ball=kind, r_crit=0.0)
    gg = ctx.groups()
    ks, perm, cube = ctx.keys()
    ps = x[perm].astype(np.float64)
    go = oracle.groups(act[perm], ps, G, 0.0, kind)
    assert np.array_equal(gg["first"], go["first"]) and np.array_equal(gg["count"], go["count"])
    scale = np.abs(go["ball"][:, :3]).max(1) + go["ball"][:, 3]
    dc = np.abs(gg["ball"][:, :3] - go["ball"][:, :3]).max(1)
    close = dc <= 1e-6 * scale
    rg, ro = gg["ball"][:, 3].astype(np.float64), go["ball"][:, 3]
    say(f"  {name} G={G}: centres close {close.mean():.5f}, radius ratio "
        f"{np.median(rg / np.maximum(ro, 1e-300)):.7f}")
    assert close.mean() >= 0.999
    # the library's radius holds every member (widened), and is tight
    assert np.all(rg[close] >= ro[close] * (1 - 1e-6) - 1e-7 * scale[close])
    assert np.all(rg[close] <= ro[close] * (1 + 2e-6) + 1e-6 * scale[close])


@pytest.mark.parametrize("name", ["SEB", "EBS", "COM", "CMP"])
def test_forces_with_each_ball(name):
    kind = KINDS[name]
    x = _unequal(ics.nfw(20000, seed=123), 133)
    act = ics.random_active(20000, 0.3, seed=124)
    ctx, out = run_gpu(x, 1 / 128, 0.5, active=act, ball=kind, multipole=2)
    ref = oracle.tree_forces(x, 1 / 128, 0.5, active=act, multipole=2, ball=kind, **tie_params())
    gate_forces(ctx, ref, out, act.astype(bool), 1 / 128, 0.5, 2, label=f"{name}: ")


def test_smaller_balls_mean_fewer_interactions():
    # Appendix B: a tighter ball cuts the interactions (SEB <= EBS, GEO <= COM)
    x = ics.nfw(30000, seed=125)
    counts = {}
    for name, kind in KINDS.items():
        ctx, _ = run_gpu(x, 1 / 128, 0.5, ball=kind, r_crit=0.0)
        counts[name] = ctx.stats()["interactions"]
    say(f"  interactions by ball: {counts}")
    assert counts["SEB"] <= counts["EBS"] and counts["SEB"] <= counts["GEO"]
    assert counts["GEO"] <= counts["COM"] and counts["CMP"] <= counts["COM"]
