"""The float64 direct summation (the accuracy reference of Section 3.2, Fig. 3)
through the C ABI, against the oracle's direct sum on the same particles.

Both sides sum every pair j != i of the Plummer-softened force in float64, in
different orders (the library in 256-particle tiles and chunks, the oracle
j = 0 .. n-1), so they agree to rounding: 1e-12 relative to the size of the
row's acceleration (and of phi).
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1610_07279_amd as g  # noqa: E402

TOL = 1e-12


def _close(got, ref):
    a_err = np.linalg.norm(got[:, :3] - ref[:, :3], axis=1) / np.linalg.norm(ref[:, :3], axis=1)
    p_err = np.abs(got[:, 3] - ref[:, 3]) / np.abs(ref[:, 3])
    return float(a_err.max()), float(p_err.max())


@pytest.mark.parametrize("n", [1, 2, 255, 3001])
def test_direct_all_targets(n):
    x = ics.plummer(n, seed=91 + n)
    say(f"[gpu] direct sum, all {n} targets")
    ctx = g.Context(device=0)
    got = ctx.direct_forces(torch.from_numpy(x).cuda(), 1 / 64).cpu().numpy()
    ref = oracle.direct(x, 1 / 64)
    if n == 1:
        assert np.array_equal(got, np.zeros((1, 4)))  # nothing to sum
        return
    ea, ep = _close(got, ref)
    say(f"  max relative difference: acc {ea:.2e}, phi {ep:.2e}")
    assert ea <= TOL and ep <= TOL


def test_direct_sampled_targets_ragged_chunks():
    # few targets: the j-particles split into many chunks, the last one ragged
    n = 70001
    x = ics.nfw(n, seed=93)
    rng = np.random.default_rng(94)
    idx = np.concatenate([[0, n - 1, 5, 5], rng.integers(0, n, 296)]).astype(np.int64)
    say(f"[gpu] direct sum, {idx.size} sampled targets of {n}")
    ctx = g.Context(device=0)
    xt = torch.from_numpy(x).cuda()
    it = torch.from_numpy(idx).cuda()
    got = ctx.direct_forces(xt, 1 / 128, idx=it).cpu().numpy()
    ref = oracle.direct(x, 1 / 128, idx)
    ea, ep = _close(got, ref)
    say(f"  max relative difference: acc {ea:.2e}, phi {ep:.2e}")
    assert ea <= TOL and ep <= TOL
    # the partials are added in a fixed order: identical on every call
    again = ctx.direct_forces(xt, 1 / 128, idx=it).cpu().numpy()
    assert np.array_equal(got, again)
    # many targets, one chunk: the same rows again
    every = ctx.direct_forces(xt, 1 / 128).cpu().numpy()
    ea2, ep2 = _close(every[idx], ref)
    assert ea2 <= TOL and ep2 <= TOL


def test_direct_coincident_particles_and_bad_indices():
    # two particles at one position: each sees the other's -m/eps and no force
    x = ics.plummer(600, seed=95)
    x[7, :3] = x[8, :3]
    idx = np.array([7, 8, -1, 600, 3], np.int64)
    ctx = g.Context(device=0)
    got = ctx.direct_forces(torch.from_numpy(x).cuda(), 1 / 32,
                            idx=torch.from_numpy(idx).cuda()).cpu().numpy()
    ref = oracle.direct(x, 1 / 32, idx[[0, 1, 4]])
    ea, ep = _close(got[[0, 1, 4]], ref)
    assert ea <= TOL and ep <= TOL
    # indices outside [0, n) give NaN rows, the others are unaffected
    assert np.all(np.isnan(got[2:4]))
    # no targets: nothing to do; targets among no particles: an argument error
    empty = torch.zeros((0,), dtype=torch.int64, device="cuda")
    assert ctx.direct_forces(torch.from_numpy(x).cuda(), 1 / 32, idx=empty).shape == (0, 4)
    with pytest.raises(g.GothicError):
        ctx.direct_forces(torch.zeros((0, 4), device="cuda"), 1 / 32,
                          idx=torch.zeros((3,), dtype=torch.int64, device="cuda"))
