"""GPU parity of the HIP library against the float64 oracle (through the C ABI).

Integer results (keys, permutation, tree arrays, groups, per-group lists away
from MAC near-ties) must be bit-exact.  Floating results: node moments to
single-precision round-off; forces of every active particle within 1e-5
relative rms of a float64 evaluation of the same list: the oracle's own tree
for groups without a near tie, and for groups with one the GPU's read-back
list, whose every decision the oracle checks (gpu_util.gate_forces).
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_util import diagnose_forces, gate_forces, rel_rms, run_gpu, say, tie_params

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def _coincident(n=300, seed=3):
    x = ics.plummer(n, seed=seed)
    x[10:60, :3] = x[9, :3]       # 51 identical positions -> level-21 leaf
    x[100:103, :3] = x[99, :3]
    return x


def _cluster(n=3000, m=130, seed=4):
    """A Plummer sphere with m particles jittered by ~1e-7 about one point:
    they share a level-21 cell, so a leaf holds more than 64 members."""
    x = ics.plummer(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    x[:m, :3] = x[0, :3] + rng.uniform(-1e-7, 1e-7, (m, 3)).astype(np.float32)
    return x


def _uniform(n, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((n, 4), np.float32)
    x[:, :3] = rng.uniform(-1, 1, (n, 3))
    x[:, 3] = rng.uniform(0.5, 1.5, n) / n
    return x


SYSTEMS = {
    # systems of at most 8192 particles take the one-workgroup octree build,
    # larger ones the level-by-level launches: both are held to the oracle
    "nfw20k": lambda: ics.nfw(20000, seed=8),
    "plummer8k": lambda: ics.plummer(8192, seed=101),
    "nfw4097": lambda: ics.nfw(4097, seed=7),
    "uniform777": lambda: _uniform(777, 5),
    "coincident": lambda: _coincident(),
    "cluster130": lambda: _cluster(),
    "one": lambda: ics.plummer(1, seed=1),
    "two": lambda: ics.plummer(2, seed=2),
    "allsame": lambda: np.tile(np.array([[0.25, -0.5, 1.0, 0.01]], np.float32), (70, 1)),
}


# ------------------------------------------------------------------ keys, tree
@pytest.mark.parametrize("key_kind", [0, 1])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_keys_sort_tree_bitexact(name, key_kind):
    x = SYSTEMS[name]()
    for n_leaf in (16, 1):
        ctx, _ = run_gpu(x, 1 / 64, 0.5, key_kind=key_kind, n_leaf=n_leaf)
        ks, perm, cube = ctx.keys()
        k_o, cube_o = oracle.keys(x, key_kind)
        ks_o, perm_o = oracle.sort(k_o)
        assert np.array_equal(cube, cube_o)
        assert np.array_equal(ks, ks_o)
        assert np.array_equal(perm, perm_o)
        # the key-order gather: positions and masses exactly the caller's
        assert np.array_equal(ctx.positions(), x[perm_o])
        t = ctx.tree()
        t_o = oracle.build(ks_o, n_leaf)
        for f in ("first", "count", "child_first", "n_child", "level"):
            assert np.array_equal(t[f], t_o[f]), f


@pytest.mark.parametrize("name", ["plummer8k", "nfw4097", "coincident", "cluster130"])
@pytest.mark.parametrize("multipole", [1, 2])
def test_moments_match(name, multipole):
    x = SYSTEMS[name]()
    ctx, _ = run_gpu(x, 1 / 64, 0.5, multipole=multipole)
    com, b, q = ctx.nodes()
    ks, perm, _ = ctx.keys()
    t = oracle.build(ks, 16)
    if name == "cluster130":  # the case it is built for: a leaf past 64 members
        assert (t["count"][t["n_child"] == 0]).max() > 64
    ps = x[perm].astype(np.float64)
    com_o, b_o, S_o = oracle.moments(t, ps)
    scale = np.abs(com_o[:, :3]).sum(1) + b_o
    assert np.all(np.abs(com[:, 3] - com_o[:, 3]) <= 2e-6 * com_o[:, 3] + 1e-30)
    assert np.all(np.abs(com[:, :3] - com_o[:, :3]).max(1) <= 2e-6 * scale + 1e-30)
    assert np.all(np.abs(b - b_o) <= 1e-5 * b_o + 2e-6 * scale)
    one = t["count"] == 1
    assert np.all(b[one] == 0) and np.all(com[one, :3] == ps[t["first"][one], :3])
    if multipole == 2:
        s_scale = com_o[:, 3] * (b_o ** 2 + (2e-6 * scale) ** 2)
        assert np.all(np.abs(q - S_o).max(1) <= 1e-4 * s_scale + 1e-30)
    else:
        assert np.all(q == 0)


@pytest.mark.parametrize("r_crit", [0.0, -0.0625, 0.05])
@pytest.mark.parametrize("G", [64, 32, 16, 1])
def test_groups_match(G, r_crit):
    x = ics.nfw(5000, seed=9)
    act = ics.random_active(5000, 0.3, seed=10)
    ctx, _ = run_gpu(x, 1 / 128, 0.5, active=act, group_size=G, r_crit=r_crit)
    gg = ctx.groups()
    ks, perm, cube = ctx.keys()
    ps = x[perm].astype(np.float64)
    rc = float(np.float32(r_crit))
    go = oracle.groups(act[perm], ps, G, -rc * cube[3] if rc < 0 else rc)
    assert np.array_equal(gg["alist"], go["alist"])
    assert np.array_equal(gg["first"], go["first"])
    assert np.array_equal(gg["count"], go["count"])
    assert np.allclose(gg["ball"][:, :3], go["ball"][:, :3], rtol=0, atol=1e-6)
    assert np.all(gg["ball"][:, 3] >= go["ball"][:, 3] * (1 - 1e-6))
    assert np.all(gg["ball"][:, 3] <= go["ball"][:, 3] * (1 + 1e-5) + 1e-6)


# ------------------------------------------------------------------ forces
def _check_forces(x, eps, theta, active=None, tol=1e-5, **params):
    ctx, out = run_gpu(x, eps, theta, active=active, **params)
    st = ctx.stats()
    multipole = params.get("multipole", 1)
    ref = oracle.tree_forces(x, eps, theta, active=active, n_leaf=params.get("n_leaf", 16),
                             group_size=params.get("group_size", 32), multipole=multipole,
                             key_kind=params.get("key_kind", 0),
                             r_crit=params.get("r_crit", -0.0625), **tie_params())
    act = np.ones(x.shape[0], bool) if active is None else active.astype(bool)
    assert np.all(np.isnan(out[~act])), "inactive rows must stay untouched"
    assert np.all(np.isfinite(out[act]))
    try:
        gate_forces(ctx, ref, out, act, eps, theta, multipole, tol=tol)
    except AssertionError:
        diagnose_forces(ctx, x, ref, out, act)
        raise
    cnt = ref["counts"]
    if (cnt[:, 2] == 0).all():
        gg = ctx.groups()
        assert st["interactions"] == int(((cnt[:, 0] + cnt[:, 1]) * gg["count"]).sum())
    assert st["sticky_flags"] == 0
    return ctx, out, ref


def test_plummer8k_config():
    _check_forces(ics.plummer(8192, seed=101), 1 / 64, 0.5)


@pytest.mark.parametrize("r_crit", [0.0, 0.3, -0.03125])
def test_critical_separation(r_crit):
    _check_forces(ics.nfw(20000, seed=23), 1 / 128, 0.5, multipole=2, r_crit=r_crit)


@pytest.mark.parametrize("G,multipole", [(64, 1), (32, 2), (8, 2)])
def test_groups_of_every_size_take_their_lane_shape(G, multipole):
    """Groups shorter than G (split by r_crit in a sparse active set) are laid
    out on the fewest power-of-two slots that hold them, with more lanes per
    i-particle: the kernel's own shape, half of it and the run-time shapes below
    must all appear and match the float64 evaluation of the same lists."""
    x = ics.nfw(30000, seed=25)
    act = ics.random_active(30000, 0.5, seed=26)
    ctx, _, _ = _check_forces(x, 1 / 128, 0.5, active=act, group_size=G, r_crit=0.4,
                              multipole=multipole)
    cnt = ctx.groups()["count"]
    slots = 2 ** np.ceil(np.log2(np.maximum(cnt, 1))).astype(int)
    say(f"  G={G}: groups {cnt.size}, by slots {dict(zip(*np.unique(slots, return_counts=True)))}")
    assert (slots == G).any() and (slots == G // 2).any() and (slots < G // 2).any()


@pytest.mark.parametrize("G", [64, 16, 8, 1])
def test_group_sizes_and_ij_parallel(G):
    _check_forces(ics.plummer(6000, seed=11), 1 / 64, 0.5, group_size=G)


@pytest.mark.parametrize("D", [64, 1024])
@pytest.mark.parametrize("comp", [0, 1])
def test_list_depth_and_compensation(D, comp):
    _check_forces(ics.nfw(7000, seed=12), 1 / 128, 0.5, list_depth=D, compensated=comp)


@pytest.mark.parametrize("G", [32, 8, 1])
def test_quadrupole(G):
    _check_forces(ics.nfw(20000, seed=13), 1 / 128, 0.5, multipole=2, group_size=G)


def test_peano_hilbert_keys():
    _check_forces(ics.plummer(5000, seed=14), 1 / 64, 0.6, key_kind=1)


@pytest.mark.parametrize("n_leaf", [1, 4, 64])
def test_leaf_sizes(n_leaf):
    _check_forces(ics.nfw(3000, seed=15), 1 / 128, 0.5, n_leaf=n_leaf)


@pytest.mark.parametrize("frac", [0.01, 0.2])
def test_active_subsets(frac):
    x = ics.nfw(30000, seed=16)
    _check_forces(x, 1 / 128, 0.5, active=ics.random_active(30000, frac, seed=17))


def test_node_capacity_overflow_grows_and_repeats():
    # a deliberately tiny node array: the first tree is abandoned on the
    # device (no kernel touches the partial tree), the host grows the arrays
    # and repeats until the tree fits
    x = ics.nfw(3000, seed=22)
    ctx, out = run_gpu(x, 1 / 128, 0.5, n_leaf=4, node_capacity=256)
    ref = oracle.tree_forces(x, 1 / 128, 0.5, n_leaf=4)  # same default r_crit (L/16)
    assert rel_rms(out, ref["acc_pot"]) <= 1e-5
    assert ctx.stats()["n_nodes"] == ref["tree"]["first"].size


def test_no_active_particles():
    x = ics.plummer(1000, seed=18)
    ctx, out = run_gpu(x, 1 / 64, 0.5, active=np.zeros(1000, np.uint8))
    assert np.all(np.isnan(out))
    assert ctx.stats()["n_groups"] == 0


@pytest.mark.parametrize("name", ["coincident", "one", "two", "allsame", "uniform777"])
def test_edge_systems(name):
    _check_forces(SYSTEMS[name](), 1 / 64, 0.5)


def test_theta_zero_is_direct_sum():
    x = ics.plummer(4096, seed=19)
    ctx, out = run_gpu(x, 1 / 64, 0.0)
    d = oracle.direct(x, 1 / 64)
    assert rel_rms(out, d) <= 1e-5
    assert rel_rms(out, d, cols=slice(3, 4)) <= 1e-5


def test_deterministic_and_reusable_context():
    import paper_1610_07279_amd as g
    ctx = g.Context(device=0)
    outs = []
    for n in (3000, 50000, 3000):
        x = torch.from_numpy(ics.nfw(n, seed=20)).cuda()
        outs.append(ctx.tree_forces(x, 1 / 128, 0.5).cpu().numpy())
    assert np.array_equal(outs[0], outs[2])


def test_argument_errors():
    import paper_1610_07279_amd as g
    ctx = g.Context(device=0)
    x = torch.from_numpy(ics.plummer(100, seed=21)).cuda()
    for eps, th in ((0.0, 0.5), (-1.0, 0.5), (0.01, 1.0), (0.01, -0.1), (float("nan"), 0.5)):
        with pytest.raises(g.GothicError) as e:
            ctx.tree_forces(x, eps, th)
        assert e.value.code == g.EINVAL
    for bad in (dict(group_size=3), dict(list_depth=100), dict(n_leaf=0), dict(multipole=3),
                dict(key_kind=2)):
        with pytest.raises(g.GothicError) as e:
            g.Context(device=0, **bad)
        assert e.value.code == g.EINVAL
    xn = ics.plummer(100, seed=21)
    xn[5, 1] = np.nan
    with pytest.raises(g.GothicError) as e:
        ctx.tree_forces(torch.from_numpy(xn).cuda(), 0.01, 0.5)
    assert e.value.code == g.ENONFINITE
    empty = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    assert ctx.tree_forces(empty, 0.01, 0.5).shape == (0, 4)
