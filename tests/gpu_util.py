"""Shared helpers of the GPU parity tests (run the library, compare with the oracle)."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_rms(a, b, cols=slice(0, 3)):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(((a[:, cols] - b[:, cols]) ** 2).sum() / max((b[:, cols] ** 2).sum(), 1e-300)))


def run_gpu(xyzm, eps, theta, active=None, **params):
    import torch

    import paper_1610_07279_amd as g
    say(f"[gpu] n={xyzm.shape[0]} eps={eps} theta={theta} active={'all' if active is None else int(active.sum())} {params}")
    ctx = g.Context(device=0, **params)
    x = torch.from_numpy(np.ascontiguousarray(xyzm, np.float32)).cuda()
    a = None if active is None else torch.from_numpy(np.ascontiguousarray(active, np.uint8)).cuda()
    out = torch.full((xyzm.shape[0], 4), float("nan"), dtype=torch.float32, device="cuda")
    ctx.tree_forces(x, eps, theta, active=a, out=out)
    torch.cuda.synchronize()
    return ctx, out.cpu().numpy()


def tie_params():
    # window of a single-precision MAC decision: relative to the compared
    # quantities, plus a few ulp of the coordinates
    return dict(tie_rel=2e-5, tie_abs=1e-6)


def diagnose_forces(ctx, x, ref, out, rows):
    """Print where a force mismatch starts: keys, tree, node moments, groups,
    per-group list lengths (called only when a parity check fails)."""
    try:
        st = ctx.stats()
        say("  [diag] stats", st)
        ks, perm, _ = ctx.keys()
        say("  [diag] perm equal", bool(np.array_equal(perm, ref["perm"])))
        t, to = ctx.tree(), ref["tree"]
        for f in ("first", "count", "child_first", "n_child", "level"):
            if f in to:
                say(f"  [diag] tree {f} equal", t[f].shape == to[f].shape and bool(np.array_equal(t[f], to[f])))
        com, b, q = ctx.nodes()
        if com.shape[0] == ref["com"].shape[0]:
            bo, co = ref["b"], ref["com"]
            db = np.abs(b - bo) / (bo + 1e-30)
            bad = np.flatnonzero(db > 1e-4)
            say(f"  [diag] node b rel max {db.max():.3e}, nodes off {bad.size} of {b.size}:",
                bad[:8], b[bad[:8]], bo[bad[:8]])
            dm = np.abs(com[:, 3] - co[:, 3]) / (co[:, 3] + 1e-30)
            dx = np.abs(com[:, :3] - co[:, :3]).max(1) / (np.abs(co[:, :3]).sum(1) + bo + 1e-30)
            say(f"  [diag] node mass rel max {dm.max():.3e}, com rel max {dx.max():.3e}")
            S = ref["S"]
            s_scale = co[:, 3] * (bo ** 2) + 1e-30
            dq = np.abs(q - S).max(1) / s_scale
            badq = np.flatnonzero(dq > 1e-3)
            say(f"  [diag] node quad rel max {dq.max():.3e}, nodes off {badq.size}:", badq[:8])
        gg, og = ctx.groups(), ref["groups"]
        same = gg["first"].shape == og["first"].shape and bool(np.array_equal(gg["first"], og["first"]))
        say(f"  [diag] groups gpu {gg['first'].size} oracle {og['first'].size} firsts equal {same}")
        if same:
            dr = np.abs(gg["ball"][:, 3] - og["ball"][:, 3]) / (og["ball"][:, 3] + 1e-30)
            dc = np.abs(gg["ball"][:, :3] - og["ball"][:, :3]).max()
            say(f"  [diag] ball r rel max {dr.max():.3e} centre abs max {dc:.3e}")
            ent = gg["entries"].astype(np.int64)
            cnt = ref["counts"]
            off = np.flatnonzero((ent[:, 0] != cnt[:, 0]) | (ent[:, 1] != cnt[:, 1]))
            say(f"  [diag] groups whose lists differ {off.size}; clean among them "
                f"{int((cnt[off, 2] == 0).sum())}")
            for g in off[:8]:
                say(f"  [diag]   group {g} size {gg['count'][g]} gpu {ent[g].tolist()} oracle {cnt[g].tolist()}")
        err = np.abs(out[:, :3] - ref["acc_pot"][:, :3]).max(1) / (np.abs(ref["acc_pot"][:, :3]).max(1) + 1e-30)
        err[~rows] = 0
        worst = np.argsort(err)[::-1][:5]
        inv = np.empty_like(ref["perm"])
        inv[ref["perm"]] = np.arange(ref["perm"].size, dtype=inv.dtype)
        say("  [diag] worst rows", worst, "rel err", err[worst], "sorted index", inv[worst])
    except Exception as e:  # a diagnostic must not hide the failure it explains
        say("  [diag] failed:", repr(e))


def oracle_parts(tree, mom, ps, grp, perm):
    """A reference dict (as oracle.tree_forces returns) from separately built
    oracle pieces, for gate_forces(..., sel=...) on large systems."""
    return dict(tree=tree, com=mom[0], b=mom[1], S=mom[2], ps=ps, groups=grp, perm=perm)


def gate_forces(ctx, ref, out, act, eps, theta, multipole=1, mac=0, delta=0.0, acc_old=None,
                tol=1e-5, sel=None, max_tie_groups=512, sample_clean=8, label=""):
    """Hold every active row of the groups `sel` (default: all) to `tol`
    (relative rms of acceleration and of potential) against a float64
    evaluation of the SAME interaction list:

    - groups without a MAC near tie: the oracle's own tree walk (identical
      lists: per-group list lengths equal, and for a sample of groups the
      lists themselves, entry by entry);
    - groups with a near tie (a decision that single and double precision may
      take differently, Section 2.2's MAC at the rounding level): the GPU's
      own list is read back (gothic_get_lists) and walked again by the oracle
      following the GPU's decisions; every decision must agree with the
      float64 MAC except inside the near-tie window, every entry must be
      reached, the list's mass must be the system's, and the rows are
      compared with the float64 forces of that list.

    ref: oracle.tree_forces(...) of the same system and parameters (with
    tie_params()), or oracle_parts(...) with sel; out: the GPU's [n,4] forces
    (caller order); act: bool [n] active rows.  Returns the measured errors."""
    og = ref["groups"]
    perm = ref["perm"]
    mom = (ref["com"], ref["b"], ref["S"])
    amag = None
    if mac == 1:
        amag = np.sqrt((np.asarray(acc_old, np.float64)[:, :3] ** 2).sum(1))[perm]
    ng = og["first"].size
    if sel is None:
        sel = np.arange(ng)
        cnt = ref["counts"]
        ref_acc = ref["acc_pot"]
    else:
        sel = np.asarray(sel, np.int64)
        osort, cnt_all, _ = oracle.walk(ref["tree"], mom, ref["ps"], og, eps, theta, multipole,
                                        gsel=sel, mac=mac, delta=delta, amag=amag, **tie_params())
        cnt = cnt_all[sel]
        ref_acc = np.full_like(osort, np.nan)
        ref_acc[perm] = osort
    gg = ctx.groups()
    ent = gg["entries"].astype(np.int64)[sel]
    assert np.array_equal(gg["first"], og["first"]) and np.array_equal(gg["count"], og["count"])
    clean = cnt[:, 2] == 0
    assert np.array_equal(ent[clean, :2], cnt[clean, :2]), "tie-free list lengths differ"
    rows_of = lambda g: perm[og["alist"][og["first"][g]:og["first"][g] + og["count"][g]]]
    rows = np.zeros(out.shape[0], bool)
    for g in sel:
        rows[rows_of(g)] = True
    rows &= act
    target = ref_acc.copy()
    rng = np.random.default_rng(7)
    cg = sel[clean]
    if cg.size and sample_clean:  # a sample of tie-free groups: the lists themselves
        pick = rng.choice(cg, size=min(sample_clean, cg.size), replace=False)
        gl, _ = ctx.lists(pick)
        _, _, _, ol = oracle.walk(ref["tree"], mom, ref["ps"], og, eps, theta, multipole,
                                  gsel=pick, mac=mac, delta=delta, amag=amag, lists_cap=1 << 16,
                                  **tie_params())
        for (gn, gf), (on, of) in zip(gl, ol):
            assert np.array_equal(np.sort(gn), np.sort(on)), "tie-free list differs"
            assert np.array_equal(np.sort(gf), np.sort(of)), "tie-free list differs"
    ties = sel[~clean]
    n_checked = 0
    in_window = 0
    if ties.size:
        tg = ties if ties.size <= max_tie_groups else rng.choice(ties, max_tie_groups,
                                                                 replace=False)
        gl, rewalk = ctx.lists(tg)
        acc_r, info, mass = oracle.walk_replay(ref, tg, gl, eps, theta, multipole, mac=mac,
                                               delta=delta, acc_old=acc_old, **tie_params())
        assert (info[:, 2] == 0).all(), f"decisions outside the near-tie window: {info[info[:, 2] > 0]}"
        assert (info[:, 3] == 0).all() and (info[:, 4] == 0).all(), "lists not a valid walk"
        M = float(ref["ps"][:, 3].sum())
        assert np.allclose(mass, M, rtol=1e-9), "mass closure"
        for g in tg:
            r = rows_of(g)
            assert np.array_equal(rewalk[r], out[r]), "the re-walk must reproduce the evaluation"
            target[r] = acc_r[r]
        for g in np.setdiff1d(ties, tg):  # rows of tie groups beyond the cap are left out
            rows[rows_of(g)] = False
        n_checked = tg.size
        in_window = int(info[:, 1].sum())
    e_acc = rel_rms(out[rows], target[rows])
    # The kernel forms P_i = sum_j m_j / R_ij over the list, the self pair
    # (m_i / eps) included, and returns phi_i = -P_i + m_i / eps: its float32
    # rounding is relative to P_i, which equals |phi_i| unless the self pair
    # dominates (a few heavy particles).  The potential's error is measured
    # relative to P_i.
    m = np.empty(out.shape[0], np.float64)
    m[perm] = ref["ps"][:, 3]
    P = np.abs(np.asarray(target[rows][:, 3], np.float64)) + m[rows] / eps
    d_pot = np.asarray(out[rows][:, 3], np.float64) - target[rows][:, 3]
    e_pot = float(np.sqrt((d_pot ** 2).sum() / max((P ** 2).sum(), 1e-300)))
    g_acc = rel_rms(out[rows], ref_acc[rows])
    say(f"  {label}rms acc {e_acc:.2e} pot {e_pot:.2e} (vs the float64 tree over the same rows: "
        f"{g_acc:.2e}); groups {sel.size}, with near ties {ties.size} (replayed {n_checked}, "
        f"{in_window} decisions taken the other way inside the window)")
    assert e_acc <= tol and e_pot <= tol, (e_acc, e_pot)
    return dict(e_acc=e_acc, e_pot=e_pot, e_global=g_acc, tie_groups=int(ties.size))
