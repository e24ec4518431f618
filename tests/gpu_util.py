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
