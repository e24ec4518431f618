#!/usr/bin/env python3
"""Benchmark of the block-step tree gravity on one MI355X.

Workload (the headline configuration): NFW sphere, N = 2^24 equal-mass
particles (r_s = 1, c = 10, truncated at 10 r_s, mass 1, seed 501), eps =
1/512, opening angle 0.5 with quadrupole pseudo j-particles, float32 forces and
float64 integration, time steps 0.1 sqrt(eps/|a|) on 8 levels below the
finest.  Inputs are synthetic (seeded generator), resident on the GPU before
timing.

One "step" is one finest sub-step of the block scheme: predict every
particle, build keys / sort / octree when the tree is rebuilt (by default
when the growth models of Section 2.6 say so, otherwise the last tree is
walked with the current positions), moments, groups, walk the groups of the
particles due at that time, correct them and assign new levels.  The same
number of shared steps (every particle at the finest step, leap-frog) is timed
for the block-versus-shared comparison.

Printed JSON line: value = interactions per second over the timed block steps
(interactions = list entries x i-particles), ms_per_step = block seconds per
sub-step; plus the shared-step figures, the walk-kernel roofline (FP32 VALU,
HIP events around every walk launch) and the float64 CPU oracle's rate on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3          # MI355X vector FP32, 256 CU x 2.4 GHz x 256 flop/clk
                                  # (packed FP32; one non-packed FMA per lane-slot is half)
FLOP_MONO = 24                    # per monopole interaction (20 + rsqrt weighted 4)
FLOP_QUAD = 60                    # per quadrupole node interaction (operations of the factored
                                  # quadrupole term, rsq weighted 4)
METRIC = "s/step + interactions/s, NFW 2^24 block vs shared step; % FP32 VALU peak"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_traffic():
    """HBM bytes per timed walk launch from the committed counter summary, while
    the walk source is the one the counters were taken on (else None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "walk_nfw16m_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1610_07279_amd", "csrc", "walk.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch: ", "walk_source_sha256: ")))
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields["walk_source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, shared, steps, warmup):
    import torch
    pos = pos0.clone()
    vel = vel0.clone()
    ctx.set_params(check=1)
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=eta, kmax=kmax, shared=shared)
    # warm-up: checked steps (they grow any scratch), the last one unchecked
    # (with params.graph it is the capture)
    for i in range(warmup):
        if i == warmup - 1:
            ctx.set_params(check=0)
        ctx.sim_step()
    ctx.set_params(check=0)
    torch.cuda.synchronize()
    ctx.sim_reset_counters()
    ctx.walk_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sim_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = ctx.sim_info()
    walk_ms, launches = ctx.walk_time()
    st = ctx.stats()
    if st["flags"]:
        raise RuntimeError(f"device flags {st['flags']} set during the timed steps")
    return dict(seconds=t1 - t0, info=info, walk_ms=walk_ms, walk_launches=launches)


def batched_bench(cycles=1, kmax=6):
    """64 independent systems (N_s log-uniform in [2^12, 2^18], Plummer / NFW,
    seed 401), monopole, theta 0.5, block steps on 6 levels below the finest:
    one full cycle of 2^kmax sub-steps with every system advanced by ONE
    captured batched sub-step (graph), against the same systems advanced by 64
    separate contexts, one sub-step each, launched in turn on the same stream.
    Also one all-active force evaluation: batched vs 64 serial calls."""
    import torch

    import ics
    import paper_1610_07279_amd as g
    x, offs, eps, v = ics.batched_systems(64, seed=401, with_vel=True)
    nsys, n = 64, x.shape[0]
    dev = torch.device("cuda", 0)
    pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
    vel0 = torch.from_numpy(v).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
    xt = torch.from_numpy(x).to(dev)
    steps = cycles << kmax

    # both sides take one untimed sub-step (the capture, the first launches),
    # then a full cycle of 2^kmax sub-steps is timed
    ctx = g.Context(device=0, graph=1)
    pos, vel = pos0.clone(), vel0.clone()
    ctx.sim_bind_batched(pos, vel, mass, offs, eps, 0.5, eta=0.1, kmax=kmax)
    ctx.set_params(check=0)
    ctx.sim_step(1)
    ctx.sim_reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sim_step(steps)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    info = ctx.sim_info()
    if ctx.stats()["flags"]:
        raise RuntimeError("device flags set in the batched steps")

    ctxs, keep = [], []
    for s in range(nsys):
        lo, hi = int(offs[s]), int(offs[s + 1])
        c = g.Context(device=0)
        p, q = pos0[lo:hi].clone(), vel0[lo:hi].clone()
        m = mass[lo:hi].contiguous()
        c.sim_bind(p, q, m, float(eps[s]), 0.5, eta=0.1, kmax=kmax)
        c.set_params(check=0)
        ctxs.append(c)
        keep.append((p, q, m))
    for c in ctxs:
        c.sim_step(1)
        c.sim_reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for c in ctxs:
            c.sim_step(1)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    active_serial = sum(c.sim_info()["active_total"] for c in ctxs)

    # one all-active evaluation
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    fctx = g.Context(device=0, check=0)
    fctx.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        fctx.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    f_b = (time.perf_counter() - t0) / reps
    sctx = g.Context(device=0, check=0)
    views = [(xt[int(offs[s]):int(offs[s + 1])], out[int(offs[s]):int(offs[s + 1])])
             for s in range(nsys)]
    for s, (xs, os_) in enumerate(views):
        sctx.tree_forces(xs, float(eps[s]), 0.5, out=os_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for s, (xs, os_) in enumerate(views):
            sctx.tree_forces(xs, float(eps[s]), 0.5, out=os_)
    torch.cuda.synchronize()
    f_s = (time.perf_counter() - t0) / reps
    return {"workload": f"64 systems, N={n} in all (N_s log-uniform in [2^12, 2^18], Plummer "
                        f"eps 1/64 / NFW eps 1/128), monopole, theta 0.5, kmax {kmax}",
            "substeps": steps,
            "batched_graph_ms_per_substep": t_b / steps * 1e3,
            "serial_64_contexts_ms_per_substep": t_s / steps * 1e3,
            "speedup": t_s / t_b,
            "active_per_substep": info["active_total"] / steps,
            "active_per_substep_serial": active_serial / steps,
            "interactions_per_s": info["interactions_total"] / t_b,
            "forces_all_active_ms": {"batched": f_b * 1e3, "serial_64_calls": f_s * 1e3,
                                     "speedup": f_s / f_b}}


def cpu_baseline(x, eps, theta, multipole, group_size, n_leaf, r_crit, target_s=15.0):
    """The float64 oracle walk on a random sample of the groups of the same
    all-active system (its tree preparation is not timed)."""
    import oracle
    t0 = time.perf_counter()
    k, _ = oracle.keys(x, 0)
    ks, perm = oracle.sort(k)
    tree = oracle.build(ks, n_leaf)
    ps = x[perm].astype(np.float64)
    mom = oracle.moments(tree, ps)
    grp = oracle.groups(np.ones(x.shape[0], np.uint8), ps, group_size, float(np.float32(r_crit)))
    prep = time.perf_counter() - t0
    ng = grp["first"].size
    rng = np.random.default_rng(7)
    nsel, spent, inter, done = 32, 0.0, 0, 0
    while spent < target_s and done < ng:
        sel = rng.choice(ng, size=min(nsel, ng), replace=False)
        t = time.perf_counter()
        _, cnt, _ = oracle.walk(tree, mom, ps, grp, eps, theta, multipole, gsel=sel)
        spent += time.perf_counter() - t
        inter += int(((cnt[sel, 0] + cnt[sel, 1]) * grp["count"][sel]).sum())
        done += sel.size
        nsel *= 2
    return dict(value=inter / spent, unit="interactions/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"float64 oracle walk of {done} random groups ({group_size} i-particles "
                       f"each) of the all-active step, {inter:.3e} interactions in {spent:.1f} s; "
                       f"tree preparation ({prep:.1f} s) not timed")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--group-size", type=int, default=32)
    ap.add_argument("--list-depth", type=int, default=384)
    ap.add_argument("--r-crit", type=float, default=0.25,
                    help="critical separation splitting groups (Section 2.4)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-shared", action="store_true", help="skip the shared-step run")
    ap.add_argument("--autotune", type=int, default=0, choices=(0, 1),
                    help="tune r_crit online during the block steps (Section 2.4)")
    ap.add_argument("--ball", type=int, default=2, choices=range(5),
                    help="enclosing ball of the groups (Appendix B): 0 GEO, 1 SEB, 2 EBS, 3 COM, 4 CMP")
    ap.add_argument("--rebuild-interval", type=int, default=0,
                    help="tree reuse: 0 = automatic (the growth models of Section 2.6), "
                         "1 = new tree every sub-step, k = every k sub-steps")
    ap.add_argument("--graph", type=int, default=1, choices=(0, 1),
                    help="replay each timed sub-step as captured HIP graphs (default 1)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-system batched / captured sub-step comparison")
    ap.add_argument("--forces-only", type=int, default=0, metavar="K",
                    help="only K all-active force evaluations of the workload (one checked, "
                         "K-1 unchecked; for counter runs) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profile to bytes) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nb = args.copy_calibration
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import ics
    import paper_1610_07279_amd as g

    n, eps, theta, eta, kmax, multipole = args.n, 1.0 / 512, 0.5, 0.1, 8, 2
    log(f"bench: generating NFW N={n} (seed 501)")
    x, v = ics.nfw(n, seed=501, with_vel=True)
    dev = torch.device("cuda", 0)
    if args.forces_only:
        ctx = g.Context(device=0, multipole=multipole, group_size=args.group_size,
                        list_depth=args.list_depth, r_crit=args.r_crit, timing=1)
        xd = torch.from_numpy(x).to(dev)
        out = ctx.tree_forces(xd, eps, theta)
        st = ctx.stats()
        ctx.set_params(check=0)
        for _ in range(args.forces_only - 1):
            ctx.tree_forces(xd, eps, theta, out=out)
        torch.cuda.synchronize()
        ms, k = ctx.walk_time()
        flags = ctx.stats()["flags"]
        print(json.dumps({"forces_only": args.forces_only, "n": n, "interactions": st["interactions"],
                          "node_interactions": st["node_interactions"],
                          "walk_ms_mean": ms / max(k, 1), "flags": flags}), flush=True)
        return
    pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
    vel0 = torch.from_numpy(v).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
    ctx = g.Context(device=0, multipole=multipole, group_size=args.group_size,
                    list_depth=args.list_depth, r_crit=args.r_crit, timing=1, graph=args.graph,
                    rebuild_interval=args.rebuild_interval, ball=args.ball,
                    autotune=args.autotune)

    log(f"bench: block steps (warmup {args.warmup}, timed {args.steps})")
    blk = run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, False, args.steps, args.warmup)
    log(f"bench: block {blk['seconds'] / args.steps * 1e3:.2f} ms/step, "
        f"{blk['info']['interactions_total'] / blk['seconds']:.3e} interactions/s, levels "
        f"{[c for c in blk['info']['level_count'] if c]}")
    shd = None
    if not args.no_shared:
        log("bench: shared steps")
        shd = run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, True, args.steps, args.warmup)
        log(f"bench: shared {shd['seconds'] / args.steps * 1e3:.2f} ms/step")

    ib = blk["info"]
    inter = ib["interactions_total"]
    quad = ib["node_interactions_total"]
    flops = FLOP_MONO * (inter - quad) + FLOP_QUAD * quad
    walk_s = blk["walk_ms"] / 1e3
    achieved = flops / walk_s / 1e12 if walk_s > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": inter / blk["seconds"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": blk["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"NFW sphere N={n}, c=10, eps=1/512, theta=0.5 quadrupole, "
                               f"block steps kmax=8 (eta=0.1), finest sub-steps",
                   "n": n, "group_size": args.group_size, "list_depth": args.list_depth,
                   "r_crit": args.r_crit, "graph": args.graph,
                   "rebuild_interval": args.rebuild_interval, "ball": args.ball,
                   "autotune": args.autotune,
                   "parallelism": "single GPU"},
        "block": {"s_per_step": blk["seconds"] / args.steps,
                  "interactions_per_s": inter / blk["seconds"],
                  "active_per_step": ib["active_total"] / args.steps,
                  "level_count": ib["level_count"][:kmax + 1],
                  "tree_builds": ib["tree_builds"],
                  "walk_ms_per_step": blk["walk_ms"] / max(blk["walk_launches"], 1)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": walk_traffic(),
                     "peak_nonpacked": FP32_PEAK_TFLOPS / 2,
                     "frac_nonpacked": achieved / (FP32_PEAK_TFLOPS / 2),
                     "kernel": "walk_k<2>", "flops_per_interaction": {"mono": FLOP_MONO,
                                                                       "quad": FLOP_QUAD}},
    }
    if shd is not None:
        inter_s = shd["info"]["interactions_total"]
        out["shared"] = {"s_per_step": shd["seconds"] / args.steps,
                         "tree_builds": shd["info"]["tree_builds"],
                         "interactions_per_s": inter_s / shd["seconds"],
                         "walk_ms_per_step": shd["walk_ms"] / max(shd["walk_launches"], 1)}
        out["speedup_block_vs_shared"] = shd["seconds"] / blk["seconds"]
    if not args.no_batched:
        log("bench: 64 systems, batched captured sub-steps vs 64 contexts")
        out["batched"] = batched_bench()
        log(f"bench: batched {out['batched']['batched_graph_ms_per_substep']:.2f} ms/sub-step, "
            f"serial {out['batched']['serial_64_contexts_ms_per_substep']:.2f}")
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(x, eps, theta, multipole, args.group_size, 16,
                                           args.r_crit)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
