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


def run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, shared, steps, warmup,
            class_groups=None):
    """class_groups: group size per sub-step class (S per step), or None."""
    import torch
    pos = pos0.clone()
    vel = vel0.clone()
    ctx.set_params(check=1)
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=eta, kmax=kmax, shared=shared)
    if class_groups and not shared:
        table = [class_groups[min(c, len(class_groups) - 1)] for c in range(kmax + 1)]
        ctx.sim_set_group_sizes(table)
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
    ctx.clear_flags()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sim_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = ctx.sim_info()
    walk_ms, launches = ctx.walk_time()
    st = ctx._stats_raw()
    if st["sticky_flags"]:  # any sub-step of the timed window, not only the last
        raise RuntimeError(f"device flags {st['sticky_flags']} set during the timed steps")
    last = {k: st[k] for k in ("n_active", "n_groups", "node_entries", "part_entries",
                               "interactions", "mac_tests")}
    ent = st["node_entries"] + st["part_entries"]
    # i-particles per group and list entry: the fraction of the walk's lanes
    # that carry an i-particle in the force loops of the last sub-step
    last["group_fill"] = st["interactions"] / max(ent * ctx.params["group_size"], 1)
    return dict(seconds=t1 - t0, info=info, walk_ms=walk_ms, walk_launches=launches,
                pos=pos.cpu().numpy().astype(np.float32), last=last)


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
    if ctx._stats_raw()["sticky_flags"]:
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, state, eps, theta, multipole, group_size, n_leaf, r_crit, ball, kmax,
                 window, target_s=15.0):
    """The float64 oracle walk on the workload of the timed block sub-steps:
    the particles (positions at the end of the timed run), their levels and
    last update sub-steps give the due sets of the next `window` sub-steps (no
    level changes assumed); random groups drawn uniformly from all groups of
    those sub-steps (r_crit, ball as the GPU run) are walked by the oracle
    until about target_s seconds; tree, moments and groups are not timed."""
    import oracle
    lev, last, s_now = state
    t0 = time.perf_counter()
    k, _ = oracle.keys(x, 0)
    ks, perm = oracle.sort(k)
    tree = oracle.build(ks, n_leaf)
    ps = x[perm].astype(np.float64)
    mom = oracle.moments(tree, ps)
    rc = float(np.float32(r_crit))
    per = []  # the groups of each sub-step (sub-steps with the same due set share them)
    seen = {}
    step = np.left_shift(1, kmax - lev.astype(np.int64))
    for t in range(s_now + 1, s_now + 1 + window):
        due = ((t - last) % step == 0) & (t > last)
        key = hash(np.packbits(due).tobytes())
        if key not in seen:
            seen[key] = oracle.groups(due[perm].astype(np.uint8), ps, group_size, rc, ball)
        per.append(seen[key])
    prep = time.perf_counter() - t0
    counts = np.array([p["first"].size for p in per], np.int64)
    ends = np.cumsum(counts)
    order = np.random.default_rng(7).permutation(int(ends[-1]))
    spent, inter, done, batch = 0.0, 0, 0, 32
    while spent < target_s and done < order.size:
        pick = order[done:done + batch]
        which = np.searchsorted(ends, pick, side="right")
        for w in np.unique(which):
            sel = pick[which == w] - (ends[w] - counts[w])
            grp = per[w]
            t = time.perf_counter()
            _, cnt, _ = oracle.walk(tree, mom, ps, grp, eps, theta, multipole, gsel=sel)
            spent += time.perf_counter() - t
            inter += int(((cnt[sel, 0] + cnt[sel, 1]) * grp["count"][sel]).sum())
        done += pick.size
        batch *= 2
    return dict(value=inter / spent, unit="interactions/s", cores=oracle.num_threads(),
                kind="oracle", cpu=cpu_model(),
                sample=f"float64 oracle walk of {done} groups drawn at random from the "
                       f"{int(counts.sum())} groups of the next {window} block sub-steps' due "
                       f"sets (G {group_size}, r_crit {r_crit}, ball {ball}, quadrupole), "
                       f"{inter:.3e} interactions in {spent:.1f} s on "
                       f"{oracle.num_threads()} threads of {cpu_model()}; tree and groups "
                       f"({prep:.1f} s) not timed")


def rel_error(tree, ref):
    """|a_tree - a_direct| / |a_direct| per target (acceleration as a vector)."""
    num = np.linalg.norm(tree[:, :3].astype(np.float64) - ref[:, :3], axis=1)
    return num / np.linalg.norm(ref[:, :3], axis=1)


def mac_sweep(args):
    """Time per step against force accuracy for the three MACs (Fig. 3 of
    Section 3.2): NFW sphere (r_s = 1, truncated at 5 r_s, seed 503), eps =
    r_s/64, quadrupole nodes.  Accuracy: the relative error of the acceleration
    vector of a random sample of particles (seed 504) against the float64 direct
    sum of the library, 50th and 99th percentiles, at t = 0 with every particle
    active (the acceleration MAC reads the accelerations of one opening-angle
    evaluation, theta = 0.5, as the previous step's).  Time: seconds per finest
    sub-step of the block and the shared scheme, as in the headline run.
    Parameters: theta = 0.9 ... 0.1 and Delta = 2^-2 ... 2^-18 (even powers)
    for the acceleration and the multipole MAC.  One JSON line per point."""
    import torch

    import ics
    import paper_1610_07279_amd as g

    n, eps, eta, kmax = args.n, 1.0 / 64, 0.1, 8
    log(f"mac sweep: NFW N={n}, truncated at 5 r_s (seed 503), eps 1/64")
    x, v = ics.nfw(n, seed=503, c=5.0, with_vel=True)
    dev = torch.device("cuda", 0)
    xd = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(504)
    idx = np.sort(rng.choice(n, size=min(args.sweep_sample, n), replace=False)).astype(np.int64)
    it = torch.from_numpy(idx).to(dev)
    t0 = time.perf_counter()
    ref = g.Context(device=0).direct_forces(xd, eps, idx=it).cpu().numpy()
    log(f"mac sweep: direct sum for {idx.size} targets in {time.perf_counter() - t0:.1f} s")
    base = dict(multipole=2, group_size=args.group_size, walk_width=args.walk_width, list_depth=args.list_depth,
                r_crit=args.r_crit, ball=args.ball, rebuild_interval=args.rebuild_interval)
    prev = g.Context(device=0, **base).tree_forces(xd, eps, 0.5)
    pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
    vel0 = torch.from_numpy(v).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
    points = [(0, 0.1 * k) for k in range(9, 0, -1)]
    points += [(m, 2.0 ** -e) for m in (1, 2) for e in range(2, 19, 2)]
    name = {0: "opening angle", 1: "acceleration", 2: "multipole"}
    for mac, val in points:
        theta = val if mac == 0 else 0.5
        ctx = g.Context(device=0, mac=mac, mac_delta=val if mac else 2.0 ** -7, timing=1,
                        graph=args.graph, **base)
        acc = ctx.tree_forces(xd, eps, theta, acc_old=prev if mac == 1 else None)
        e = rel_error(acc[it].cpu().numpy(), ref)
        inter = ctx.stats()["interactions"]
        blk = run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, False, args.steps,
                      args.warmup)
        shd = run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, True, args.steps,
                      args.warmup)
        row = {"mac": name[mac], "param": val, "err50": float(np.percentile(e, 50)),
               "err99": float(np.percentile(e, 99)), "interactions_all_active": inter,
               "block_s_per_step": blk["seconds"] / args.steps,
               "shared_s_per_step": shd["seconds"] / args.steps,
               "n": n, "sample": int(idx.size), "steps": args.steps}
        log(f"mac sweep: {name[mac]:13s} {val:.3g}: err50 {row['err50']:.2e} err99 "
            f"{row['err99']:.2e}  block {row['block_s_per_step'] * 1e3:.2f} ms  shared "
            f"{row['shared_s_per_step'] * 1e3:.2f} ms")
        print(json.dumps(row), flush=True)
        del ctx
        torch.cuda.empty_cache()


def ball_sweep(args):
    """The five enclosing balls of the pseudo i-particles (Appendix B, Fig. 10
    and Table 3) on two particle distributions of N = 2^23 with every particle
    active: the NFW sphere of the headline run (eps 1/512) and the
    three-component galaxy (NFW halo, Hernquist bulge, exponential disk; a
    stand-in for the M31 model, eps 1/512).  The groups do not depend on the
    ball, so each group's radius is compared with its smallest enclosing ball
    (SEB): percentiles of r_ball / r_SEB; plus the interactions and the walk
    time of an evaluation with each ball.  The cost of each ball kernel is the
    group_ball_k<kind> line of a kernel trace of this run.  One JSON line per
    (model, ball)."""
    import torch

    import ics
    import paper_1610_07279_amd as g

    n, eps, theta = args.n, 1.0 / 512, 0.5
    names = ["GEO", "SEB", "EBS", "COM", "CMP"]
    models = [("NFW", lambda: ics.nfw(n, seed=501)), ("galaxy", lambda: ics.galaxy(n))]
    for model, make in models:
        log(f"ball sweep: {model} N={n}")
        xd = torch.from_numpy(make()).to(torch.device("cuda", 0))
        radii, firsts = {}, {}
        for kind in (1, 0, 2, 3, 4):  # SEB first: the reference radius
            ctx = g.Context(device=0, multipole=2, group_size=args.group_size, walk_width=args.walk_width,
                            list_depth=args.list_depth, r_crit=args.r_crit, ball=kind, timing=1)
            out = ctx.tree_forces(xd, eps, theta)
            ctx.set_params(check=0)
            ctx.walk_time()
            for _ in range(args.steps):
                ctx.tree_forces(xd, eps, theta, out=out)
            torch.cuda.synchronize()
            ms, k = ctx.walk_time()
            st = ctx.stats()
            grp = ctx.groups()
            radii[kind], firsts[kind] = grp["ball"][:, 3].astype(np.float64), grp["first"]
            if not np.array_equal(firsts[kind], firsts[1]):
                raise RuntimeError("the groups changed with the ball kind")
            seb = radii[1]
            ok = seb > 0
            q = radii[kind][ok] / seb[ok]
            row = {"model": model, "ball": names[kind], "n": n, "groups": int(st["n_groups"]),
                   "ratio_p50": float(np.percentile(q, 50)), "ratio_p90": float(np.percentile(q, 90)),
                   "ratio_p99": float(np.percentile(q, 99)), "ratio_max": float(q.max()),
                   "interactions": st["interactions"], "walk_ms": ms / max(k, 1)}
            log(f"ball sweep: {model:6s} {names[kind]}: r/r_SEB p50 {row['ratio_p50']:.4f} p99 "
                f"{row['ratio_p99']:.4f} max {row['ratio_max']:.4f}, interactions "
                f"{row['interactions']:.4e}, walk {row['walk_ms']:.2f} ms")
            print(json.dumps(row), flush=True)
            del ctx
        del xd
        torch.cuda.empty_cache()


def n_sweep(args):
    """Time per step against the number of particles (Fig. 8 of Section 3.4):
    the NFW sphere of the headline run (c = 10, seed 501; the paper shows the
    M31 model and quotes the NFW sphere at 2^23 and 2^24), eps 1/512, the
    acceleration MAC with Delta = 2^-7, quadrupole nodes, block
    steps on 8 levels, at N = 2^10, 2^12, ..., 2^24 (or the one N of --n);
    seconds per finest sub-step of the block and the shared scheme and the part
    spent in the walk kernel (HIP events).  The split over the other functions
    comes from kernel traces of runs at one N each (--n N --no-shared).  One
    JSON line per N."""
    import torch

    import ics
    import paper_1610_07279_amd as g

    eps, eta, kmax = 1.0 / 512, 0.1, 8
    dev = torch.device("cuda", 0)
    sizes = [args.n] if "--n" in sys.argv else [1 << lg for lg in range(10, 25, 2)]
    for n in sizes:
        x, v = ics.nfw(n, seed=501, with_vel=True)
        pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
        vel0 = torch.from_numpy(v).to(dev)
        mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
        ctx = g.Context(device=0, multipole=2, group_size=args.group_size, walk_width=args.walk_width,
                        list_depth=args.list_depth, r_crit=args.r_crit, timing=1,
                        graph=args.graph, rebuild_interval=args.rebuild_interval, ball=args.ball,
                        mac=1, mac_delta=2.0 ** -7)
        row = {"n": n, "steps": args.steps, "model": "NFW", "mac": "acceleration 2^-7"}
        modes = (("block", False),) if args.no_shared else (("block", False), ("shared", True))
        for mode, shared in modes:
            r = run_sim(ctx, pos0, vel0, mass, eps, 0.5, eta, kmax, shared, args.steps,
                        args.warmup)
            row[f"{mode}_s_per_step"] = r["seconds"] / args.steps
            row[f"{mode}_walk_s_per_step"] = r["walk_ms"] / 1e3 / args.steps
            row[f"{mode}_interactions_per_s"] = r["info"]["interactions_total"] / r["seconds"]
            row[f"{mode}_tree_builds"] = r["info"]["tree_builds"]
        msg = (f"n sweep: N={n}: block {row['block_s_per_step'] * 1e3:.3f} ms (walk "
               f"{row['block_walk_s_per_step'] * 1e3:.3f})")
        if not args.no_shared:
            msg += (f", shared {row['shared_s_per_step'] * 1e3:.3f} ms (walk "
                    f"{row['shared_walk_s_per_step'] * 1e3:.3f})")
        log(msg)
        print(json.dumps(row), flush=True)
        del ctx, pos0, vel0, mass
        torch.cuda.empty_cache()


def _rel_stats(tree, ref):
    """global rms, 50th / 99th percentile / max of |a_tree - a_ref| / |a_ref|."""
    e = rel_error(tree, ref)
    d = tree[:, :3].astype(np.float64) - ref[:, :3]
    g = float(np.sqrt((d ** 2).sum() / (ref[:, :3] ** 2).sum()))
    return {"rms": g, "p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
            "max": float(e.max())}


def _time_forces(ctx, xd, eps, theta, out, reps, warm=3):
    """wall ms per evaluation (reps back-to-back, unchecked) and walk ms (events)."""
    import torch
    for _ in range(warm):
        ctx.tree_forces(xd, eps, theta, out=out)
    torch.cuda.synchronize()
    ctx.walk_time()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.tree_forces(xd, eps, theta, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps * 1e3
    ms, k = ctx.walk_time()
    return wall, ms / max(k, 1)


def config_c1(args):
    """Plummer N = 8192 (seed 101), eps 1/64, theta 0.5, monopole, one
    shared-step force with every particle active: GPU time per evaluation
    (latency-bound at this N), interactions, errors against the library's
    float64 direct sum; cpu_baseline: the float64 oracle's direct sum and tree
    on every host thread, and the GPU forces against the oracle tree."""
    import torch

    import ics
    import paper_1610_07279_amd as g
    n, eps, theta = 8192, 1 / 64, 0.5
    x = ics.plummer(n, seed=101)
    xd = torch.from_numpy(x).cuda()
    ctx = g.Context(device=0, timing=1)
    out = ctx.tree_forces(xd, eps, theta)
    st = ctx.stats()
    ctx.set_params(check=0)
    wall, walk = _time_forces(ctx, xd, eps, theta, out, reps=200)
    a = out.cpu().numpy()
    # the same evaluation captured once in a HIP graph by the caller and replayed
    # (the pipeline is some two hundred small launches at this N)
    ctx.set_params(timing=0)
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        ctx.tree_forces(xd, eps, theta, out=out)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(200):
        graph.replay()
    torch.cuda.synchronize()
    replay_us = (time.perf_counter() - t0) / 200 * 1e6
    if not np.array_equal(out.cpu().numpy(), a):
        raise RuntimeError("the captured evaluation differs from the eager one")
    ref = g.Context(device=0).direct_forces(xd, eps).cpu().numpy()
    # the same evaluation with the tunables gothic_autotune picks for it
    tctx = g.Context(device=0, timing=1)
    res = tctx.autotune(xd, eps, theta)
    tout = tctx.tree_forces(xd, eps, theta)
    tst = tctx.stats()
    tctx.set_params(check=0)
    twall, twalk = _time_forces(tctx, xd, eps, theta, tout, reps=200)
    row = {"config": "C1", "workload": "Plummer N=8192 (seed 101), eps 1/64, theta 0.5, "
                                        "monopole, all active",
           "us_per_evaluation": wall * 1e3, "us_per_evaluation_graph_replay": replay_us,
           "walk_us": walk * 1e3,
           "interactions": st["interactions"], "groups": st["n_groups"],
           "vs_float64_direct": _rel_stats(a, ref),
           "tuned": {"autotune": {k: res[k] for k in ("group_size", "walk_width", "list_depth",
                                                      "r_crit", "evaluations")},
                     "us_per_evaluation": twall * 1e3, "walk_us": twalk * 1e3,
                     "interactions": tst["interactions"], "groups": tst["n_groups"],
                     "vs_float64_direct": _rel_stats(tout.cpu().numpy(), ref)}}
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        od = oracle.direct(x, eps)
        t_direct = time.perf_counter() - t0
        t0 = time.perf_counter()
        ot = oracle.tree_forces(x, eps, theta)
        t_tree = time.perf_counter() - t0
        row["vs_float64_oracle_tree"] = _rel_stats(a, ot["acc_pot"])
        row["oracle_tree_vs_direct"] = _rel_stats(ot["acc_pot"].astype(np.float32), od)
        row["cpu_baseline"] = {"kind": "oracle", "cores": oracle.num_threads(), "cpu": cpu_model(),
                               "direct_s": t_direct, "tree_s": t_tree,
                               "value": 1.0 / t_tree, "unit": "evaluations/s (tree)",
                               "sample": "one whole evaluation of each (float64; tree: keys, "
                                         "sort, octree, moments, groups, walk)"}
    return row


def config_c2(args):
    """NFW N = 2^20 (seed 201), eps 1/128, quadrupole, theta 0.5, block steps
    on kmax = 8 levels: one full block cycle (2^(kmax - k_lo) finest sub-steps,
    k_lo the coarsest populated level at t = 0), timed after one untimed cycle,
    against shared steps at the finest step (mean of 5 after 2 untimed);
    speed-up = 2^(kmax - k_lo) t_shared / t_cycle.  cpu_baseline: the float64
    oracle walk on a sample of groups of an all-active evaluation."""
    import torch

    import ics
    import paper_1610_07279_amd as g
    n, eps, theta, kmax = 1 << 20, 1 / 128, 0.5, 8
    x, v = ics.nfw(n, seed=201, with_vel=True)
    dev = torch.device("cuda", 0)
    pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
    vel0 = torch.from_numpy(v).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
    kw = dict(multipole=2, group_size=args.group_size, walk_width=args.walk_width, list_depth=args.list_depth,
              r_crit=args.r_crit, ball=args.ball, rebuild_interval=args.rebuild_interval,
              graph=args.graph, timing=1)
    ctx = g.Context(device=0, **kw)
    pos, vel = pos0.clone(), vel0.clone()
    ctx.sim_bind(pos, vel, mass, eps, theta, eta=0.1, kmax=kmax)
    hist0 = ctx.sim_info()["level_count"][:kmax + 1]
    k_lo = min(k for k, c in enumerate(hist0) if c)
    cycle = 1 << (kmax - k_lo)
    ctx.set_params(check=0)
    ctx.sim_step(cycle)  # untimed cycle: captures, first trees
    torch.cuda.synchronize()
    ctx.sim_reset_counters()
    t0 = time.perf_counter()
    ctx.sim_step(cycle)
    torch.cuda.synchronize()
    t_cycle = time.perf_counter() - t0
    ib = ctx.sim_info()
    if ctx._stats_raw()["sticky_flags"]:
        raise RuntimeError("device flags set in the block cycle")
    shd = run_sim(g.Context(device=0, **kw), pos0, vel0, mass, eps, theta, 0.1, kmax, True, 5, 2)
    t_shared = shd["seconds"] / 5
    row = {"config": "C2", "workload": "NFW N=2^20 (seed 201), eps 1/128, theta 0.5, "
                                        "quadrupole, block steps kmax 8",
           "level_count_t0": hist0, "k_lo": k_lo, "cycle_substeps": cycle,
           "cycle_s": t_cycle, "cycle_interactions": ib["interactions_total"],
           "cycle_tree_builds": ib["tree_builds"],
           "cycle_interactions_per_s": ib["interactions_total"] / t_cycle,
           "shared_s_per_step": t_shared,
           "shared_interactions_per_s": shd["info"]["interactions_total"] / shd["seconds"],
           "speedup_block_vs_shared": cycle * t_shared / t_cycle,
           "level_count_end": ib["level_count"][:kmax + 1],
           "tunables": {k: kw[k] for k in ("group_size", "list_depth", "r_crit", "ball")}}
    if not args.no_cpu:
        lev = np.full(n, kmax, np.uint8)
        last = np.zeros(n, np.int64)
        row["cpu_baseline"] = cpu_baseline(x, (lev, last, 0), eps, theta, 2, args.group_size, 16,
                                           args.r_crit, args.ball, kmax, 1, target_s=10.0)
    return row


def config_c3(args):
    """Galaxy N = 2^22 (NFW halo 80 %, Hernquist bulge 5 %, exponential disk
    15 %; seeds 301-303), eps 1/256, theta 0.5, monopole, all active: float32
    and Neumaier-compensated accumulation, errors against the library's float64
    direct sum on 4096 random particles (seed 304); cpu_baseline: the float64
    oracle's direct sum for the same 4096 targets."""
    import torch

    import ics
    import paper_1610_07279_amd as g
    n, eps, theta = 1 << 22, 1 / 256, 0.5
    x = ics.galaxy(n)
    xd = torch.from_numpy(x).cuda()
    idx = np.sort(np.random.default_rng(304).choice(n, 4096, replace=False)).astype(np.int64)
    it = torch.from_numpy(idx).cuda()
    ref = g.Context(device=0).direct_forces(xd, eps, idx=it).cpu().numpy()
    row = {"config": "C3", "workload": "galaxy N=2^22 (seeds 301-303), eps 1/256, theta 0.5, "
                                        "monopole, all active; 4096 targets (seed 304)"}
    outs = {}
    for comp in (0, 1):
        ctx = g.Context(device=0, timing=1, compensated=comp, group_size=args.group_size, walk_width=args.walk_width,
                        list_depth=args.list_depth)
        out = ctx.tree_forces(xd, eps, theta)
        st = ctx.stats()
        ctx.set_params(check=0)
        wall, walk = _time_forces(ctx, xd, eps, theta, out, reps=5, warm=1)
        a = out[it].cpu().numpy()
        outs[comp] = a
        row["compensated" if comp else "fp32"] = {
            "ms_per_evaluation": wall, "walk_ms": walk, "interactions": st["interactions"],
            "vs_float64_direct": _rel_stats(a, ref)}
    d = outs[0][:, :3].astype(np.float64) - outs[1][:, :3]
    row["fp32_vs_compensated_rms"] = float(np.sqrt((d ** 2).sum() / (ref[:, :3] ** 2).sum()))
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        od = oracle.direct(x, eps, idx=idx)
        t_direct = time.perf_counter() - t0
        row["library_direct_vs_oracle_direct"] = _rel_stats(ref.astype(np.float64), od)
        row["cpu_baseline"] = {"kind": "oracle", "cores": oracle.num_threads(),
                               "cpu": cpu_model(), "direct_s": t_direct,
                               "value": 4096.0 * n / t_direct, "unit": "pairs/s",
                               "sample": f"float64 direct sum of 4096 targets against all {n}"}
    return row


def config_c4(args):
    """64 systems (N_s log-uniform in [2^12, 2^18], Plummer / NFW, seed 401),
    monopole, theta 0.5: the timed autotuner's choice of (group size, walk
    width, list depth, r_crit) for one all-active batched evaluation, its time
    against the default tunables, and the batched block-step comparison of the
    headline run (one captured batched sub-step vs 64 contexts)."""
    import torch

    import ics
    import paper_1610_07279_amd as g
    x, offs, eps, _ = ics.batched_systems(64, seed=401, with_vel=True)
    n = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    ctx = g.Context(device=0)
    res = ctx.autotune(xt, eps, 0.5, offsets=offs, out=out)
    ref = g.Context(device=0, check=0)
    ref.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        ref.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    t_def = (time.perf_counter() - t0) / 10 * 1e3
    ctx.set_params(check=0)
    ctx.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        ctx.tree_forces_batched(xt, offs, eps, 0.5, out=out)
    torch.cuda.synchronize()
    t_tuned = (time.perf_counter() - t0) / 10 * 1e3
    row = {"config": "C4", "workload": f"64 systems, N={n} in all", "autotune": res,
           "all_active_ms_default": t_def, "all_active_ms_tuned": t_tuned}
    row["batched_block_steps"] = batched_bench()
    return row


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--group-size", type=int, default=32)
    ap.add_argument("--walk-width", type=int, default=64, choices=(16, 32, 64),
                    help="lanes sharing one traversal (64: one group per wave)")
    ap.add_argument("--class-groups", default="auto",
                    help="group size per sub-step class of the block steps (S per step), "
                         "comma-separated from class 0 (the last value repeats); 'auto' "
                         "(default, with --walk-width 64 and no --autotune 2): 1,<--group-size>, "
                         "i.e. in the sparse "
                         "class 0 (only the finest level due) every due particle walks the tree "
                         "alone with 64 lanes, the other classes groups of --group-size "
                         "(measured at NFW 2^24, fixed rebuild interval 4: 12.03 against 12.42 "
                         "ms per sub-step with 8,32); '' = --group-size for every class")
    ap.add_argument("--list-depth", type=int, default=384)
    ap.add_argument("--r-crit", type=float, default=0.25,
                    help="critical separation splitting groups (Section 2.4)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-shared", action="store_true", help="skip the shared-step run")
    ap.add_argument("--autotune", type=int, default=0, choices=(0, 1, 2),
                    help="1: tune r_crit online during the block steps (Section 2.4); 2: first "
                         "pick the group size of each sub-step class, then tune r_crit")
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
    ap.add_argument("--sweep", choices=("mac", "ball", "n"), default=None,
                    help="mac: time per step against force accuracy for the three MACs; "
                         "ball: the five enclosing balls (both at N = 2^23 unless --n is "
                         "given); n: time per step for N = 2^10 ... 2^24; then exit")
    ap.add_argument("--sweep-sample", type=int, default=1 << 14,
                    help="particles whose force error a sweep measures")
    ap.add_argument("--config", choices=("C1", "C2", "C3", "C4"), default=None,
                    help="the report of one of the smaller workloads (C1 Plummer 8192 forces, "
                         "C2 NFW 2^20 block cycle vs shared, C3 galaxy 2^22 float32 vs "
                         "compensated, C4 64 batched systems with the autotuner), one JSON "
                         "line, then exit")
    args = ap.parse_args()
    if args.config:
        fn = {"C1": config_c1, "C2": config_c2, "C3": config_c3, "C4": config_c4}[args.config]
        print(json.dumps(fn(args)), flush=True)
        return
    if args.sweep:
        if "--n" not in sys.argv:
            args.n = 1 << 23
        {"mac": mac_sweep, "ball": ball_sweep, "n": n_sweep}[args.sweep](args)
        return
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
        ctx = g.Context(device=0, multipole=multipole, group_size=args.group_size, walk_width=args.walk_width,
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
                          "node_entries": st["node_entries"], "part_entries": st["part_entries"],
                          "n_groups": st["n_groups"], "mac_tests": st["mac_tests"],
                          "walk_ms_mean": ms / max(k, 1), "flags": flags}), flush=True)
        return
    pos0 = torch.from_numpy(x[:, :3].astype(np.float64)).to(dev)
    vel0 = torch.from_numpy(v).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(x[:, 3])).to(dev)
    ctx = g.Context(device=0, multipole=multipole, group_size=args.group_size, walk_width=args.walk_width,
                    list_depth=args.list_depth, r_crit=args.r_crit, timing=1, graph=args.graph,
                    rebuild_interval=args.rebuild_interval, ball=args.ball,
                    autotune=args.autotune)

    log(f"bench: block steps (warmup {args.warmup}, timed {args.steps})")
    if args.class_groups == "auto":
        # the online picker (autotune 2) chooses the shapes itself
        args.class_groups = (f"1,{args.group_size}"
                             if args.walk_width == 64 and args.autotune != 2 else "")
    class_groups = [int(v) for v in args.class_groups.split(",") if v.strip()]
    blk = run_sim(ctx, pos0, vel0, mass, eps, theta, eta, kmax, False, args.steps, args.warmup,
                  class_groups=class_groups or None)
    tuning = None
    if args.autotune:
        # the online tuner's state after the block run: r_crit and (with
        # autotune 2) the group shape picked for each sub-step class
        r, k, gs, ws = ctx.sim_tuning(kmax + 1, with_groups=True)
        tuning = [{"class": c, "group_size": int(gs[c]), "walk_width": int(ws[c]),
                   "r_crit_best": float(r[c]), "searches": int(k[c])} for c in range(kmax + 1)]
    # the state the CPU baseline's due sets come from (end of the block run)
    _, lev_end, last_end = ctx.sim_state()
    state_end = (lev_end, last_end, blk["info"]["substep"])
    x_end = x.copy()
    x_end[:, :3] = blk["pos"]
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
                   "n": n, "group_size": args.group_size, "walk_width": args.walk_width,
                   "list_depth": args.list_depth, "r_crit": args.r_crit, "graph": args.graph,
                   "rebuild_interval": args.rebuild_interval, "ball": args.ball,
                   "autotune": args.autotune, "class_groups": args.class_groups or None,
                   "parallelism": "single GPU"},
        "block": {"s_per_step": blk["seconds"] / args.steps,
                  "interactions_per_s": inter / blk["seconds"],
                  "interactions": inter,
                  "quad_node_interactions": quad,
                  "mono_interactions": inter - quad,
                  "active_per_step": ib["active_total"] / args.steps,
                  "level_count": ib["level_count"][:kmax + 1],
                  "tree_builds": ib["tree_builds"],
                  "walk_launches": blk["walk_launches"],
                  "walk_ms_per_step": blk["walk_ms"] / max(blk["walk_launches"], 1),
                  "last_substep": blk["last"]},
        # achieved = (mono x 24 + quad x 60) flop / (walk launches x walk_ms_mean),
        # the walk timed by HIP events around every launch on its own stream
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": walk_traffic(),
                     "traffic_source": "profiles/walk_nfw16m_hbm_traffic.md: rocprofv3 "
                                       "FETCH_SIZE + WRITE_SIZE per walk launch, scaled by a "
                                       "copy kernel; null unless the walk source is the one "
                                       "the counters were taken on",
                     "kernel": "walk_k<2>", "flops": flops,
                     "walk_ms_mean": blk["walk_ms"] / max(blk["walk_launches"], 1),
                     "flops_per_interaction": {"mono": FLOP_MONO, "quad": FLOP_QUAD}},
    }
    if tuning is not None:
        out["block"]["tuning_per_class"] = tuning
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
        out["cpu_baseline"] = cpu_baseline(x_end, state_end, eps, theta, multipole,
                                           args.group_size, 16, args.r_crit, args.ball, kmax,
                                           args.steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
