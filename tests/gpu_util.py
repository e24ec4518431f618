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
