"""Learned warm start: training and use of the network that predicts the GDP
multipliers from local geometry (not part of the paper's method).

Training data are produced by the method itself: instances are solved cold
to a certified optimum and every node contributes (features, lambda*/scale),
lambda* = Lam*/2 of the certificate's duals.  Features, forward, backward and
the optimizer all run in libf2m's kernels (BF16 MFMA operands, FP32
accumulate); this module only sequences them.

    python -m paper_2011_08170_amd.warm --instances 2000 --out weights.npy

A solve with `mlp_theta=` starts the GDP from round-half-even(2*scale*y);
the certified optimum is the cold start's, only the iteration count changes.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import f2m, instances

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warm_mlp.npy")


def init_theta(seed=0):
    """He-style initial parameters (FP32), in the library's order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.normal(0, math.sqrt(2.0 / 16), 128 * 16), np.zeros(128),
             rng.normal(0, math.sqrt(2.0 / 128), 128 * 128), np.zeros(128),
             rng.normal(0, math.sqrt(1.0 / 128), 128), np.zeros(1)]
    t = np.concatenate(parts).astype(np.float32)
    assert t.size == f2m.MLP_PARAMS
    return t


def make_dataset(ctx, count, lo=5000, hi=50000, seed=10000, log=print):
    """Cold-solves `count` instances (sizes log-uniform in [lo, hi], half
    uniform, half clustered) and returns device tensors (features, targets)."""
    import torch
    sizes = instances.batch_sizes(count, lo, hi, seed)
    feats, targs = [], []
    t0 = time.time()
    for i, n in enumerate(sizes):
        s = seed + i
        xy = instances.uniform(int(n), 1_000_000, s) if i % 2 == 0 else instances.clustered(int(n), 1_000_000, s)
        d = torch.from_numpy(xy).cuda()
        r = ctx.solve(d)
        if not r["certified"]:
            continue
        feat = torch.empty((int(n), 16), dtype=torch.int16, device="cuda")
        scale = ctx.features(d, feat)
        lam = torch.from_numpy(r["lambda2"].astype(np.float64) / (2.0 * scale)).float().cuda()
        feats.append(feat)
        targs.append(lam)
        if log and (i + 1) % max(1, count // 20) == 0:
            log("  dataset %d/%d instances, %.1f s" % (i + 1, count, time.time() - t0))
    return torch.cat(feats), torch.cat(targs)


def train(ctx, feat, target, epochs=4, batch=65536, lr=2e-3, wd=1e-4, seed=0, log=print):
    """AdamW with cosine decay on the library's gradient kernels."""
    import torch
    theta = torch.from_numpy(init_theta(seed)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    n = target.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps = epochs * ((n + batch - 1) // batch)
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            fb = feat[idx].contiguous()
            tb = target[idx].contiguous()
            loss = ctx.mlp_grad(theta, fb, tb, grad)
            step += 1
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
            ctx.mlp_adamw(theta, grad, m, v, step, cur, wd)
            tot += loss * idx.shape[0]
        losses.append(tot / n)
        if log:
            log("  epoch %d: mse %.5f" % (ep, losses[-1]))
    return theta, losses


def load(path=DEFAULT_WEIGHTS):
    """Trained parameters as a CUDA tensor."""
    import torch
    return torch.from_numpy(np.load(path, allow_pickle=False).astype(np.float32)).cuda()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=2000)
    ap.add_argument("--lo", type=int, default=5000)
    ap.add_argument("--hi", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)   # noqa: E731
    with f2m.Context(0) as ctx:
        t = time.time()
        feat, target = make_dataset(ctx, args.instances, args.lo, args.hi, log=log)
        log("dataset: %d nodes in %.1f s" % (target.shape[0], time.time() - t))
        t = time.time()
        theta, losses = train(ctx, feat, target, epochs=args.epochs, log=log)
        log("training: %.1f s" % (time.time() - t))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, theta.cpu().numpy())
    log("saved", args.out)


if __name__ == "__main__":
    main()
