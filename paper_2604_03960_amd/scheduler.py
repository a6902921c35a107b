"""Learned bond-dimension scheduler: dataset, training and evaluation helpers.

The network (25 -> 64 -> 64 -> 1, see include/tna.h) is the learned stand-in
for the predictive scheduler of Sec. 7 of the paper.  Training data are the
per-visit records of DMRG runs of this library: the inputs are the 25
scheduler features the sweep logs at each visit (last 8 EMA entropies, 16
largest log singular values, relative bond position); the label of visit t
of a bond is log2 of the smallest rank whose truncation error meets the
target at the bond's next visit, clamped to [chi_min, chi_max].  Training and
inference run in the library's FP32 kernels; this module only assembles
arrays.  Random numbers (initial weights, epoch orders) come from `synth`.
"""
from __future__ import annotations

import math

import numpy as np

import synth

from . import MLP_NPARAM, Mlp


def build_dataset(runs, chi_min: int, chi_max: int):
    """runs: iterable of per-chain visit-record lists (in visit order).
    Returns X (n, 25) float32 and T (n,) float32."""
    xs, ts = [], []
    for recs in runs:
        last = {}
        for r in recs:
            b = int(r["bond"])
            if b in last:
                k = min(max(int(r["k_needed"]), chi_min), chi_max)
                xs.append(last[b])
                ts.append(math.log2(k))
            last[b] = np.asarray(r["feat"], dtype=np.float32)
    if not xs:
        return np.zeros((0, 25), np.float32), np.zeros(0, np.float32)
    return np.stack(xs).astype(np.float32), np.asarray(ts, dtype=np.float32)


def init_params(seed: int = 0) -> np.ndarray:
    """Weights N(0, 1/fan_in), biases 0, output bias log2(16)."""
    z = synth.normal(seed, MLP_NPARAM)
    p = np.zeros(MLP_NPARAM)
    o = 0
    for fan_in, n_w, n_b in ((25, 64 * 25, 64), (64, 64 * 64, 64), (64, 64, 1)):
        p[o:o + n_w] = z[o:o + n_w] / math.sqrt(fan_in)
        o += n_w + n_b
    p[-1] = 4.0
    return p.astype(np.float32)


def normalization(X: np.ndarray):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


def train(ctx, X: np.ndarray, T: np.ndarray, epochs: int = 100, batch: int = 256, lr: float = 1e-3, seed: int = 0):
    """Trains a fresh network on the device; returns (Mlp, per-epoch losses)."""
    import torch
    net = Mlp(ctx, init_params(seed))
    mean, std = normalization(X)
    net.set_normalization(mean, std)
    n = X.shape[0]
    perm = np.stack([np.argsort(synth.uniform53(seed * 7919 + e, 0, n)) for e in range(epochs)]).astype(np.int32)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T)).cuda()
    Pd = torch.from_numpy(perm).cuda()
    losses = net.train(Xd, Td, Pd, epochs=epochs, batch=batch, lr=lr)
    return net, losses


def summarize(recs, eps_target: float):
    """Cost and accuracy summary of one run's visit records."""
    k = np.array([r["k"] for r in recs], dtype=np.float64)
    eps = np.array([r["eps"] for r in recs])
    fb = np.array([r.get("fallback", 0) for r in recs])
    sched = np.array([r.get("chi_sched", 0) for r in recs])
    used = sched > 0
    return {
        "visits": len(recs),
        "sum_k3": float(np.sum(k ** 3)),
        "mean_k": float(k.mean()),
        "frac_eps_ok": float(np.mean(eps <= eps_target)),
        "max_eps": float(eps.max()),
        "fallback_rate": float(fb[used].mean()) if used.any() else 0.0,
        "scheduler_visits": int(used.sum()),
    }
