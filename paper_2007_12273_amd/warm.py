"""Training driver of the learned warm start (host loop over library calls).

The network, its loss, gradients and optimiser run in the gm_warm kernels;
this module only draws the mini-batch order and sequences the calls:

  1. fit each training cell with plain (cold-start) EM on the GPU,
  2. compute features, frames and whitened targets of those fits,
  3. run Adam over shuffled mini-batches for a fixed number of epochs.
"""
from __future__ import annotations

import time

import torch

from . import api


def training_set(batches, kmax, seed=0, device="cuda"):
    """Features [N, 128] and targets [N, 160] (device tensors) of every cell
    in `batches`, a list of {v, alpha, cell_off} host arrays; the targets
    are the plain-EM fits of the cells."""
    feats, targs = [], []
    for b in batches:
        v = torch.from_numpy(b["v"]).to(device)
        a = torch.from_numpy(b["alpha"]).to(device)
        off = torch.from_numpy(b["cell_off"]).to(device)
        r = api.compress(v, a, off, kmax, seed=seed)
        f, fr = api.warm_features(v, a, off)
        feats.append(f)
        targs.append(api.warm_targets(r, fr))
        del v, a, off, r
    return torch.cat(feats), torch.cat(targs)


def train(model, feats, targets, epochs=50, lr=1e-3, lam=1.0, seed=0, log=None):
    """Adam over shuffled mini-batches of model.batch rows (the last partial
    batch of each epoch is dropped).  Returns per-epoch mean batch losses."""
    n = feats.shape[0]
    B = model.batch
    steps = n // B
    if steps < 1:
        raise ValueError("need at least one full batch of %d rows, have %d" % (B, n))
    gen = torch.Generator(device="cpu").manual_seed(seed)
    loss_rows = torch.zeros(steps, B, dtype=torch.float32, device=feats.device)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(torch.int32).to(feats.device)
        for s in range(steps):
            model.train_step(feats, targets, perm[s * B:(s + 1) * B], lr=lr, lam=lam, loss_rows=loss_rows[s])
        hist.append(float(loss_rows.sum().item()) / (steps * B))
        if log is not None:
            log("epoch %d: loss %.4f (%.1f s)" % (ep + 1, hist[-1], time.perf_counter() - t0))
    return hist
