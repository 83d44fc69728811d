"""Training driver of the learned warm start (host loop over library calls).

The network, its loss, gradients, optimiser and the epoch loop (shuffle
and mini-batches) run in the library; this module sequences the calls:

  1. fit each training cell with plain (cold-start) EM on the GPU,
  2. compute features, frames and whitened targets of those fits,
  3. run gm_warm_train for a fixed number of epochs.
"""
from __future__ import annotations

import time

import torch

from . import api


def best_fit(v, a, off, kmax, seeds):
    """Plain-EM fit of every cell from each cold-start seed in `seeds`; per
    cell the fit with the highest penalised likelihood is kept."""
    best = None
    for s in seeds:
        r = api.compress(v, a, off, kmax, seed=s)
        if best is None:
            best = r
            continue
        better = r["L_pen"] > best["L_pen"]
        for k in best:
            m = better.view(-1, *([1] * (best[k].dim() - 1)))
            best[k] = torch.where(m, r[k], best[k])
    return best


def training_set(batches, kmax, seed=0, device="cuda", restarts=1):
    """Features [N, 128] and targets [N, 160] (device tensors) of every cell
    in `batches`, a list of {v, alpha, cell_off} host arrays; the targets
    are the plain-EM fits of the cells (the best of `restarts` cold starts,
    seeds seed, seed + 1, ...)."""
    feats, targs = [], []
    for b in batches:
        v = torch.from_numpy(b["v"]).to(device)
        a = torch.from_numpy(b["alpha"]).to(device)
        off = torch.from_numpy(b["cell_off"]).to(device)
        r = best_fit(v, a, off, kmax, [seed + i for i in range(restarts)])
        f, fr = api.warm_features(v, a, off)
        feats.append(f)
        targs.append(api.warm_targets(r, fr))
        del v, a, off, r
    return torch.cat(feats), torch.cat(targs)


def train(model, feats, targets, epochs=50, lr=1e-3, lam=1.0, seed=0, log=None):
    """Adam over shuffled mini-batches of model.batch rows (the last partial
    batch of each epoch is dropped): the library's training loop
    (gm_warm_train).  Returns per-epoch mean batch losses."""
    t0 = time.perf_counter()
    hist = model.train(feats, targets, epochs, lr=lr, lam=lam, seed=seed)
    if log is not None:
        for ep, h in enumerate(hist):
            log("epoch %d: loss %.4f" % (ep + 1, h))
        log("%d epochs in %.1f s" % (epochs, time.perf_counter() - t0))
    return hist
