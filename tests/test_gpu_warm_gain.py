"""What the trained warm-start network gains over the method without it.

The network is trained (gm_warm_train) on plain-EM fits of held-out
batches of the Weibel-like recipe and evaluated on a fresh batch, under the
judged protocol the benchmark uses: a cell whose warm-started fit ends with
a penalised likelihood more than 1e-4 (relative) below the cold fit's is
refitted from the cold start and its cold record is the output, so every
cell's output is at least as good as plain EM's to that margin.  EM work is
counted in component updates (visits): the warm fit of every cell plus the
cold refit of the judged cells, against the cold fit of every cell.

Asserted:
* the trained network cuts the work below 0.85 of plain EM's (measured
  0.69 on 4096 cells), while an untrained network of the same shape (its
  start keeps all sixteen slots) and a cold fit from another seed both cost
  more than plain EM;
* the refit of the judged cells, run on a batch in which every other cell
  is empty so that each cell keeps its index and therefore its cold-start
  draws, reproduces the cold fit of those cells bit for bit (K, L_pen,
  visits, mixture) -- the benchmark's refit does exactly this;
* the protocol's output conserves mass, momentum and the second-moment
  tensor of every cell to 1e-12 and keeps every cell's penalised likelihood
  within 1e-4 of plain EM's or above it.
The trained network's judged fraction (about 0.54) is higher than that of a
reseeded cold fit (about 0.31): its starts land in worse local maxima more
often than a random restart does, and the gain comes from the much shorter
fits of the other cells.  The fractions are printed and bounded loosely.
"""
import numpy as np
import pytest

from paper_2007_12273_amd import synth

from gpu_util import dev, host, torch

pytestmark = pytest.mark.gpu

JUDGE_REL = 1e-4


def _gpu(d):
    g = dev()
    return tuple(torch.from_numpy(np.ascontiguousarray(d[k])).to(g) for k in ("v", "alpha", "cell_off"))


def _judged(w, cold):
    ok = np.isfinite(w["L_pen"]) & np.isfinite(cold["L_pen"])
    rel = np.full(len(cold["K"]), -np.inf)
    rel[ok] = (w["L_pen"][ok] - cold["L_pen"][ok]) / np.abs(cold["L_pen"][ok])
    rel[~np.isfinite(cold["L_pen"])] = 0.0
    return rel < -JUDGE_REL


def _work(w, cold):
    j = _judged(w, cold)
    return (w["visits"].sum() + cold["visits"][j].sum()) / cold["visits"].sum(), j.mean()


def test_trained_network_cuts_em_work_at_equal_mml():
    from paper_2007_12273_amd import api, warm
    train = [synth.weibel_3v(seed=5000 + i, n_cells=2048) for i in range(6)]
    feats, targs = warm.training_set(train, 16, seed=2003, device=dev())
    model = api.WarmStart(16, batch=1024, seed=7, device=dev())
    hist = warm.train(model, feats, targs, epochs=60, lr=1e-3, lam=1.0, seed=0)
    del feats, targs

    d = synth.weibel_3v(seed=6001, n_cells=2048)
    v, a, off = _gpu(d)
    n_cells = off.numel() - 1
    cold = host(api.compress(v, a, off, 16, seed=2003))
    reseed = host(api.compress(v, a, off, 16, seed=2003 + 7919))
    w = host(api.compress(v, a, off, 16, seed=2003, init=model.initial_mixtures(v, a, off)))
    fresh = api.WarmStart(16, batch=1024, seed=7, device=dev())
    init_u = fresh.initial_mixtures(v, a, off)
    wu = host(api.compress(v, a, off, 16, seed=2003, init=init_u))

    r_t, j_t = _work(w, cold)
    r_u, j_u = _work(wu, cold)
    r_r, j_r = _work(reseed, cold)
    print("training loss %.3f -> %.3f; EM work under the judged protocol relative to plain EM: trained %.3f "
          "(judged %.3f), untrained %.3f (judged %.3f, mean start K %.1f), reseeded cold %.3f (judged %.3f)"
          % (hist[0], hist[-1], r_t, j_t, r_u, j_u, init_u["K"].float().mean().item(), r_r, j_r))
    assert r_t < 0.85
    assert r_u > 1.0 and r_r > 1.0
    assert j_t < 0.7

    # the refit of the judged cells keeps each cell's index: a batch with
    # every other cell empty
    judged = np.nonzero(_judged(w, cold))[0]
    offh = d["cell_off"]
    counts = np.zeros(n_cells, np.int64)
    counts[judged] = np.diff(offh)[judged]
    so = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    idx = np.concatenate([np.arange(offh[c], offh[c + 1]) for c in judged])
    sub = {"v": d["v"][idx], "alpha": d["alpha"][idx], "cell_off": so}
    sv, sa, soff = _gpu(sub)
    refit = host(api.compress(sv, sa, soff, 16, seed=2003))
    for k in ("K", "L_pen", "L_final", "visits", "sweeps", "status", "omega", "mu", "sigma"):
        assert np.array_equal(refit[k][judged], cold[k][judged]), k

    # the protocol's output
    out = {k: w[k].copy() for k in ("K", "omega", "mu", "sigma", "moments", "L_pen")}
    for k in out:
        out[k][judged] = cold[k][judged]
    ok = np.isfinite(cold["L_pen"])
    assert (out["L_pen"][ok] >= cold["L_pen"][ok] - JUDGE_REL * np.abs(cold["L_pen"][ok])).all()
    assert np.array_equal(out["moments"], cold["moments"])
    _conserves(out)
    model.close()
    fresh.close()


def _conserves(g, D=3):
    K = g["K"]
    keep = K > 0
    mom = g["moments"][keep]
    W, P, S = mom[:, 0], mom[:, 1:1 + D], mom[:, 1 + D:]
    w, mu, sig = g["omega"][keep], g["mu"][keep], g["sigma"][keep]
    iu = np.triu_indices(D)
    Pm = W[:, None] * (w[:, :, None] * mu).sum(1)
    Sm = W[:, None] * (w[:, :, None] * (sig + mu[:, :, iu[0]] * mu[:, :, iu[1]])).sum(1)
    tr = S[:, [0, 3, 5]].sum(1)
    assert np.abs(w.sum(1) - 1.0).max() < 1e-12
    assert (np.abs(Pm - P).max(1) / np.sqrt(W * tr)).max() < 1e-12
    assert (np.abs(Sm - S).max(1) / tr).max() < 1e-12
