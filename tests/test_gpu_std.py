"""Standard EM with K-means start and Anderson acceleration on the GPU
(gm_compress_standard through the C ABI) against the FP64 oracle.

* plain EM, a fixed number of EM steps (tol 0): parameters after the same
  steps to the FP32 bars of the adaptive path's replay mode (1e-4 in 90% of
  cells, never above 1e-2), moments 1e-12;
* K-means start: the FP64 Lloyd passes equal (same assignments), then two
  EM steps as above;
* Anderson-accelerated, converged mode: the reset and rejection decisions
  compare FP32 likelihoods, so trajectories can part; where both reach the
  same maximum (log-likelihood within 1e-5) the parameters agree to the
  converged-mode bars, in most cells; moments exact everywhere.
"""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

from gpu_util import dev, host, mixture_errors, to_gpu, torch
from test_gpu_compress import _subset

pytestmark = pytest.mark.gpu


def _gpu(d, K, kmeans, aa, max_sweeps, tol, seed, kmax=16):
    from paper_2007_12273_amd import api
    v, a, off = to_gpu(d)
    n_cells = len(d["cell_off"]) - 1
    s = api.StandardEM(n_cells, len(d["alpha"]), 3, kmax, device=dev(), seed=seed, max_sweeps=max_sweeps, tol=tol)
    out = s(v, a, off, K, kmeans=kmeans, aa_memory=aa)
    torch.cuda.synchronize()
    g = host(out.as_dict())
    g["resets"] = s.resets.cpu().numpy()
    g["kmeans_passes"] = s.kmeans_passes.cpu().numpy()
    return g


def _compare(g, o, cells, label, bar=1e-4, frac=0.9, worst=1e-2):
    errs = []
    for c in cells:
        if g["K"][c] != o["K"][c]:
            continue
        errs.append(max(mixture_errors(g, o, c, 3)))
    errs = np.array(errs)
    print("%s: %d cells, K equal in %d; parameter error median %.1e p90 %.1e max %.1e"
          % (label, len(cells), len(errs), np.median(errs), np.quantile(errs, 0.9), errs.max()))
    return errs


def _moments_exact(g, o):
    scale = np.abs(o["moments"]).max(1, keepdims=True)
    assert (np.abs(g["moments"] - o["moments"]) <= 1e-12 * scale).all()
    from gpu_util import conservation
    for c in range(len(g["K"])):
        if g["K"][c] > 0:
            assert max(conservation(g, c, 3)) < 1e-12


@pytest.mark.parametrize("kmeans", [False, True])
def test_fixed_steps_match_oracle(kmeans):
    d = _subset(synth.make("weibel_3v"), 40)
    steps = 2 if kmeans else 12
    o = oracle.compress_std(d["v"], d["alpha"], d["cell_off"], 6, seed=2003, kmax=16, kmeans=kmeans,
                            max_iter=steps, tol=0.0)
    g = _gpu(d, 6, kmeans, 0, steps, 0.0, 2003)
    if kmeans:
        np.testing.assert_array_equal(g["kmeans_passes"], o["kmeans_passes"])
    assert (g["sweeps"] == steps).all() and (o["iters"] == steps).all()
    assert (g["K"] == o["K"]).mean() >= 0.95
    errs = _compare(g, o, range(40), "standard EM, %d steps, %s start" % (steps, "K-means" if kmeans else "random"))
    assert (errs <= 1e-4).mean() >= 0.9 and errs.max() <= 1e-2
    _moments_exact(g, o)


def test_anderson_converged_matches_oracle():
    d = _subset(synth.make("weibel_3v"), 48)
    o = oracle.compress_std(d["v"], d["alpha"], d["cell_off"], 4, seed=2003, kmax=16, aa_m=5, max_iter=1000)
    g = _gpu(d, 4, False, 5, 1000, 1e-7, 2003)
    same = np.abs(g["L_pen"] - o["ll"]) <= 1e-5 * np.abs(o["ll"])
    print("Anderson, converged: same maximum in %d / 48 cells; iterations gpu median %d, oracle %d; resets gpu %d "
          "oracle %d" % (same.sum(), np.median(g["sweeps"]), np.median(o["iters"]), g["resets"].sum(),
                         o["resets"].sum()))
    assert same.mean() >= 0.8
    errs = _compare(g, o, list(np.nonzero(same)[0]), "Anderson same-maximum cells")
    assert np.median(errs) <= 2e-3 and (errs <= 3e-2).mean() >= 0.9
    _moments_exact(g, o)
