"""Host-side parts of bench.py (no GPU): the one-GPU contract and the
conservation check of reconstructed particles."""
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _cells(rng, counts, D):
    v = rng.normal(size=(counts.sum(), D))
    w = rng.uniform(0.5, 1.5, size=counts.sum())
    mom = np.zeros((len(counts), 1 + D + D * (D + 1) // 2))
    iu = np.triu_indices(D)
    o = 0
    for c, n in enumerate(counts):
        vc, wc = v[o:o + n], w[o:o + n]
        mom[c, 0] = wc.sum()
        mom[c, 1:1 + D] = (wc[:, None] * vc).sum(0)
        mom[c, 1 + D:] = np.einsum("p,pi,pj->ij", wc, vc, vc)[iu]
        o += n
    return v, w, mom


def test_conservation_check_finds_a_moment_error():
    import bench
    rng = np.random.default_rng(0)
    for D in (1, 3):
        counts = np.array([5, 40, 1, 17], dtype=np.int64)
        v, w, mom = _cells(rng, counts, D)
        status = torch.zeros(len(counts), dtype=torch.int32)
        rec = SimpleNamespace(v=torch.from_numpy(v.copy()), w=torch.from_numpy(w.copy()), status=status)
        r = bench.conservation(rec, mom, counts, D, torch)
        assert r["cells_checked"] == 4 and r["lemons_skipped"] == 0 and r["max_rel_err"] < 1e-13
        # a mass error of 1e-6 in cell 1 is found
        w2 = w.copy()
        w2[counts[0]] *= 1 + 1e-6 * w.sum() / w[counts[0]]
        rec.w = torch.from_numpy(w2)
        assert bench.conservation(rec, mom, counts, D, torch)["max_rel_err"] > 1e-7
        # ... unless the cell's projection was skipped (status LEMONS_SKIPPED)
        rec.status = torch.tensor([0, 128, 0, 0], dtype=torch.int32)
        r = bench.conservation(rec, mom, counts, D, torch)
        assert r["cells_checked"] == 3 and r["lemons_skipped"] == 1 and r["max_rel_err"] < 1e-13


def test_cpu_baseline_sample_is_clamped_to_the_batch():
    """A batch with fewer cells than the sample sizes is sampled whole,
    once per cell, and the line says so."""
    import bench
    rng = np.random.default_rng(3)
    counts = np.array([40, 60, 50])
    v = rng.normal(size=(counts.sum(), 3))
    data = {"v": v, "alpha": np.ones(counts.sum()), "cell_off": np.concatenate([[0], np.cumsum(counts)])}
    W = {"kmax": 4, "init_seed": 1, "D": 3, "dx": 1, "recon_seed": 2}
    r = bench.cpu_baseline(data, W, 256, 16)
    assert r["sample"].startswith("3 of 3 cells") and "%d particles" % counts.sum() in r["sample"]
    assert r["single_thread"]["sample"].startswith("3 evenly spaced cells, %d particles" % counts.sum())
