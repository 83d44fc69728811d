"""FP64 iterations (gm_opts.estep_fp64 = 1) against the FP64 oracle, with
the decisions of the method compared exactly.

With both sides iterating in FP64 the GPU path must take every decision the
oracle takes: the cold-start draws (Sec. 2.3), each annihilation (eq.
omegak: N_k - T/2 <= 0), and the stop test on the relative change of eq.
(lnL-GM).  So per cell the component count K, the sweep count, the number
of component updates (visits) and the status flags are identical, and the
mixture parameters and likelihoods differ only by rounding: parameters
within 1e-8 (|d omega|, |d mu| / sqrt(tr C / D), |d Sigma|_F / |Sigma|_F),
L_pen and L_final within 1e-10 relative, preserved moments and the
conservation of the output mixture within 1e-12.  NEAR_TIE cells (a
decision within 1e-5 T/2 of the threshold) would be exempt from the
decision checks; the batches below have none, and the test says so.

Batches cover every length bucket of both component-slot classes:
Weibel-like 1D3V cells (kmax 16) and 2D3V grid cells (kmax 8) picked by
size from the workload generators, plus cells of the same recipes drawn at
sizes the workloads rarely or never reach (11-200 and 4100-8192
particles, and above 8192, where the streaming launch takes over), in
converged mode and in replay of the oracle's sweep counts;
also the 1D1V mixed workload, supplied starting mixtures and the outer
search over K.
"""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

from gpu_util import conservation, dev, host, mixture_errors, take_cells, to_gpu, torch

pytestmark = pytest.mark.gpu

NEAR = oracle.STATUS["NEAR_TIE"]
MAX_SWEEPS = 200

# largest cell of each length bucket for 16 and 8 component slots
BUCKETS16 = [128, 256, 512, 768, 1024, 1280, 1536, 1792, 2048, 2560, 4096, 8192]
BUCKETS8 = [64, 128, 256, 512, 1024, 1536, 2048, 2560, 3072, 3584, 4096, 8192]


def _pick(d, bounds, per):
    """Up to `per` cells of each length bucket, the first ones in the batch."""
    n = np.diff(d["cell_off"])
    sel, lo = [], 0
    for hi in bounds:
        sel += list(np.nonzero((n > lo) & (n <= hi))[0][:per])
        lo = hi
    return np.array(sorted(sel))


def _covering_batch(d, bounds, extra_small, extra_big):
    part = take_cells(d, _pick(d, bounds, 2))
    b = synth.concat_cells([part, extra_small, extra_big])
    n = np.diff(b["cell_off"])
    lo = 0
    for hi in bounds:
        assert ((n > lo) & (n <= hi)).any(), ("bucket without a cell", lo, hi)
        lo = hi
    return b


def _gpu(d, kmax, **kw):
    from paper_2007_12273_amd import api
    v, a, off = to_gpu(d)
    fs = kw.pop("fixed_sweeps", None)
    if fs is not None:
        fs = torch.from_numpy(np.ascontiguousarray(fs, dtype=np.int32)).to(dev())
    init = kw.pop("init", None)
    if init is not None:
        init = {k: torch.from_numpy(np.ascontiguousarray(x)).to(dev()) for k, x in init.items()}
        init["K"] = init["K"].to(torch.int32)
    r = api.compress(v, a, off, kmax, fp64=True, fixed_sweeps=fs, init=init, **kw)
    torch.cuda.synchronize()
    return host(r)


def _exact(g, o, D, label):
    n_cells = len(o["K"])
    near = ((g["status"] | o["status"]) & NEAR).astype(bool)
    print("%s: %d cells, %d NEAR_TIE, K histogram %s, sweeps max %d" % (
        label, n_cells, near.sum(), np.bincount(o["K"]).tolist(), o["sweeps"].max()))
    keep = ~near
    for key in ("K", "sweeps", "visits", "status"):
        diff = np.nonzero(g[key][keep] != o[key][keep])[0]
        assert len(diff) == 0, (label, key, np.nonzero(keep)[0][diff], g[key][keep][diff], o[key][keep][diff])
    worst_p, worst_L = 0.0, 0.0
    for c in np.nonzero(keep)[0]:
        scale = np.abs(o["moments"][c]).max()
        assert np.abs(g["moments"][c] - o["moments"][c]).max() <= 1e-12 * scale, (label, c)
        if o["K"][c] == 0:
            continue
        dw, dp, ds = conservation(g, c, D)
        assert max(dw, dp, ds) < 1e-12, (label, c, dw, dp, ds)
        e = max(mixture_errors(g, o, c, D))
        eL = max(abs(g["L_pen"][c] - o["L_pen"][c]) / abs(o["L_pen"][c]),
                 abs(g["L_final"][c] - o["L_final"][c]) / abs(o["L_final"][c]))
        worst_p, worst_L = max(worst_p, e), max(worst_L, eL)
        assert e <= 1e-8, (label, c, e)
        assert eL <= 1e-10, (label, c, eL)
    print("%s: largest parameter difference %.1e, largest L difference %.1e" % (label, worst_p, worst_L))


def _both_modes(d, kmax, seed, label, **kw):
    D = 1 if d["v"].ndim == 1 else d["v"].shape[1]
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=MAX_SWEEPS, **kw)
    g = _gpu(d, kmax, seed=seed, max_sweeps=MAX_SWEEPS, **kw)
    _exact(g, o, D, label + ", converged")
    # replay of the converged run's sweep counts (the cap flag is not raised in replay)
    fs = np.maximum(o["sweeps"], 1)
    orp = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=kmax, seed=seed, max_sweeps=MAX_SWEEPS,
                          fixed_sweeps=fs, **kw)
    grp = _gpu(d, kmax, seed=seed, max_sweeps=MAX_SWEEPS, fixed_sweeps=fs, **kw)
    _exact(grp, orp, D, label + ", replay")
    return g, o


def test_weibel_3v_every_bucket_fp64_exact():
    small = synth.random_cells(301, 6, 3, 11, 200, k_lo=1, k_hi=3, weights="equal")
    big = synth.random_cells(302, 3, 3, 4100, 8192, k_lo=1, k_hi=3, weights="equal")
    d = _covering_batch(synth.make("weibel_3v"), BUCKETS16, small, big)
    _both_modes(d, 16, 2003, "Weibel-like kmax 16")


def _one_per_range(seed, D, ranges, **kw):
    return synth.concat_cells([synth.random_cells(seed + i, 1, D, lo, hi, **kw) for i, (lo, hi) in enumerate(ranges)])


def test_grid_3v_every_bucket_fp64_exact():
    small = synth.random_cells(303, 6, 3, 11, 200, k_lo=1, k_hi=4, aniso=False)
    big = _one_per_range(304, 3, [(1537, 2048), (2049, 2560), (2561, 3072), (3073, 3584), (3585, 4096), (4097, 8192)],
                         k_lo=1, k_hi=4, aniso=False)
    d = _covering_batch(synth.grid_3v(n_cells=8192), BUCKETS8, small, big)
    _both_modes(d, 8, 2004, "grid kmax 8")


def test_cells_larger_than_the_buckets_fp64_exact():
    """Cells of 8193 to 16384 particles (the streaming launch) among
    bucket-sized ones, 3V and 1V."""
    for D, kmax, seed in ((3, 16, 310), (3, 8, 320), (1, 8, 330)):
        d = _one_per_range(seed, D, [(8193, 9000), (9001, 16384), (300, 2000)], k_lo=1, k_hi=3, aniso=False)
        _both_modes(d, kmax, seed, "cells above 8192, D %d kmax %d" % (D, kmax))


def test_mix_1v_fp64_exact():
    small = synth.random_cells(305, 6, 1, 11, 400, k_lo=1, k_hi=4, aniso=False)
    d = synth.concat_cells([take_cells(synth.make("mix_1v"), np.arange(16)), small])
    _both_modes(d, 8, 2002, "1D1V mixed kmax 8")


def test_supplied_start_fp64_exact():
    """Starting mixtures supplied by the caller (the warm-start entry): the
    oracle's own fits after 30 sweeps from a cold start, continued."""
    d = take_cells(synth.make("weibel_3v"), np.arange(0, 64, 2))
    o0 = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=9, max_sweeps=30)
    init = {"K": o0["K"], "omega": o0["omega"], "mu": o0["mu"], "sigma": o0["sigma"]}
    _both_modes(d, 16, 9, "supplied start", init=init)


def test_outer_search_fp64_exact():
    d = take_cells(synth.make("weibel_3v"), np.arange(1, 48, 3))
    D = 3
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=4, max_sweeps=MAX_SWEEPS,
                        mode=oracle.MODE_OUTER_K)
    g = _gpu(d, 16, seed=4, max_sweeps=MAX_SWEEPS, outer_k=True)
    _exact(g, o, D, "outer search over K")
