#!/usr/bin/env python3
"""Throughput of batched Gaussian-mixture checkpoint-restart on one MI355X.

One step = the whole hot path over one batch of cells with the inputs
resident in HBM: gm_compress (FP64 moments, FP32 adaptive EM sweeps to
convergence, FP64 unpenalised finish) followed by gm_reconstruct (ancestral
sampling of n' = n particles per cell plus the FP64 moment-matching
projection).  The metric is particles fit per second (sum of cell sizes per
step / step time).

Prints one JSON line.  Besides the throughput it reports the roofline of
the dominant kernel (the EM sweeps, bound by FP32 vector ALU) from HIP
events recorded around those launches, and the FP64 CPU oracle timed on a
bounded sample of the same cells.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles fit/s, batched GM-EM 1D3V: learned warm-start vs plain EM"

WORKLOADS = {
    "weibel_3v": dict(
        D=3, kmax=16, dx=1, init_seed=2003, recon_seed=3003,
        desc="1D3V Weibel-like: 4096 cells, log-normal counts (median ~880, sigma 0.5, clipped 50..5000, "
             "~4.1M particles), 1-6 anisotropic Gaussians per cell (T_perp = 4 T_par), equal weights, kmax 16; "
             "compress to convergence (tol 1e-7, <= 1000 sweeps) + reconstruct n' = n, dx = 1"),
    "grid_3v": dict(
        D=3, kmax=8, dx=2, init_seed=2004, recon_seed=3004,
        desc="2D3V grid: 65536 cells, log-normal counts mean 256 (2^24 particles), 1-4 isotropic Maxwellians, "
             "weights U(0.5,1.5), kmax 8; compress + reconstruct n' = n, dx = 2"),
    "mix_1v": dict(
        D=1, kmax=8, dx=1, init_seed=2002, recon_seed=3002,
        desc="1D1V: 1024 cells, counts max(200, Poisson(2000)), 1-4 Maxwellians, weights U(0.5,1.5), kmax 8"),
}

PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed), published
PEAK_HBM_GBPS = 8000.0
# algorithmic flops per (particle, component update), transcendentals as 1:
# density 19 + exp 1 + denominator 5 + responsibility 2 + moment sums 22 in 3V
FLOPS_PER_UPDATE = {3: 49, 1: 18}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="weibel_3v", choices=sorted(WORKLOADS))
    p.add_argument("--cpu-cells", type=int, default=32, help="cells in the CPU-oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    return p.parse_args()


def cpu_baseline(data, W, n_cells_sample):
    """The FP64 oracle on an evenly spaced sample of the same cells, all host
    threads (capped at 16)."""
    import numpy as np

    import oracle

    off = data["cell_off"]
    n_cells = len(off) - 1
    idx = np.linspace(0, n_cells - 1, n_cells_sample).astype(np.int64)
    vs, al, counts = [], [], []
    for c in idx:
        vs.append(data["v"][off[c]:off[c + 1]])
        al.append(data["alpha"][off[c]:off[c + 1]])
        counts.append(off[c + 1] - off[c])
    v = np.concatenate(vs)
    a = np.concatenate(al)
    so = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    threads = oracle.default_threads()
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.compress(v, a, so, kmax=W["kmax"], seed=W["init_seed"], nthreads=threads)
    tg = oracle.targets_from_moments(r["moments"], W["D"])
    oracle.reconstruct(r["K"], r["omega"], r["mu"], r["sigma"], so, tg, W["D"], W["dx"], seed=W["recon_seed"],
                       nthreads=threads)
    dt = time.perf_counter() - t0
    npart = int(so[-1])
    return {"value": npart / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d cells (evenly spaced), %d particles, compress to convergence + reconstruct, "
                      "%.1f s wall" % (n_cells_sample, n_cells, npart, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (cells are independent; "
              "see the sharding note in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2007_12273_amd import api, synth

    W = WORKLOADS[args.workload]
    data = synth.make(args.workload)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(data["v"]).to(dev)
    alpha = torch.from_numpy(data["alpha"]).to(dev)
    off = torch.from_numpy(data["cell_off"]).to(dev)
    n_cells = off.numel() - 1
    n_part = int(data["cell_off"][-1])
    D, kmax, dx = W["D"], W["kmax"], W["dx"]

    comp = api.Compressor(n_cells, D, kmax, device=dev, seed=W["init_seed"])
    recon = api.Reconstructor(off, D, dx, device=dev)

    def step():
        r = comp(v, alpha, off)
        recon(r.K, r.omega, r.mu, r.sigma, r.moments, W["recon_seed"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    print("timed %d steps: %.3f ms/step" % (args.steps, ms), file=sys.stderr, flush=True)

    # phase durations from HIP events recorded by the library on this stream
    api.profile_enable(True)
    phases = {"plan": [], "em": [], "finish": [], "reconstruct": []}
    for _ in range(max(2, min(args.steps, 5))):
        step()
        ph = api.profile_read()
        for k in phases:
            phases[k].append(ph[k])
    api.profile_enable(False)
    ph = {k: float(np.mean(x)) for k, x in phases.items()}

    K = comp.out.K.cpu().numpy()
    visits = comp.out.visits.cpu().numpy()
    sweeps = comp.out.sweeps.cpu().numpy()
    status = comp.out.status.cpu().numpy()
    counts = np.diff(data["cell_off"])
    em_flops = float((counts * visits).sum()) * FLOPS_PER_UPDATE[D]
    achieved = em_flops / (ph["em"] * 1e-3) / 1e12
    recon_bytes = n_part * 8 * (D + 1 + dx)
    line = {
        "metric": METRIC,
        "value": n_part / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload + ": " + W["desc"],
            "cells": n_cells, "particles": n_part, "kmax": kmax, "D": D, "start": "cold",
            "precision": "EM sweeps f32; moments, finish, reconstruct f64",
        },
        "roofline": {
            "kernel": "k_em (all length buckets)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None,
            "flops_per_launch": em_flops,
            "ms_per_launch": ph["em"],
        },
        "cells_per_s": n_cells / (ms * 1e-3),
        "phase_ms": ph,
        "reconstruct_hbm_gbps": recon_bytes / (ph["reconstruct"] * 1e-3) / 1e9,
        "mean_K": float(K.mean()),
        "mean_sweeps": float(sweeps.mean()),
        "maxsweeps_cells": int(((status & 8) != 0).sum()),
        # the paper's ratio: particles per Gaussian component
        "compression_ratio": float(counts.sum() / max(1, K.sum())),
    }
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(data, W, args.cpu_cells)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
