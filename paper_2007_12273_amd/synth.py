"""Seeded synthetic particle data shaped like the paper's PIC cells.

This module only draws inputs.  It holds none of the method's arithmetic
(no moments, no mixture fitting, no resampling), so it can feed both the
FP64 oracle and the HIP path without coupling them.

Workloads (data seed 1000+i for workload i unless given):

* ``two_stream_1v``  32 cells x 1000 equal-weight particles, two 1-D
  Maxwellian beams at drift +-0.2 with thermal speed 0.05 (500 each) --
  the shape of the paper's 1D-1V two-stream restart (Sec. 3.1).
* ``mix_1v``  1024 cells, counts max(200, Poisson(2000)), each cell 1-4
  Maxwellians (Dirichlet(1) fractions, drift U(-0.5,0.5), vth U(0.02,0.2)),
  weights U(0.5,1.5).
* ``weibel_3v``  4096 cells, counts LogNormal(ln 1000 - 0.125, 0.5) clipped
  to [50, 5000]; 1-6 anisotropic Gaussians per cell with T_perp = 4 T_par
  around a random unit axis b (Sigma = T_perp I + (T_par - T_perp) b b^T),
  equal weights -- the temperature-anisotropy shape of the paper's Weibel
  runs (Sec. 3.2).
* ``grid_3v``  256x256 cells, LogNormal counts (mean 256, sigma 0.5) clipped
  to [50, 5000] and rescaled by largest remainder to exactly 2^24
  particles; 1-4 isotropic 3-D Maxwellians per cell; weights U(0.5,1.5).
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    # name: (D, kmax, dx)
    "two_stream_1v": (1, 8, 1),
    "mix_1v": (1, 8, 1),
    "weibel_3v": (3, 16, 1),
    "grid_3v": (3, 8, 2),
}
WORKLOAD_INDEX = {"two_stream_1v": 1, "mix_1v": 2, "weibel_3v": 3, "grid_3v": 4}


def _offsets(counts):
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def _sample_cells(rng, counts, D, kmax_true_lo, kmax_true_hi, aniso, vth_lo=0.02, vth_hi=0.2):
    """Draw per-cell Gaussian mixtures and particles from them (vectorised)."""
    n_cells = len(counts)
    n_tot = int(np.sum(counts))
    ktrue = rng.integers(kmax_true_lo, kmax_true_hi + 1, size=n_cells)
    kk = int(kmax_true_hi)
    frac = rng.dirichlet(np.ones(kk), size=n_cells)
    mask = np.arange(kk)[None, :] < ktrue[:, None]
    frac = np.where(mask, frac, 0.0)
    frac /= frac.sum(axis=1, keepdims=True)
    drift = rng.uniform(-0.5, 0.5, size=(n_cells, kk, D))
    vth = rng.uniform(vth_lo, vth_hi, size=(n_cells, kk))
    if aniso and D == 3:
        b = rng.standard_normal(size=(n_cells, kk, 3))
        b /= np.linalg.norm(b, axis=2, keepdims=True)
        tpar = vth ** 2
        tperp = 4.0 * tpar
        cov = (tperp[..., None, None] * np.eye(3)[None, None]
               + (tpar - tperp)[..., None, None] * b[..., :, None] * b[..., None, :])
    else:
        cov = (vth ** 2)[..., None, None] * np.eye(D)[None, None]
    chol = np.linalg.cholesky(cov)
    cell_of = np.repeat(np.arange(n_cells), counts)
    cum = np.cumsum(frac, axis=1)
    cum[:, -1] = 1.0
    u = rng.random(n_tot)
    # per-particle inverse CDF over its cell's fractions (column by column,
    # without an n_tot x K temporary)
    comp = np.zeros(n_tot, dtype=np.int64)
    for k in range(kk):
        comp += u >= cum[cell_of, k]
    comp = np.minimum(comp, ktrue[cell_of] - 1)
    z = rng.standard_normal(size=(n_tot, D))
    flat = cell_of * kk + comp
    dr = drift.reshape(n_cells * kk, D)
    Lf = chol.reshape(n_cells * kk, D, D)
    v = np.empty((n_tot, D))
    for i in range(D):
        acc = dr[flat, i].copy()
        for j in range(i + 1):
            acc += Lf[flat, i, j] * z[:, j]
        v[:, i] = acc
    truth = {"K": ktrue, "omega": frac, "mu": drift, "sigma": cov, "label": comp}
    return v, truth


def two_stream_1v(seed=1001, n_cells=32, n_per_cell=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.full(n_cells, n_per_cell, dtype=np.int64)
    half = n_per_cell // 2
    v = np.empty((n_cells * n_per_cell, 1))
    label = np.empty(n_cells * n_per_cell, dtype=np.int64)
    for c in range(n_cells):
        s = c * n_per_cell
        v[s:s + half, 0] = 0.2 + 0.05 * rng.standard_normal(half)
        v[s + half:s + n_per_cell, 0] = -0.2 + 0.05 * rng.standard_normal(n_per_cell - half)
        label[s:s + half] = 0
        label[s + half:s + n_per_cell] = 1
    alpha = np.ones(n_cells * n_per_cell)
    truth = {"K": np.full(n_cells, 2), "label": label}
    return dict(v=v, alpha=alpha, cell_off=_offsets(counts), D=1, kmax=8, dx=1, truth=truth)


def mix_1v(seed=1002, n_cells=1024):
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.maximum(200, rng.poisson(2000, size=n_cells)).astype(np.int64)
    v, truth = _sample_cells(rng, counts, 1, 1, 4, aniso=False)
    alpha = rng.uniform(0.5, 1.5, size=len(v))
    return dict(v=v, alpha=alpha, cell_off=_offsets(counts), D=1, kmax=8, dx=1, truth=truth)


def lognormal_counts(rng, n_cells, mean, sigma=0.5, lo=50, hi=5000, total=None):
    mu_ln = np.log(mean) - 0.5 * sigma * sigma
    c = np.clip(rng.lognormal(mu_ln, sigma, size=n_cells), lo, hi)
    if total is None:
        return np.round(c).astype(np.int64)
    # largest-remainder rescale to an exact total, keeping the clip bounds
    x = c * (total / c.sum())
    base = np.floor(x).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(x - base), kind="stable")
    base[order[:rem]] += 1
    return base


def weibel_3v(seed=1003, n_cells=4096, mean=1000.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = lognormal_counts(rng, n_cells, mean)
    v, truth = _sample_cells(rng, counts, 3, 1, 6, aniso=True)
    alpha = np.ones(len(v))
    # cell-local positions on the 1D mesh (drawn last: earlier draws unchanged)
    x = rng.random((len(v), 1))
    return dict(v=v, alpha=alpha, x=x, cell_off=_offsets(counts), D=3, kmax=16, dx=1, nx=n_cells, truth=truth)


def grid_3v(seed=1004, n_cells=65536, total=1 << 24):
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = lognormal_counts(rng, n_cells, 256.0, total=total if n_cells == 65536 else None)
    v, truth = _sample_cells(rng, counts, 3, 1, 4, aniso=False)
    alpha = rng.uniform(0.5, 1.5, size=len(v))
    # cell-local positions on the 2D mesh, x fastest (drawn last)
    x = rng.random((len(v), 2))
    nx = int(round(np.sqrt(n_cells)))
    if nx * nx != n_cells:
        nx = n_cells
    return dict(v=v, alpha=alpha, x=x, cell_off=_offsets(counts), D=3, kmax=8, dx=2, nx=nx, truth=truth)


def make(name, seed=None, **kw):
    fn = {"two_stream_1v": two_stream_1v, "mix_1v": mix_1v,
          "weibel_3v": weibel_3v, "grid_3v": grid_3v}[name]
    if seed is None:
        seed = 1000 + WORKLOAD_INDEX[name]
    return fn(seed=seed, **kw)


def random_cells(seed, n_cells, D, n_lo, n_hi, k_lo=1, k_hi=4, weights="uniform", aniso=True):
    """Small ragged batches for parity tests: counts U{n_lo..n_hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.integers(n_lo, n_hi + 1, size=n_cells).astype(np.int64)
    v, truth = _sample_cells(rng, counts, D, k_lo, k_hi, aniso=aniso)
    if weights == "uniform":
        alpha = rng.uniform(0.5, 1.5, size=len(v))
    else:
        alpha = np.ones(len(v))
    return dict(v=v, alpha=alpha, cell_off=_offsets(counts), D=D, truth=truth)


def concat_cells(parts):
    """Join several {v, alpha, cell_off} batches into one."""
    vs, al, counts = [], [], []
    for p in parts:
        vs.append(p["v"])
        al.append(p["alpha"])
        counts.append(np.diff(p["cell_off"]))
    counts = np.concatenate(counts)
    return dict(v=np.concatenate(vs), alpha=np.concatenate(al), cell_off=_offsets(counts))


def split_start_cells(seed, n_cells=8, n=1000, kmax=16, shift=0.8):
    """Single isotropic Gaussian 3V cells and a deliberately poor
    two-component starting mixture per cell that has the generating mean and
    covariance: components at the generating mean +- shift * vth along x,
    covariance vth^2 diag(1 - shift^2, 1, 1), weights 1/2.
    Returns (data, init) with init in the gm_init layout (kmax slots)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.full(n_cells, n, dtype=np.int64)
    v, truth = _sample_cells(rng, counts, 3, 1, 1, aniso=False)
    alpha = np.ones(len(v))
    K = np.full(n_cells, 2, np.int32)
    w = np.zeros((n_cells, kmax))
    mu = np.zeros((n_cells, kmax, 3))
    S = np.zeros((n_cells, kmax, 6))
    for c in range(n_cells):
        m0 = truth["mu"][c, 0]
        t = truth["sigma"][c, 0][0, 0]
        for k, sgn in enumerate((-1.0, 1.0)):
            w[c, k] = 0.5
            mu[c, k] = m0
            mu[c, k, 0] += sgn * shift * np.sqrt(t)
            S[c, k] = [t * (1.0 - shift * shift), 0.0, 0.0, t, 0.0, t]
    data = dict(v=v, alpha=alpha, cell_off=_offsets(counts), D=3, truth=truth)
    return data, {"K": K, "omega": w, "mu": mu, "sigma": S}
