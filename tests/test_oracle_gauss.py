"""Pins of the oracle's Gauss'-law weight correction (Sec. 2.4.1):

* the quadratic B-spline's closed-form values and its partition of unity;
* the deposit conserves total charge (1D and 2D periodic meshes) and
  equals a per-mesh-cell brute-force sum written separately;
* every column of the mass matrix is the deposit's response to a unit
  weight change of the particles of that cell (brute force), and sums to the
  cell's particle count;
* after the correction the deposit equals the target to rounding;
* correction followed by the projection restores charge density, momentum
  and the second-moment tensor together (the projection uses the corrected
  mass N').
"""
import numpy as np
import pytest

import oracle
from oracle import gauss
from paper_2007_12273_amd import synth

from gpu_util import deposit_at


def test_s2_values_and_partition_of_unity():
    assert gauss.s2(0.0) == 0.75 and gauss.s2(0.5) == 0.5 and gauss.s2(1.0) == 0.125
    assert gauss.s2(1.5) == 0.0 and gauss.s2(-1.0) == 0.125 and gauss.s2(2.0) == 0.0
    s = np.linspace(-0.5, 0.5, 101)
    np.testing.assert_allclose(gauss.s2(s - 1) + gauss.s2(s) + gauss.s2(s + 1), 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dx,n_cells,nx", [(1, 17, 17), (2, 30, 6), (1, 2, 2), (2, 4, 2), (2, 3, 1)])
def test_deposit_equals_brute_force_per_cell(dx, n_cells, nx):
    """The vectorised deposit against a per-mesh-cell sum over the particles
    of the neighbouring cells, written separately (also on meshes narrower
    than the stencil, where a cell is its own neighbour)."""
    x, w, off = _layout(dx, 9, n_cells, 1, 20)
    D = gauss.deposit(x, w, off, dx, nx)
    np.testing.assert_allclose(D, deposit_at(x, w, off, dx, nx, range(n_cells)), rtol=0, atol=1e-13)


def _layout(dx, seed, n_cells, lo=5, hi=40):
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, size=n_cells)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    x = rng.random((off[-1], dx))
    w = rng.uniform(0.5, 1.5, size=off[-1])
    return x, w, off


@pytest.mark.parametrize("dx,n_cells,nx", [(1, 17, 17), (2, 30, 6)])
def test_deposit_and_mass_matrix(dx, n_cells, nx):
    x, w, off = _layout(dx, 3, n_cells)
    D = gauss.deposit(x, w, off, dx, nx)
    assert abs(D.sum() - w.sum()) <= 1e-12 * w.sum()
    M = gauss.mass_matrix(x, off, dx, nx).toarray()
    np.testing.assert_allclose(M.sum(0), np.diff(off), rtol=1e-13)
    cell_of = np.repeat(np.arange(n_cells), np.diff(off))
    for j in range(n_cells):
        dw = (cell_of == j).astype(float)
        col = gauss.deposit(x, w + dw, off, dx, nx) - D
        np.testing.assert_allclose(col, M[:, j], rtol=0, atol=1e-12)
    # each particle reaches its own cell and the 2 (1D) or 8 (2D) around it
    assert ((M > 0).sum(0) <= (3 if dx == 1 else 9)).all()


@pytest.mark.parametrize("dx,n_cells,nx", [(1, 64, 64), (2, 64, 8)])
def test_correction_restores_the_target_deposit(dx, n_cells, nx):
    x0, w0, off0 = _layout(dx, 5, n_cells, 20, 60)
    target = gauss.deposit(x0, w0, off0, dx, nx)
    # a resampled set: as many particles per cell, new positions, equal
    # weights carrying each cell's mass
    off1 = off0
    x1 = np.random.default_rng(6).random((off1[-1], dx))
    W = np.add.reduceat(w0, off0[:-1])
    w1 = np.repeat(W / np.diff(off1), np.diff(off1))
    dA, w2 = gauss.gauss_correct(x1, w1, off1, target, dx, nx)
    after = gauss.deposit(x1, w2, off1, dx, nx)
    assert np.abs(after - target).max() <= 1e-12 * np.abs(target).max()
    # total charge: sum_j n'_j dA_j = sum(target) - sum(deposit before)
    assert abs((dA * np.diff(off1)).sum() - (target.sum() - w1.sum())) <= 1e-10 * target.sum()
    # the correction is small next to the weights
    assert np.abs(dA).max() < 0.5 * w1.min()


def test_correction_then_projection_restores_density_momentum_and_tensor():
    d = synth.make("weibel_3v", n_cells=32)
    off = d["cell_off"]
    mix = oracle.compress(d["v"], d["alpha"], off, kmax=8, seed=2, max_sweeps=30)
    target = gauss.deposit(d["x"], d["alpha"], off, 1, 32)
    tg = oracle.targets_from_moments(mix["moments"], 3)
    r = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off, tg, 3, 1, seed=11)
    _, w2 = gauss.gauss_correct(r["x"], r["w"], off, target, 1, 32)
    v2, st = oracle.project(r["v"], w2, off, mix["moments"], 3, tensor=True)
    assert (st == 0).all()
    np.testing.assert_allclose(gauss.deposit(r["x"], w2, off, 1, 32), target, rtol=1e-12)
    iu = np.triu_indices(3)
    for c in range(32):
        sl = slice(off[c], off[c + 1])
        m = mix["moments"][c]
        P = (w2[sl, None] * v2[sl]).sum(0)
        S = (w2[sl, None, None] * v2[sl, :, None] * v2[sl, None, :]).sum(0)[iu]
        assert np.abs(P - m[1:4]).max() <= 1e-12 * np.sqrt(m[0] * np.abs(m[4:]).max())
        assert np.abs(S - m[4:]).max() <= 1e-12 * np.abs(m[4:]).max()
    # the corrected masses differ from the recorded W: the projection used N'
    Wc = np.add.reduceat(w2, off[:-1])
    assert np.abs(Wc - mix["moments"][:, 0]).max() > 1e-6 * mix["moments"][:, 0].max()
