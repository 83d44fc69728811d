"""GPU Gauss'-law weight correction and projection of given particles
(gm_deposit, gm_gauss_correct, gm_project through the C ABI) against the
FP64 oracle (Sec. 2.4.1).

Bars: deposits 1e-13 of the largest |D_i| (FP64 sums in another order);
corrected weights 1e-11 of the largest weight (the oracle solves with a
sparse direct solver, the GPU with BiCGSTAB to a relative residual of
1e-13; the mass matrix's condition number is about 7 in 1D and 15 in 2D);
the corrected deposit equal to the target to 1e-12; projected velocities
1e-12 of the cell's velocity scale and statuses exactly; after the whole
restart chain (sample, correct, project) the deposit, momentum and second
moment of every cell equal the recorded ones to 1e-12.
"""
import numpy as np
import pytest

import oracle
from oracle import gauss
from paper_2007_12273_amd import synth

from gpu_util import deposit_at, dev, torch

pytestmark = pytest.mark.gpu

SKIPPED = oracle.STATUS["LEMONS_SKIPPED"]


def _t(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev()).to(dt)


def _layout(dx, seed, counts):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    x = rng.random((off[-1], dx))
    w = rng.uniform(0.5, 1.5, size=off[-1])
    return x, w, off


def _counts(seed, n_cells, lo, hi):
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n_cells)


MESHES = [(1, 300, 300), (2, 480, 24), (1, 1, 1), (1, 2, 2), (2, 3, 1), (2, 4, 2), (2, 6, 3)]


@pytest.mark.parametrize("dx,n_cells,nx", MESHES)
def test_deposit_matches_oracle(dx, n_cells, nx):
    from paper_2007_12273_amd import api
    counts = _counts(1, n_cells, 1, 80)
    x, w, off = _layout(dx, 2, counts)
    gl = api.GaussLaw(n_cells, dx, nx, device=dev())
    g = gl.deposit(_t(x), _t(w), _t(off, torch.int64)).cpu().numpy()
    o = gauss.deposit(x, w, off, dx, nx)
    assert np.abs(g - o).max() <= 1e-13 * np.abs(o).max()
    assert abs(g.sum() - w.sum()) <= 1e-12 * w.sum()


@pytest.mark.parametrize("dx,n_cells,nx", MESHES)
def test_correction_matches_oracle(dx, n_cells, nx):
    """Original particles fix the target; a resampled set (as many particles
    per cell, new positions, equal weights carrying each cell's mass) is
    corrected on both sides."""
    from paper_2007_12273_amd import api
    counts = _counts(3, n_cells, 1, 60)
    x0, w0, off = _layout(dx, 4, counts)
    target = gauss.deposit(x0, w0, off, dx, nx)
    x1 = np.random.default_rng(5).random((off[-1], dx))
    W = np.add.reduceat(w0, off[:-1])
    w1 = np.repeat(W / counts, counts)
    dA, wo = gauss.gauss_correct(x1, w1, off, target, dx, nx)
    gl = api.GaussLaw(n_cells, dx, nx, device=dev())
    wg = _t(w1)
    it, res = gl.correct(_t(x1), wg, _t(off, torch.int64), _t(target), tol=1e-13)
    wg = wg.cpu().numpy()
    print("mesh dx=%d %d cells: %d iterations, residual %.1e, |dA| max %.2e" % (dx, n_cells, it, res,
                                                                                 np.abs(dA).max()))
    assert res <= 1e-13
    assert np.abs(wg - wo).max() <= 1e-11 * np.abs(wo).max()
    after = deposit_at(x1, wg, off, dx, nx, range(n_cells))
    assert np.abs(after - target).max() <= 1e-12 * np.abs(target).max()
    # one correction per cell: w' - w is constant within every cell
    dg = wg - w1
    for c in range(n_cells):
        sl = slice(off[c], off[c + 1])
        assert np.ptp(dg[sl]) <= 1e-15 * np.abs(wo).max()


def test_correction_rejects_an_empty_cell_and_reports_a_stalled_solve():
    from paper_2007_12273_amd import api
    counts = _counts(6, 64, 1, 30)
    counts[17] = 0
    x, w, off = _layout(2, 7, counts)
    target = np.ones(64)
    gl = api.GaussLaw(64, 2, 8, device=dev())
    wg = _t(w)
    with pytest.raises(RuntimeError, match="invalid argument"):
        gl.correct(_t(x), wg, _t(off, torch.int64), _t(target))
    assert np.array_equal(wg.cpu().numpy(), w)  # weights untouched
    counts[17] = 5
    x, w, off = _layout(2, 7, counts)
    with pytest.raises(RuntimeError, match="did not reach"):
        gl.correct(_t(x), _t(w), _t(off, torch.int64), _t(target), max_iter=1)


def _project_case(D, seed):
    """Cells of weighted particles (weights not all equal, as after the
    correction) and moments records of other particle sets; an empty cell,
    a one-particle cell and a cell of D particles (the tensor projection
    needs more than D)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(D + 2, 700, size=40)
    counts[3], counts[7], counts[11] = 0, 1, D
    counts[5] = 3000  # above the register-resident size: two passes
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = off[-1]
    v = rng.normal(size=(n, D)) * rng.uniform(0.05, 0.3, size=(n, 1)) + rng.uniform(-0.3, 0.3, size=(n, D))
    w = rng.uniform(0.8, 1.2, size=n)
    iu = np.triu_indices(D)
    mom = np.zeros((40, 1 + D + D * (D + 1) // 2))
    for c in range(40):
        m = 50 + c
        u = rng.normal(size=(m, D)) * 0.2 + rng.uniform(-0.2, 0.2, size=D)
        a = rng.uniform(0.5, 1.5, size=m)
        # a target mass within 1% of the cell's own (as after the correction)
        a *= max(w[off[c]:off[c + 1]].sum(), 1.0) * (1 + 0.01 * rng.uniform(-1, 1)) / a.sum()
        mom[c, 0] = a.sum()
        mom[c, 1:1 + D] = (a[:, None] * u).sum(0)
        mom[c, 1 + D:] = (a[:, None, None] * u[:, :, None] * u[:, None, :]).sum(0)[iu]
    return v, w, off, mom


@pytest.mark.parametrize("D,tensor", [(1, False), (1, True), (3, False), (3, True)])
def test_project_matches_oracle(D, tensor):
    from paper_2007_12273_amd import api
    v, w, off, mom = _project_case(D, 20 + D + 2 * tensor)
    vo, so = oracle.project(v, w, off, mom, D, tensor=tensor)
    vg_in = _t(v)
    vg, sg = api.project(vg_in, _t(w), _t(off, torch.int64), _t(mom), tensor=tensor)
    vg, sg = vg.cpu().numpy(), sg.cpu().numpy()
    assert np.array_equal(sg, so)
    assert so[3] == 0 and so[7] == SKIPPED
    if D == 3:  # D particles: the centred S' is singular, E' is not
        assert (so[11] == SKIPPED) == tensor
    others = np.setdiff1d(np.arange(40), [3, 7, 11])
    assert (so[others] == 0).all()
    scale = np.sqrt(np.repeat(mom[:, 1 + D] / mom[:, 0], np.diff(off)))
    assert (np.abs(vg - vo).max(1) / scale).max() < 1e-12
    # in place: the same result
    vi, si = api.project(vg_in, _t(w), _t(off, torch.int64), _t(mom), tensor=tensor, out=vg_in)
    assert np.array_equal(vi.cpu().numpy(), vg) and np.array_equal(si.cpu().numpy(), sg)


@pytest.mark.parametrize("name,n_cells,tensor", [("weibel_3v", 48, True), ("grid_3v", 256, True),
                                                 ("grid_3v", 256, False)])
def test_restart_chain_matches_oracle_and_conserves(name, n_cells, tensor):
    """Compress (oracle) -> deposit of the original particles -> sample with
    the projection -> Gauss'-law correction -> projection with the corrected
    mass, on the GPU and in the oracle.  The projection has no solution in a
    cell whose corrected mass cannot carry the recorded momentum with the
    recorded energy (Sec. 2.4.2 names this failure mode; the cell is left as
    sampled): cold drifting beams of the 2D grid workload meet it where the
    correction is large, so statuses must agree and the moments are checked
    where the projection ran."""
    from paper_2007_12273_amd import api
    d = synth.make(name, n_cells=n_cells)
    off, D, dx, nx = d["cell_off"], d["D"], d["dx"], d["nx"]
    mix = oracle.compress(d["v"], d["alpha"], off, kmax=d["kmax"], seed=2, max_sweeps=30)
    target = gauss.deposit(d["x"], d["alpha"], off, dx, nx)
    # oracle chain
    if tensor:
        ro = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off, mix["moments"], D, dx,
                                       seed=41)
    else:
        ro = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off,
                                oracle.targets_from_moments(mix["moments"], D), D, dx, seed=41)
    _, wo = gauss.gauss_correct(ro["x"], ro["w"], off, target, dx, nx)
    vo, so = oracle.project(ro["v"], wo, off, mix["moments"], D, tensor=tensor)
    # GPU chain
    offg = _t(off, torch.int64)
    gl = api.GaussLaw(n_cells, dx, nx, device=dev())
    tg = gl.deposit(_t(d["x"]), _t(d["alpha"]), offg)
    rec = api.Reconstructor(offg, D, dx, device=dev(), projection="tensor" if tensor else "scalar")
    r = rec(_t(mix["K"], torch.int32), _t(mix["omega"]), _t(mix["mu"]), _t(mix["sigma"]), _t(mix["moments"]), 41)
    it, res = gl.correct(r["x"], r["w"], offg, tg, tol=1e-13)
    vg, sg = api.project(r["v"], r["w"], offg, _t(mix["moments"]), tensor=tensor, out=r["v"])
    torch.cuda.synchronize()
    tgh, xg, wg, vg, sg = (t.cpu().numpy() for t in (tg, r["x"], r["w"], vg, sg))
    ok = so == 0
    print("%s (%s projection): %d iterations, residual %.1e; projection ran in %d / %d cells"
          % (name, "tensor" if tensor else "scalar", it, res, ok.sum(), n_cells))
    assert np.abs(tgh - target).max() <= 1e-13 * np.abs(target).max()
    assert np.array_equal(xg, ro["x"])
    assert np.abs(wg - wo).max() <= 1e-11 * np.abs(wo).max()
    assert np.array_equal(sg, so) and ok.mean() >= (1.0 if name == "weibel_3v" else 0.75)
    assert ((so == 0) | (so == SKIPPED)).all()
    mom = mix["moments"]
    tr = mom[:, 1 + D] + mom[:, 1 + D + 3] + mom[:, -1]
    scale = np.sqrt(np.repeat(tr / mom[:, 0], np.diff(off)))
    assert (np.abs(vg - vo).max(1) / scale).max() < 1e-10
    # conservation of the whole chain
    after = deposit_at(xg, wg, off, dx, nx, range(n_cells))
    assert np.abs(after - target).max() <= 1e-12 * np.abs(target).max()
    iu = np.triu_indices(D)
    P = np.add.reduceat(wg[:, None] * vg, off[:-1], axis=0)
    S = np.add.reduceat((wg[:, None, None] * vg[:, :, None] * vg[:, None, :])[:, iu[0], iu[1]], off[:-1], axis=0)
    assert (np.abs(P - mom[:, 1:1 + D]).max(1)[ok] / np.sqrt(mom[ok, 0] * tr[ok])).max() < 1e-12
    if tensor:
        assert (np.abs(S - mom[:, 1 + D:]).max(1)[ok] / tr[ok]).max() < 1e-12
    else:
        trS = S[:, 0] + S[:, 3] + S[:, 5]
        assert (np.abs(trS - tr)[ok] / tr[ok]).max() < 1e-12
