"""GPU reconstruct (gm_reconstruct through the C ABI) against the FP64 oracle
on the same mixtures: every particle to 1e-12 (the same Philox streams,
categorical draws and Box-Muller normals), statuses exactly, and the
projected sample's W, P, E equal to the targets to 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

from gpu_util import dev, host, torch

pytestmark = pytest.mark.gpu


def _gpu_recon(mix, moments, out_off, D, dx, seed):
    from paper_2007_12273_amd import api
    g = dev()
    t = lambda x, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(x)).to(g).to(dt)
    r = api.reconstruct(t(mix["K"], torch.int32), t(mix["omega"]), t(mix["mu"]), t(mix["sigma"]),
                        t(out_off, torch.int64), t(moments), D, dx, seed)
    torch.cuda.synchronize()
    return host(r)


@pytest.mark.parametrize("name,nc,dx,factor", [("weibel_3v", 40, 1, 1.0), ("grid_3v", 300, 2, 1.0),
                                               ("mix_1v", 40, 1, 0.5), ("weibel_3v", 12, 3, 3.0)])
def test_reconstruct_matches_oracle(name, nc, dx, factor):
    d = synth.make(name) if name != "grid_3v" else synth.make(name, n_cells=1024)
    off = d["cell_off"]
    D, kmax = d["D"], d["kmax"]
    sub = dict(v=d["v"][:off[nc]], alpha=d["alpha"][:off[nc]], cell_off=off[:nc + 1])
    mix = oracle.compress(sub["v"], sub["alpha"], sub["cell_off"], kmax=kmax, seed=1, max_sweeps=25)
    counts = np.maximum(0, np.round(np.diff(sub["cell_off"]) * factor)).astype(np.int64)
    counts[0] = 1  # a cell where the projection has no solution
    out_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    tg = oracle.targets_from_moments(mix["moments"], D)
    o = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], out_off, tg, D, dx, seed=3003)
    g = _gpu_recon(mix, mix["moments"], out_off, D, dx, 3003)
    assert np.array_equal(g["status"], o["status"])
    assert o["status"][0] == oracle.STATUS["LEMONS_SKIPPED"]
    np.testing.assert_allclose(g["w"], o["w"], rtol=1e-15, atol=0)
    if dx:
        assert np.array_equal(g["x"], o["x"])  # positions are raw uniforms
    scale = np.sqrt(np.maximum(tg[:, 1 + D] / tg[:, 0], 1e-300))  # thermal-plus-drift speed per cell
    cell_of = np.repeat(np.arange(nc), counts)
    err = np.abs(g["v"] - o["v"]).max(axis=1) / scale[cell_of]
    assert err.max() < 1e-12, err.max()
    # conservation of the projected sample
    for c in range(1, nc):
        sl = slice(out_off[c], out_off[c + 1])
        if sl.stop == sl.start:
            continue
        w, v = g["w"][sl], g["v"][sl]
        assert abs(w.sum() - tg[c, 0]) <= 1e-13 * tg[c, 0]
        P = (w[:, None] * v).sum(0)
        E = 0.5 * (w * (v * v).sum(1)).sum()
        assert np.abs(P - tg[c, 1:1 + D]).max() <= 1e-12 * np.sqrt(2 * tg[c, 0] * tg[c, 1 + D])
        assert abs(E - tg[c, 1 + D]) <= 1e-12 * tg[c, 1 + D]


def test_reconstruct_large_cell_regenerates():
    """A cell above the register-resident size takes the two-pass path."""
    D = 3
    K = np.array([2], np.int32)
    w = np.array([[0.7, 0.3]])
    mu = np.array([[[0.1, 0.0, 0.0], [-0.2, 0.1, 0.0]]])
    S = np.array([[[0.01, 0.001, 0, 0.02, 0, 0.015], [0.004, 0, 0, 0.004, 0, 0.004]]])
    mom = np.array([[2.0, 0.05, 0.02, 0.0, 0.05, 0.0, 0.0, 0.04, 0.0, 0.035]])
    out_off = np.array([0, 5000], np.int64)
    tg = oracle.targets_from_moments(mom, D)
    o = oracle.reconstruct(K, w, mu, S, out_off, tg, D, 1, seed=9)
    g = _gpu_recon({"K": K, "omega": w, "mu": mu, "sigma": S}, mom, out_off, D, 1, 9)
    assert np.array_equal(g["status"], o["status"])
    assert np.abs(g["v"] - o["v"]).max() < 1e-12 * np.sqrt(tg[0, 1 + D] / tg[0, 0])


@pytest.mark.parametrize("name,nc,dx", [("weibel_3v", 40, 1), ("mix_1v", 40, 0)])
def test_tensor_reconstruct_matches_oracle(name, nc, dx):
    """The full-second-moment projection: every particle within 1e-12 of
    the oracle's, statuses equal (a one-particle cell is skipped), and the
    projected sample's W, P and whole S equal the record's."""
    from paper_2007_12273_amd import api
    d = synth.make(name)
    off = d["cell_off"]
    D, kmax = d["D"], d["kmax"]
    sub = dict(v=d["v"][:off[nc]], alpha=d["alpha"][:off[nc]], cell_off=off[:nc + 1])
    mix = oracle.compress(sub["v"], sub["alpha"], sub["cell_off"], kmax=kmax, seed=1, max_sweeps=25)
    counts = np.diff(sub["cell_off"]).copy()
    counts[0] = 1
    counts[1] = 3000  # more particles than the registers hold: regenerated in the second pass
    out_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    o = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], out_off, mix["moments"], D, dx,
                                  seed=4004)
    g = dev()
    t = lambda x, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(x)).to(g).to(dt)
    r = host(api.reconstruct(t(mix["K"], torch.int32), t(mix["omega"]), t(mix["mu"]), t(mix["sigma"]),
                             t(out_off, torch.int64), t(mix["moments"]), D, dx, 4004, projection="tensor"))
    assert np.array_equal(r["status"], o["status"])
    assert o["status"][0] == oracle.STATUS["LEMONS_SKIPPED"] and (o["status"][1:] == 0).all()
    tg = oracle.targets_from_moments(mix["moments"], D)
    scale = np.sqrt(np.maximum(tg[:, 1 + D] / tg[:, 0], 1e-300))
    cell_of = np.repeat(np.arange(nc), counts)
    err = np.abs(r["v"] - o["v"]).max(axis=1) / scale[cell_of]
    assert err.max() < 1e-12, err.max()
    iu = np.triu_indices(D)
    for c in range(1, nc):
        sl = slice(out_off[c], out_off[c + 1])
        w, v = r["w"][sl], r["v"][sl]
        m = mix["moments"][c]
        S = m[1 + D:]
        assert abs(w.sum() - m[0]) <= 1e-13 * m[0]
        assert np.abs((w[:, None] * v).sum(0) - m[1:1 + D]).max() <= 1e-12 * np.sqrt(m[0] * np.abs(S).max())
        Sv = (w[:, None, None] * v[:, :, None] * v[:, None, :]).sum(0)[iu]
        assert np.abs(Sv - S).max() <= 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("projection", ["scalar", "tensor"])
def test_reconstruct_cell_sizes_around_the_wave_limit(projection):
    """Cells drawn by one wave (at most 512 particles) and by the whole
    workgroup (more) side by side in the same group of four cells, empty
    cells among them, and a cell count that is not a multiple of four:
    every particle within 1e-12 of the oracle's, statuses equal, and the
    projected sample's moments equal to the record's."""
    from paper_2007_12273_amd import api
    D, dx = 3, 2
    counts = np.array([0, 1, 64, 65, 511, 512, 513, 2048, 2049, 0, 5000, 7, 300], np.int64)
    nc = len(counts)
    d = synth.make("weibel_3v")
    off = d["cell_off"]
    sub = dict(v=d["v"][:off[nc]], alpha=d["alpha"][:off[nc]], cell_off=off[:nc + 1])
    mix = oracle.compress(sub["v"], sub["alpha"], sub["cell_off"], kmax=16, seed=1, max_sweeps=25)
    out_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    if projection == "tensor":
        o = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], out_off, mix["moments"], D,
                                      dx, seed=5005)
    else:
        o = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], out_off,
                               oracle.targets_from_moments(mix["moments"], D), D, dx, seed=5005)
    g = dev()
    t = lambda x, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(x)).to(g).to(dt)
    r = host(api.reconstruct(t(mix["K"], torch.int32), t(mix["omega"]), t(mix["mu"]), t(mix["sigma"]),
                             t(out_off, torch.int64), t(mix["moments"]), D, dx, 5005, projection=projection))
    assert np.array_equal(r["status"], o["status"])
    assert np.array_equal(r["x"], o["x"])
    np.testing.assert_allclose(r["w"], o["w"], rtol=1e-15, atol=0)
    tg = oracle.targets_from_moments(mix["moments"], D)
    scale = np.sqrt(np.maximum(tg[:, 1 + D] / tg[:, 0], 1e-300))
    cell_of = np.repeat(np.arange(nc), counts)
    err = np.abs(r["v"] - o["v"]).max(axis=1) / scale[cell_of]
    assert err.max() < 1e-12, err.max()
    for c in range(nc):
        if counts[c] < 2:
            continue
        sl = slice(out_off[c], out_off[c + 1])
        w, v = r["w"][sl], r["v"][sl]
        m = mix["moments"][c]
        assert abs(w.sum() - m[0]) <= 1e-13 * m[0]
        assert np.abs((w[:, None] * v).sum(0) - m[1:1 + D]).max() <= 1e-12 * np.sqrt(m[0] * np.abs(m[1 + D:]).max())
