"""The whole step captured in a HIP graph (through torch.cuda.graph on the
caller's stream; the library's length buckets fork onto its own streams
with events, which the capture follows): every replay, with eager work and
synchronisations in between, reproduces the eager results bit for bit."""
import numpy as np
import pytest

from paper_2007_12273_amd import synth

from gpu_util import dev, to_gpu, torch
from test_gpu_compress import _subset

pytestmark = pytest.mark.gpu


def _snapshot(mix, rec):
    out = {k: t.detach().cpu().numpy().copy() for k, t in mix.as_dict().items()}
    out.update({"rv": rec["v"].cpu().numpy().copy(), "rw": rec["w"].cpu().numpy().copy(),
                "rx": rec["x"].cpu().numpy().copy(), "rs": rec["status"].cpu().numpy().copy()})
    return out


def test_graph_replays_match_eager():
    from paper_2007_12273_amd import api
    from paper_2007_12273_amd import warm as warmlib
    d = _subset(synth.make("weibel_3v"), 256)
    v, a, off = to_gpu(d)
    n_cells = off.numel() - 1
    comp = api.Compressor(n_cells, 3, 16, device=dev(), seed=2003)
    recon = api.Reconstructor(off, 3, 1, device=dev())
    tr = _subset(synth.make("weibel_3v", seed=5001), 1024)
    feats, targs = warmlib.training_set([tr], 16, seed=2003, device=dev())
    model = api.WarmStart(16, batch=256, seed=7, device=dev())
    warmlib.train(model, feats, targs, epochs=3)
    bufs = model.init_buffers(n_cells)

    def step():
        init = model.initial_mixtures(v, a, off, bufs=bufs)
        r = comp(v, a, off, init=init)
        return r, recon(r.K, r.omega, r.mu, r.sigma, r.moments, 3003)

    r, rec = step()
    torch.cuda.synchronize()
    eager = _snapshot(r, rec)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        # scribble over the outputs eagerly, then replay
        comp.out.K.fill_(-1)
        comp.out.omega.fill_(np.nan)
        recon.v.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(comp.out, {"v": recon.v, "w": recon.w, "x": recon.x, "status": recon.status})
        for k in eager:
            assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
        step()  # eager work between replays
        torch.cuda.synchronize()
    model.close()


def test_graph_replays_match_eager_on_the_full_grid():
    """The 2D3V grid at full size (65536 cells, 2^24 particles, kmax 8, dx = 2):
    cold compress and reconstruct captured in one graph; replays equal the
    eager results bit for bit, and sampled cells of the replayed record
    match the oracle (FP32 bars of fp32_parity)."""
    from paper_2007_12273_amd import api
    import fp32_parity
    from test_gpu_fullsize import _sample_batch
    d = synth.make("grid_3v")
    v, a, off = to_gpu(d)
    n_cells = off.numel() - 1
    assert n_cells == 65536 and d["cell_off"][-1] == 1 << 24
    comp = api.Compressor(n_cells, 3, 8, device=dev(), seed=2004)
    recon = api.Reconstructor(off, 3, 2, device=dev())

    def step():
        r = comp(v, a, off)
        return r, recon(r.K, r.omega, r.mu, r.sigma, r.moments, 3004)

    r, rec = step()
    torch.cuda.synchronize()
    eager = _snapshot(r, rec)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(2):
        comp.out.K.fill_(-1)
        comp.out.sigma.fill_(np.nan)
        recon.v.fill_(np.nan)
        recon.x.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(comp.out, {"v": recon.v, "w": recon.w, "x": recon.x, "status": recon.status})
        for k in eager:
            assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
        del got
        step()
        torch.cuda.synchronize()
    rng = np.random.default_rng(53)
    cells = sorted(set(rng.choice(n_cells, 16, replace=False).tolist()) | {0, n_cells - 1})
    vs, al, so = _sample_batch(d, cells)
    fp32_parity.converged(eager, dict(v=vs, alpha=al, cell_off=so), 8, 2004, "grid graph replay", cells=cells)
    del g
