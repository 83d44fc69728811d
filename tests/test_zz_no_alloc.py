"""gm_compress_noalloc (the entry point for callers that cannot allocate)
against gm_compress through the C ABI: two calls in a row on one GPU, the
second with a smaller batch, each compared field by field with gm_compress
on the same input (the same kernels and launch plan, so the records are
identical bit for bit), and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2007_12273_amd import synth

from gpu_util import dev, host, take_cells, to_gpu, torch

pytestmark = pytest.mark.gpu


def _both(d, D, kmax, seed):
    from paper_2007_12273_amd import api
    v, a, off = to_gpu(d)
    n_cells = len(d["cell_off"]) - 1
    ref = host(api.compress(v, a, off, kmax, seed=seed, max_sweeps=300))
    out = api.MixtureBuffers(n_cells, D, kmax, dev())
    for t in out.as_dict().values():
        t.fill_(7)  # every field must be written by the call
    api.compress_noalloc(v, a, off, out, api.make_opts(D, kmax, seed=seed, max_sweeps=300))
    torch.cuda.synchronize()
    got = host(out.as_dict())
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    return got


def test_noalloc_equals_compress_on_two_calls():
    big = take_cells(synth.make("weibel_3v"), np.arange(300))
    small = take_cells(synth.make("weibel_3v"), np.arange(1000, 1060))
    g1 = _both(big, 3, 16, 11)
    g2 = _both(small, 3, 16, 12)
    assert (g1["K"] > 0).all() and (g2["K"] > 0).all()
    # a 1V batch on the same scratch
    _both(take_cells(synth.make("mix_1v"), np.arange(40)), 1, 8, 13)


def test_noalloc_rejects_batches_above_its_limit():
    from paper_2007_12273_amd import _lib, api
    L = _lib.load()
    n_cells = _lib.GM_NOALLOC_MAX_CELLS + 1
    opts = api.make_opts(3, 8)
    off = torch.zeros(n_cells + 1, dtype=torch.int64, device=dev())
    v = torch.zeros(3, dtype=torch.float64, device=dev())
    a = torch.zeros(1, dtype=torch.float64, device=dev())
    out = api.MixtureBuffers(n_cells, 3, 8, dev())
    mix = out.struct()
    rc = L.gm_compress_noalloc(ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                               ctypes.c_void_p(off.data_ptr()), n_cells, ctypes.byref(opts), None, None,
                               ctypes.byref(mix), None)
    assert rc == _lib.GM_ETOOBIG
