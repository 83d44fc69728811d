"""GPU warm start (gm_warm_* through the C ABI) against the FP64 oracle.

Bars:
  * features: the oracle's FP64 features rounded to BF16, within one BF16
    ulp (FP64 sums in another order, 2^-40 fixed-point histogram weights),
    histogram bins also within a few particle weights (a whitened velocity
    on a bin edge can land either side); frames 1e-12 relative;
  * network products (BF16 operands, FP32 accumulation on matrix cores)
    against the oracle's BF16-emulating FP64 pass on the same BF16 inputs:
    1e-3 relative per tensor (outputs, every gradient, the loss);
  * decode and targets: FP64 on both sides, K exact, 1e-12 / FP32 rounding;
  * warm-started compress: the compress bars of the cold path, and the
    fallback decision exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

from gpu_util import dev, host, to_gpu, torch
import fp32_parity
from test_gpu_compress import _subset

pytestmark = pytest.mark.gpu

FALLBACK = oracle.STATUS["WARM_FALLBACK"]


def _api():
    from paper_2007_12273_amd import api
    return api


def _bf16_bits_to_f64(bits):
    b = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def _round_bf16(x):
    return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _oracle_feature_bits(d):
    """The oracle's features rounded to BF16: (GPU int16 tensor [n, 128] of
    bit patterns, the same values as FP64 [n, 105], the oracle's frames).
    Both sides of a network comparison start from these inputs."""
    of, ofr = oracle.features(d["v"], d["alpha"], d["cell_off"])
    b = torch.zeros(of.shape[0], 128, dtype=torch.int16)
    b[:, :105] = torch.from_numpy(of).to(torch.bfloat16).view(torch.int16)
    return b.to(dev()), _bf16_bits_to_f64(b[:, :105].numpy()), ofr


def _params(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(size=(105, 256)) * scale, "b1": rng.normal(size=256) * 0.05,
            "W2": rng.normal(size=(256, 256)) * scale * 0.5, "b2": rng.normal(size=256) * 0.05,
            "W3": rng.normal(size=(256, 160)) * scale * 0.5, "b3": rng.normal(size=160) * 0.05}


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def _edge_batch():
    """Weibel-like cells plus an empty cell, a cell of identical velocities
    (singular covariance) and a one-particle cell."""
    d = _subset(synth.make("weibel_3v"), 40)
    counts = list(np.diff(d["cell_off"]))
    v, a = [d["v"]], [d["alpha"]]
    counts.append(0)
    v.append(np.tile([[0.1, -0.2, 0.3]], (7, 1)))
    a.append(np.ones(7))
    counts.append(7)
    v.append(np.array([[0.5, 0.5, 0.5]]))
    a.append(np.ones(1))
    counts.append(1)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return dict(v=np.concatenate(v), alpha=np.concatenate(a), cell_off=off, D=3)


def test_features_match_oracle():
    d = _edge_batch()
    v, a, off = to_gpu(d)
    f, fr = _api().warm_features(v, a, off)
    torch.cuda.synchronize()
    g = _bf16_bits_to_f64(f.cpu().numpy())
    gfr = fr.cpu().numpy()
    of, ofr = oracle.features(d["v"], d["alpha"], d["cell_off"])
    n_cells = len(d["cell_off"]) - 1
    assert (g[:, 105:] == 0).all()
    np.testing.assert_allclose(gfr, ofr, rtol=1e-12, atol=1e-15)
    ob = _round_bf16(of)
    exact = (g[:, :105] == ob).mean()
    counts = np.diff(d["cell_off"])
    for c in range(n_cells):
        tol = 2.0 ** -7 * np.abs(of[c]) + 1e-30
        tol[:96] += 3.0 / max(counts[c], 1)
        assert (np.abs(g[c, :105] - of[c]) <= tol + np.abs(ob[c] - of[c])).all(), c
    print("features: %.4f of values bit-identical to the rounded oracle" % exact)
    assert exact >= 0.98
    # empty / singular / single-particle cells: zero features, zero factor
    for c in range(n_cells - 3, n_cells):
        assert (g[c] == 0).all() and (gfr[c, 3:] == 0).all()


def test_forward_matches_oracle_bf16():
    """Three MFMA products with fused bias and ReLU against the oracle's
    BF16-rounding forward pass, on 300 rows (ragged 32-row tiles)."""
    api = _api()
    d = _subset(synth.make("weibel_3v"), 300)
    f, X, _ = _oracle_feature_bits(d)
    P = _params(11)
    m = api.WarmStart(16, batch=64, seed=1)
    m.set_params(api.params_to_flat(P))
    Y = m.forward(f)
    torch.cuda.synchronize()
    _, _, Yo = oracle.mlp_forward(X, P, bf16=True)
    err = _rel(Y.cpu().numpy(), Yo)
    print("forward: relative error %.2e" % err)
    assert err < 1e-3
    m.close()


def test_model_file_round_trip(tmp_path):
    """gm_warm_save then gm_warm_load gives the same parameters bit for bit
    and the same network outputs; the loaded model trains on."""
    api = _api()
    d = _subset(synth.make("weibel_3v"), 200)
    f, _, _ = _oracle_feature_bits(d)
    m = api.WarmStart(16, batch=64, seed=1)
    m.set_params(api.params_to_flat(_params(23)))
    path = tmp_path / "model.gmw"
    m.save(path)
    assert path.stat().st_size == 8 + 4 + 4 + 8 + 4 * m.n_param
    m2 = api.WarmStart.load(path, batch=32)
    assert m2.kmax == 16
    np.testing.assert_array_equal(m2.get_params(), m.get_params())
    y1, y2 = m.forward(f), m2.forward(f)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    m.close()
    m2.close()


def _epoch_permutation(n, seed, epoch):
    """The documented shuffle of gm_warm_train, written out (splitmix64 draws,
    Fisher-Yates from the top index down)."""
    M = (1 << 64) - 1
    x = (seed ^ (0xD1B54A32D192ED03 * (epoch + 1))) & M
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        x = (x + 0x9E3779B97F4A7C15) & M
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z ^= z >> 31
        j = (z * (i + 1)) >> 64
        perm[i], perm[j] = perm[j], perm[i]
    return perm


def test_training_loop_equals_its_steps():
    """gm_warm_train over 3 epochs gives bit for bit the parameters of the
    same Adam steps called one by one on the documented permutations; the
    shuffle is a permutation and differs between epochs."""
    api = _api()
    n, B = 300, 64
    d = _subset(synth.make("weibel_3v"), n)
    f, _, _ = _oracle_feature_bits(d)
    rng = np.random.default_rng(3)
    t = torch.from_numpy(rng.normal(size=(n, 160)).astype(np.float32) * 0.3).to(dev())
    a = api.WarmStart(16, batch=B, seed=5)
    b = api.WarmStart(16, batch=B, seed=5)
    hist = a.train(f, t, 3, lr=2e-3, lam=0.5, seed=77)
    losses = []
    for e in range(3):
        perm = _epoch_permutation(n, 77, e)
        assert sorted(perm) == list(range(n))
        idx = torch.tensor(perm, dtype=torch.int32, device=dev())
        rows = torch.zeros(n // B, B, dtype=torch.float32, device=dev())
        for s in range(n // B):
            b.train_step(f, t, idx[s * B:(s + 1) * B], lr=2e-3, lam=0.5, loss_rows=rows[s])
        losses.append(float(rows.double().sum().item()) / (n // B * B))
    assert _epoch_permutation(n, 77, 0) != _epoch_permutation(n, 77, 1)
    np.testing.assert_array_equal(a.get_params(), b.get_params())
    np.testing.assert_allclose(hist, losses, rtol=1e-6)
    a.close()
    b.close()


def test_train_step_matches_oracle_gradients_and_adam():
    api = _api()
    B = 200
    d = _subset(synth.make("weibel_3v"), 256)
    f, Xall, _ = _oracle_feature_bits(d)
    rng = np.random.default_rng(8)
    T = np.zeros((256, 160))
    for r in range(256):
        k = rng.integers(1, 6)
        w = np.sort(rng.dirichlet(np.ones(k)))[::-1]
        for j in range(k):
            T[r, 10 * j] = w[j]
            T[r, 10 * j + 1:10 * j + 10] = rng.normal(size=9) * 0.5
    idx = rng.permutation(256)[:B].astype(np.int32)
    P = _params(12)
    m = api.WarmStart(16, batch=B, seed=1)
    flat0 = api.params_to_flat(P)
    m.set_params(flat0)
    Tg = torch.from_numpy(T.astype(np.float32)).to(dev())
    loss_rows = torch.zeros(B, dtype=torch.float32, device=dev())
    lr = 1e-3
    m.train_step(f, Tg, torch.from_numpy(idx).to(dev()), lr=lr, lam=1.0, loss_rows=loss_rows)
    grads = api.flat_to_params(m.gradients())
    X = Xall[idx]
    Lo, go = oracle.mlp_loss_backward(X, P, T[idx].astype(np.float32), lam=1.0, bf16=True)
    loss = float(loss_rows.sum().item()) / B
    print("loss gpu %.6f oracle %.6f" % (loss, Lo))
    assert abs(loss - Lo) <= 1e-3 * abs(Lo)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        gg = grads[name][:105] if name == "W1" else grads[name]
        err = _rel(gg, go[name])
        print("grad %s: relative error %.2e" % (name, err))
        assert err < 1e-3, name
    assert (grads["W1"][105:] == 0).all()
    # first Adam step: m_hat = g, v_hat = g^2, so w -= lr g / (|g| + eps)
    g = m.gradients().astype(np.float64)
    expect = flat0.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    got = m.get_params().astype(np.float64)
    np.testing.assert_allclose(got, expect, rtol=1e-6, atol=1e-6 * lr)
    m.close()


def test_adam_steps_match_torch_adam():
    """Several training steps of the library (gm_warm_train_step: Adam on
    FP32 master weights, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected)
    against torch.optim.Adam, the library implementation of the published
    method, fed the library's own gradient of each step: the moment
    estimates, their bias corrections and the step count must carry over
    from step to step.  FP64 reference, FP32 library: every parameter
    within 2e-6 relative and 1e-4 of the learning rate."""
    api = _api()
    B = 128
    d = _subset(synth.make("weibel_3v"), 256)
    f, _, _ = _oracle_feature_bits(d)
    rng = np.random.default_rng(17)
    T = np.zeros((256, 160), np.float32)
    for r in range(256):
        k = rng.integers(1, 6)
        w = np.sort(rng.dirichlet(np.ones(k)))[::-1]
        for j in range(k):
            T[r, 10 * j] = w[j]
            T[r, 10 * j + 1:10 * j + 10] = rng.normal(size=9) * 0.5
    Tg = torch.from_numpy(T).to(dev())
    m = api.WarmStart(16, batch=B, seed=3)
    lr = 2e-3
    ref = torch.tensor(m.get_params().astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([ref], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for step in range(6):
        idx = torch.from_numpy(rng.permutation(256)[:B].astype(np.int32)).to(dev())
        m.train_step(f, Tg, idx, lr=lr, lam=1.0)
        g = m.gradients().astype(np.float64)
        assert np.abs(g).max() > 0
        opt.zero_grad()
        ref.grad = torch.from_numpy(g)
        opt.step()
        got = m.get_params().astype(np.float64)
        want = ref.detach().numpy()
        err = np.abs(got - want)
        print("step %d: max |library - torch Adam| %.2e (lr %.0e)" % (step + 1, err.max(), lr))
        np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-4 * lr)
    m.close()


def test_decode_matches_oracle():
    api = _api()
    d = _edge_batch()
    _, _, ofr = _oracle_feature_bits(d)
    fr = torch.from_numpy(ofr).to(dev())
    off = torch.from_numpy(d["cell_off"]).to(dev())
    n_cells = len(d["cell_off"]) - 1
    rng = np.random.default_rng(9)
    Y = np.zeros((n_cells, 160), np.float32)
    for j in range(16):
        Y[:, 10 * j] = rng.normal(size=n_cells) * 3.0
        Y[:, 10 * j + 1:10 * j + 4] = rng.normal(size=(n_cells, 3)) * 0.7
        Y[:, 10 * j + 4:10 * j + 10] = rng.normal(size=(n_cells, 6)) * 0.3
    for kmax in (16, 4):
        g = host(api.warm_decode(torch.from_numpy(Y).to(dev()), fr, off, kmax))
        o = oracle.warm_decode(Y, ofr, d["cell_off"], kmax)
        np.testing.assert_array_equal(g["K"], o["K"])
        for k in ("omega", "mu", "sigma"):
            np.testing.assert_allclose(g[k], o[k], rtol=1e-12, atol=1e-15)
        assert (g["K"][-3:] == 0).all() and (g["K"][:-3] >= 1).all()


def test_targets_match_oracle():
    api = _api()
    d = _subset(synth.make("weibel_3v"), 24)
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=3, max_sweeps=40)
    _, ofr = oracle.features(d["v"], d["alpha"], d["cell_off"])
    To = oracle.warm_targets(o, ofr)
    gm = {k: torch.from_numpy(np.ascontiguousarray(o[k])).to(dev()) for k in ("K", "omega", "mu", "sigma")}
    Tg = api.warm_targets(gm, torch.from_numpy(ofr).to(dev())).cpu().numpy()
    np.testing.assert_allclose(Tg, To.astype(np.float32), rtol=1e-6, atol=1e-6)


def _to_dev(init):
    gi = {k: torch.from_numpy(np.ascontiguousarray(val)).to(dev()) for k, val in init.items()}
    gi["K"] = gi["K"].to(torch.int32)
    return gi


def test_pipeline_warm_compress_matches_oracle():
    """features -> network -> decode -> compress on the GPU against the
    oracle's compress started from the same decoded mixtures.  The network
    is set to emit a fixed whitened two-component split (W3 = 0, the split
    in b3), so every cell starts from two components with its own mean and
    covariance.  Converged mode: fallback decisions, K and L agree; the
    stopping sweep of such slowly converging starts is sensitive to FP32
    rounding, so the parameters are compared in replay of the oracle's
    sweep counts."""
    api = _api()
    d = _subset(synth.make("weibel_3v"), 48)
    v, a, off = to_gpu(d)
    P = _params(13)
    P["W3"][:] = 0.0
    b3 = np.zeros(160)
    b3[0::10] = -30.0
    for j, sgn in enumerate((-1.0, 1.0)):
        b3[10 * j] = 0.0
        b3[10 * j + 1] = 0.8 * sgn
        b3[10 * j + 4] = np.log(0.6)
    P["b3"] = b3
    m = api.WarmStart(16, batch=64, seed=1)
    m.set_params(api.params_to_flat(P))
    gi = m.initial_mixtures(v, a, off)
    hg = host(gi)
    # the oracle's own chain: features, BF16 forward pass, decode
    _, X, ofr = _oracle_feature_bits(d)
    _, _, Yo = oracle.mlp_forward(X, P, bf16=True)
    init = oracle.warm_decode(Yo.astype(np.float32), ofr, d["cell_off"], 16)
    assert (init["K"] == 2).all() and (hg["K"] == 2).all()
    for k in ("omega", "mu", "sigma"):
        np.testing.assert_allclose(hg[k], init[k], rtol=1e-6, atol=1e-9)
    g = host(api.compress(v, a, off, 16, seed=4, max_sweeps=150, init=gi))
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=4, max_sweeps=150, init=init)
    fb_g, fb_o = (g["status"] & FALLBACK) != 0, (o["status"] & FALLBACK) != 0
    same_fb = fb_g == fb_o
    near = ((g["status"] | o["status"]) & oracle.STATUS["NEAR_TIE"]) != 0
    sameK = (g["K"] == o["K"]) | near
    print("pipeline: fallback %d (gpu) %d (oracle), decisions equal in %d / 48, K equal in %d, sweeps equal in %d"
          % (fb_g.sum(), fb_o.sum(), same_fb.sum(), sameK.sum(), (g["sweeps"] == o["sweeps"]).sum()))
    assert same_fb.mean() >= 0.95 and sameK.mean() >= 0.9
    eL = np.abs(g["L_final"] - o["L_final"]) / np.abs(o["L_final"])
    assert np.median(eL[sameK & same_fb]) < 1e-5 and np.quantile(eL[sameK & same_fb], 0.9) < 1e-4
    # replay of the oracle's sweeps from the same start (no restarts)
    keep = ~fb_o
    fs = torch.from_numpy(np.where(keep, o["sweeps"], 1).astype(np.int32)).to(dev())
    o2 = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=4, max_sweeps=150, init=init,
                         fixed_sweeps=np.where(keep, o["sweeps"], 1))
    g2 = host(api.compress(v, a, off, 16, seed=4, max_sweeps=150, init=gi, fixed_sweeps=fs))
    np.testing.assert_array_equal(g2["sweeps"], o2["sweeps"])
    res = fp32_parity.resolution(d, 16, 4, o2["sweeps"], o2, init=init)
    fp32_parity.check(g2, o2, d, res, "pipeline replay", cells=list(np.nonzero(keep)[0]))
    m.close()


def test_warm_fallback_matches_oracle():
    d, init = synth.split_start_cells(91, n_cells=12, n=1000, kmax=16)
    v, a, off = to_gpu(d)
    g = host(_api().compress(v, a, off, 16, seed=5, max_sweeps=5, init=_to_dev(init)))
    o = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=16, seed=5, max_sweeps=5, init=init)
    assert ((o["status"] & FALLBACK) != 0).all()
    np.testing.assert_array_equal(g["status"] & FALLBACK, o["status"] & FALLBACK)
    np.testing.assert_array_equal(g["sweeps"], o["sweeps"])
    # every cell fell back: its record is the cold fit's
    res = fp32_parity.resolution(d, 16, 5, o["sweeps"], o)
    fp32_parity.check(g, o, d, res, "fallback")
    # a start at the generating Gaussian is kept
    iu = np.triu_indices(3)
    good = {"K": np.ones(12, np.int32), "omega": np.zeros((12, 16)), "mu": np.zeros((12, 16, 3)),
            "sigma": np.zeros((12, 16, 6))}
    good["omega"][:, 0] = 1.0
    good["mu"][:, 0] = d["truth"]["mu"][:, 0]
    good["sigma"][:, 0] = d["truth"]["sigma"][:, 0][:, iu[0], iu[1]]
    g = host(_api().compress(v, a, off, 16, seed=5, init=_to_dev(good)))
    assert ((g["status"] & FALLBACK) == 0).all() and (g["K"] == 1).all()


def test_training_lowers_the_loss():
    """A few hundred Adam steps on plain-EM targets of 512 cells lower the
    batch loss (trained quality itself is parity unpinned)."""
    api = _api()
    d = _subset(synth.make("weibel_3v", seed=5000), 512)
    v, a, off = to_gpu(d)
    r = api.compress(v, a, off, 16, seed=6)
    f, fr = api.warm_features(v, a, off)
    T = api.warm_targets(r, fr)
    m = api.WarmStart(16, batch=128, seed=2)
    gen = torch.Generator(device="cpu").manual_seed(0)
    loss_rows = torch.zeros(128, dtype=torch.float32, device=dev())
    hist = []
    for step in range(300):
        idx = torch.randperm(512, generator=gen)[:128].to(torch.int32).to(dev())
        m.train_step(f, T, idx, lr=1e-3, lam=1.0, loss_rows=loss_rows)
        if step < 10 or step >= 290:
            hist.append(float(loss_rows.sum().item()) / 128)
    first, last = np.mean(hist[:10]), np.mean(hist[-10:])
    print("training loss %.4f -> %.4f" % (first, last))
    assert np.isfinite(last) and last < 0.7 * first
    m.close()


def test_single_call_warm_compress_equals_composed_path():
    """gm_compress_warm (features, network, decode and compress in one
    library call) gives the record of the composed calls bit for bit, and
    rejects a kmax other than the model's."""
    api = _api()
    d = _subset(synth.make("weibel_3v"), 200)
    v, a, off = to_gpu(d)
    tr = _subset(synth.make("weibel_3v", seed=5002), 1024)
    from paper_2007_12273_amd import warm as warmlib
    feats, targs = warmlib.training_set([tr], 16, seed=2003, device=dev())
    m = api.WarmStart(16, batch=256, seed=7, device=dev())
    warmlib.train(m, feats, targs, epochs=3)
    ref = host(api.compress(v, a, off, 16, seed=2003, init=m.initial_mixtures(v, a, off)))
    wc = api.WarmCompressor(200, m, device=dev(), seed=2003)
    got = host(wc(v, a, off).as_dict())
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    assert (got["K"] > 0).all()
    import ctypes
    from paper_2007_12273_amd import _lib
    bad = api.make_opts(3, 8)
    mix = wc.out.struct()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    assert _lib.load().gm_compress_warm(P(v), P(a), P(off), 200, ctypes.byref(bad), m._h, ctypes.byref(mix), P(wc.ws),
                                        wc.ws.numel(), None) == _lib.GM_EINVAL
    m.close()


def test_unusable_supplied_start_starts_cold_on_gpu():
    """Supplied starts for which eq. (omegak) is undefined (N - T K / 2 <= 0,
    or a component with N w_k <= T/2) are not used: those cells give the cold
    fit bit for bit, flagged as rejected warm starts, as in the oracle."""
    d = synth.concat_cells([synth.random_cells(21 + i, 1, 3, m, m, k_lo=1, k_hi=2) for i, m in enumerate((50, 300, 300))])
    off = d["cell_off"]
    kmax = 16
    init = {"K": np.array([16, 2, 1], np.int32), "omega": np.zeros((3, kmax)), "mu": np.zeros((3, kmax, 3)),
            "sigma": np.zeros((3, kmax, 6))}
    for c in range(3):
        init["mu"][c, :] = d["v"][off[c]:off[c + 1]].mean(0)
        init["sigma"][c, :] = [0.01, 0, 0, 0.01, 0, 0.01]
    init["omega"][0, :16] = 1.0 / 16
    init["omega"][1, :2] = [1.0, 4.0 / 300]
    init["omega"][2, 0] = 1.0
    v, a, offg = to_gpu(d)
    api = _api()
    cold = host(api.compress(v, a, offg, kmax, seed=4, max_sweeps=50))
    g = host(api.compress(v, a, offg, kmax, seed=4, max_sweeps=50, init=_to_dev(init)))
    o = oracle.compress(d["v"], d["alpha"], off, kmax=kmax, seed=4, max_sweeps=50, init=init)
    np.testing.assert_array_equal(g["status"] & FALLBACK, o["status"] & FALLBACK)
    assert (g["status"][:2] & FALLBACK).all() and not (g["status"][2] & FALLBACK)
    for c in (0, 1):
        for k in ("K", "sweeps", "visits", "omega", "mu", "sigma", "L_pen", "L_final"):
            assert np.array_equal(g[k][c], cold[k][c]), (c, k)
        assert g["status"][c] == cold["status"][c] | FALLBACK


def test_fused_inference_equals_forward_and_decode():
    """gm_warm_infer (three layers and the decode in one launch, 32 cells per
    workgroup) gives the mixtures of gm_warm_forward followed by
    gm_warm_decode bit for bit, on a batch that is not a multiple of the
    tile, with trained and with seeded weights."""
    api = _api()
    d = _subset(synth.make("weibel_3v"), 1000)
    v, a, off = to_gpu(d)
    f, fr = api.warm_features(v, a, off)
    from paper_2007_12273_amd import warm as warmlib
    tr = _subset(synth.make("weibel_3v", seed=5003), 1024)
    feats, targs = warmlib.training_set([tr], 16, seed=2003, device=dev())
    for trained in (False, True):
        m = api.WarmStart(16, batch=256, seed=11, device=dev())
        if trained:
            warmlib.train(m, feats, targs, epochs=4)
        ref = host(api.warm_decode(m.forward(f), fr, off, 16))
        out = {"K": torch.empty(1000, dtype=torch.int32, device=dev()),
               "omega": torch.empty(1000, 16, dtype=torch.float64, device=dev()),
               "mu": torch.empty(1000, 16, 3, dtype=torch.float64, device=dev()),
               "sigma": torch.empty(1000, 16, 6, dtype=torch.float64, device=dev())}
        got = host(m.infer(f, fr, off, out))
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (trained, k)
        m.close()
