"""Pins of the FP64 oracle of the learned warm start:

* forward pass against numpy matmuls (a library routine);
* the analytic backward pass against central finite differences of the loss;
* BF16 rounding against torch's float32 -> bfloat16 conversion;
* features against numpy histograms and moments of the whitened velocities;
* targets -> decode round trip: decoding the targets of a mixture (logits =
  log weights) returns that mixture (components above the N w > T/2 cut).
"""
import numpy as np
import pytest

import oracle
from paper_2007_12273_amd import synth

torch = pytest.importorskip("torch")


def _params(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(size=(105, 256)) * scale, "b1": rng.normal(size=256) * 0.05,
            "W2": rng.normal(size=(256, 256)) * scale * 0.5, "b2": rng.normal(size=256) * 0.05,
            "W3": rng.normal(size=(256, 160)) * scale * 0.5, "b3": rng.normal(size=160) * 0.05}


def _targets(rng, B):
    T = np.zeros((B, 160))
    for r in range(B):
        k = rng.integers(1, 5)
        w = np.sort(rng.dirichlet(np.ones(k)))[::-1]
        for j in range(k):
            T[r, 10 * j] = w[j]
            T[r, 10 * j + 1:10 * j + 10] = rng.normal(size=9) * 0.5
    return T


def test_forward_matches_numpy():
    P = _params(1)
    X = np.random.default_rng(2).normal(size=(7, 105))
    H1, H2, Y = oracle.mlp_forward(X, P)
    h1 = np.maximum(X @ P["W1"] + P["b1"], 0)
    h2 = np.maximum(h1 @ P["W2"] + P["b2"], 0)
    y = h2 @ P["W3"] + P["b3"]
    np.testing.assert_allclose(H1, h1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Y, y, rtol=1e-11, atol=1e-11)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-5, 5, size=2000), [0.0, -0.0, 1.0, 3.0]])
    P = {"W1": np.zeros((105, 256)), "b1": np.zeros(256), "W2": np.eye(256), "b2": np.zeros(256),
         "W3": np.zeros((256, 160)), "b3": np.zeros(160)}
    # route values through the first layer's input rounding: X[:,0] * W1[0,:] with W1 = 1
    X = np.zeros((len(x), 105))
    X[:, 0] = x
    P["W1"][0, 0] = 1.0
    H1, _, _ = oracle.mlp_forward(X, P, bf16=True)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    pos = ref > 0
    np.testing.assert_array_equal(H1[pos, 0], ref[pos])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    P = _params(5)
    B = 6
    X = rng.normal(size=(B, 105))
    Tg = _targets(rng, B)
    L0, g = oracle.mlp_loss_backward(X, P, Tg)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = P[name].reshape(-1)
        idx = rng.choice(flat.size, 12, replace=False)
        for i in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name].reshape(-1)[i] += h
            Pm[name].reshape(-1)[i] -= h
            Lp, _ = oracle.mlp_loss_backward(X, Pp, Tg)
            Lm, _ = oracle.mlp_loss_backward(X, Pm, Tg)
            fd = (Lp - Lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-7 + 1e-5 * abs(fd), (name, i, fd, an)


def test_features_match_numpy():
    d = synth.make("weibel_3v")
    nc = 6
    off = d["cell_off"][:nc + 1]
    v, a = d["v"][:off[-1]], d["alpha"][:off[-1]]
    f, fr = oracle.features(v, a, off)
    for c in range(nc):
        vc, ac = v[off[c]:off[c + 1]], a[off[c]:off[c + 1]]
        W = ac.sum()
        m = (ac[:, None] * vc).sum(0) / W
        C = np.cov(vc.T, aweights=ac, bias=True)
        L = np.linalg.cholesky(C)
        u = np.linalg.solve(L, (vc - m).T).T
        q = ac / W
        np.testing.assert_allclose(fr[c, :3], m, rtol=1e-12, atol=1e-14)
        for dd in range(3):
            h, _ = np.histogram(np.clip(u[:, dd], -4, 4 - 1e-12), bins=32, range=(-4, 4), weights=q)
            np.testing.assert_allclose(f[c, 32 * dd:32 * dd + 32], h, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(f[c, 96 + dd], (q * u[:, dd] ** 3).sum(), rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(f[c, 99 + dd], (q * u[:, dd] ** 4).sum() - 3, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(f[c, 102], (q * u[:, 0] ** 2 * u[:, 1] ** 2).sum() - 1, rtol=1e-9, atol=1e-12)
        # whitening: the weighted second moment of u is the identity
        np.testing.assert_allclose((q[:, None, None] * u[:, :, None] * u[:, None, :]).sum(0), np.eye(3), atol=1e-10)


def test_targets_decode_round_trip():
    d = synth.make("weibel_3v")
    nc = 8
    off = d["cell_off"][:nc + 1]
    v, a = d["v"][:off[-1]], d["alpha"][:off[-1]]
    mix = oracle.compress(v, a, off, kmax=16, seed=3, max_sweeps=40)
    f, fr = oracle.features(v, a, off)
    Tg = oracle.warm_targets(mix, fr)
    Y = Tg.copy()
    for j in range(16):
        w = Tg[:, 10 * j]
        Y[:, 10 * j] = np.where(w > 0, np.log(np.maximum(w, 1e-300)), -1e4)
    dec = oracle.warm_decode(Y, fr, off, 16)
    for c in range(nc):
        n = off[c + 1] - off[c]
        K = mix["K"][c]
        keep = [k for k in range(K) if n * mix["omega"][c, k] > 4.5]
        assert dec["K"][c] == len(keep)
        # decode keeps slot order = targets' order (weight descending)
        order = sorted(keep, key=lambda k: (-mix["omega"][c, k], 0))
        wsum = mix["omega"][c, keep].sum()
        for q, k in enumerate(order):
            assert dec["omega"][c, q] == pytest.approx(mix["omega"][c, k] / wsum, rel=1e-12)
            np.testing.assert_allclose(dec["mu"][c, q], mix["mu"][c, k], rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(dec["sigma"][c, q], mix["sigma"][c, k], rtol=1e-8, atol=1e-14)


def test_decode_without_frame_keeps_cold_start():
    """Cells with no whitening frame (empty, singular covariance) decode to
    K = 0 with zero slots, so compress starts them cold."""
    Y = np.random.default_rng(1).normal(size=(3, 160))
    fr = np.zeros((3, 9))
    fr[0, :3] = 0.2
    off = np.array([0, 0, 7, 8], np.int64)
    dec = oracle.warm_decode(Y, fr, off, 16)
    assert (dec["K"] == 0).all()
    assert not dec["omega"].any() and not dec["mu"].any() and not dec["sigma"].any()


def _tri_sym(s):
    return np.array([[s[0], s[1], s[2]], [s[1], s[3], s[4]], [s[2], s[4], s[5]]])


def test_decode_and_targets_follow_the_cell_frame():
    """Decode and targets written out as maps between a cell's frame (mean
    m, lower Cholesky factor L of its covariance) and the whitened network
    space, checked for what those maps must satisfy whatever their formulas:
    under a change of velocity coordinates v -> a + B v with B lower
    triangular (so the new frame is a + B m, B L), decoding the same network
    output gives means a + B mu and covariances B Sigma B^T with the same
    K and weights, and the targets of a mixture moved the same way are
    unchanged; adding a constant to every slot's logit changes nothing.  A
    transposed frame factor, a mean added in the wrong space or a whitening
    on the wrong side fails the first two."""
    rng = np.random.default_rng(21)
    d = synth.make("weibel_3v")
    nc = 6
    off = d["cell_off"][:nc + 1]
    v, al = d["v"][:off[-1]], d["alpha"][:off[-1]]
    _, fr = oracle.features(v, al, off)
    Y = rng.normal(size=(nc, 160)) * 0.4
    Y[:, 0::10] = rng.normal(size=(nc, 16)) * 2.0  # logits
    a = rng.normal(size=3)
    B = np.tril(rng.normal(size=(3, 3)) * 0.3) + np.diag(rng.uniform(0.5, 2.0, 3))
    fr2 = fr.copy()
    for c in range(nc):
        L = np.array([[fr[c, 3], 0, 0], [fr[c, 4], fr[c, 5], 0], [fr[c, 6], fr[c, 7], fr[c, 8]]])
        L2 = B @ L
        fr2[c, :3] = a + B @ fr[c, :3]
        fr2[c, 3:] = [L2[0, 0], L2[1, 0], L2[1, 1], L2[2, 0], L2[2, 1], L2[2, 2]]
    d1 = oracle.warm_decode(Y, fr, off, 16)
    d2 = oracle.warm_decode(Y, fr2, off, 16)
    np.testing.assert_array_equal(d1["K"], d2["K"])
    assert (d1["K"] >= 1).all()
    np.testing.assert_allclose(d1["omega"], d2["omega"], rtol=1e-14)
    iu = np.triu_indices(3)
    for c in range(nc):
        for q in range(d1["K"][c]):
            np.testing.assert_allclose(d2["mu"][c, q], a + B @ d1["mu"][c, q], rtol=1e-12, atol=1e-12)
            S2 = B @ _tri_sym(d1["sigma"][c, q]) @ B.T
            np.testing.assert_allclose(d2["sigma"][c, q], S2[iu], rtol=1e-10, atol=1e-14)
    # the same logits shifted by a constant decode alike
    Ys = Y.copy()
    Ys[:, 0::10] += 7.5
    d3 = oracle.warm_decode(Ys, fr, off, 16)
    for k in d1:
        np.testing.assert_allclose(d3[k], d1[k], rtol=1e-12, atol=1e-15)
    # targets of a mixture are invariant under the same move of mixture and frame
    mix = oracle.compress(v, al, off, kmax=16, seed=3, max_sweeps=40)
    mix2 = {"K": mix["K"], "omega": mix["omega"], "mu": mix["mu"].copy(), "sigma": mix["sigma"].copy()}
    for c in range(nc):
        for k in range(mix["K"][c]):
            mix2["mu"][c, k] = a + B @ mix["mu"][c, k]
            mix2["sigma"][c, k] = (B @ _tri_sym(mix["sigma"][c, k]) @ B.T)[iu]
    t1 = oracle.warm_targets(mix, fr)
    t2 = oracle.warm_targets(mix2, fr2)
    np.testing.assert_allclose(t2, t1, rtol=1e-9, atol=1e-9)
