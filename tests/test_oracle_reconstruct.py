"""Pins of the FP64 oracle's reconstruct path (Sec. 2.4):

* Lemons' projection (eqs. alpha, beta) makes the sample's mass, momentum
  and energy equal the targets to rounding -- a closed form;
* ancestral sampling: component counts follow the mixing weights (chi^2),
  per-component sample means/covariances sit within CLT bounds, whitened
  marginals pass KS against N(0,1), positions pass KS against U(0,1);
* the failure mode of the projection (a negative numerator, or n' = 1 where
  the denominator vanishes) leaves the sample as drawn and flags the cell;
* compress -> reconstruct round trip preserves the original particles'
  W, P and E exactly.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2007_12273_amd import synth


def _pack(S):
    D = S.shape[0]
    return np.array([S[i, j] for i in range(D) for j in range(i, D)])


def _mix_targets(W, w, mu, S):
    P = W * (w[:, None] * mu).sum(0)
    E = 0.5 * W * sum(w[k] * (np.trace(S[k]) + mu[k] @ mu[k]) for k in range(len(w)))
    return np.concatenate([[W], P, [E]])


def _sample_moments(v, w):
    return w.sum(), (w[:, None] * v).sum(0), 0.5 * (w * (v * v).sum(1)).sum()


@pytest.mark.parametrize("D,dx", [(1, 1), (3, 1), (3, 2), (3, 0)])
def test_projection_matches_targets_exactly(D, dx):
    rng = np.random.default_rng(D * 10 + dx)
    n_cells, kmax = 20, 4
    K = rng.integers(1, kmax + 1, size=n_cells).astype(np.int32)
    w = np.zeros((n_cells, kmax))
    mu = np.zeros((n_cells, kmax, D))
    S = np.zeros((n_cells, kmax, D * (D + 1) // 2))
    tg = np.zeros((n_cells, 2 + D))
    for c in range(n_cells):
        w[c, :K[c]] = rng.dirichlet(np.ones(K[c]))
        mu[c, :K[c]] = rng.uniform(-0.5, 0.5, size=(K[c], D))
        Ss = []
        for k in range(K[c]):
            A = rng.normal(size=(D, D)) * 0.05
            Ss.append(A @ A.T + 1e-3 * np.eye(D))
            S[c, k] = _pack(Ss[-1])
        # targets: slightly off the mixture's own moments, as after a weight correction
        tg[c] = _mix_targets(rng.uniform(0.5, 2.0), w[c, :K[c]], mu[c, :K[c]], np.array(Ss))
        tg[c, 1:1 + D] *= 1.01
    counts = rng.integers(20, 400, size=n_cells)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    r = oracle.reconstruct(K, w, mu, S, off, tg, D, dx, seed=3003, stats=True)
    feasible = 2 * tg[:, 1 + D] * tg[:, 0] - (tg[:, 1:1 + D] ** 2).sum(1) > 0
    assert np.all(r["status"][~feasible] == oracle.STATUS["LEMONS_SKIPPED"])
    assert np.all(r["status"][feasible] == 0) and feasible.sum() >= n_cells // 2
    for c in np.nonzero(feasible)[0]:
        sl = slice(off[c], off[c + 1])
        W, P, E = _sample_moments(r["v"][sl], r["w"][sl])
        scale = np.sqrt(2 * tg[c, 0] * tg[c, 1 + D])
        assert W == pytest.approx(tg[c, 0], rel=1e-14)
        assert np.abs(P - tg[c, 1:1 + D]).max() / scale < 1e-13
        assert E == pytest.approx(tg[c, 1 + D], rel=1e-13)
        assert np.all(r["w"][sl] == tg[c, 0] / counts[c])
        if dx:
            assert r["x"][sl].min() >= 0.0 and r["x"][sl].max() < 1.0


def test_projection_failure_modes():
    D = 3
    K = np.array([1, 1, 1], np.int32)
    w = np.array([[1.0], [1.0], [1.0]])
    mu = np.zeros((3, 1, D))
    S = np.tile(_pack(0.01 * np.eye(D)), (3, 1, 1))
    tg = np.array([[1.0, 0, 0, 0, 0.015],      # n' = 1: denominator is zero
                   [1.0, 1.0, 0, 0, 0.1],      # 2 E N' < |P|^2: numerator negative
                   [1.0, 0, 0, 0, 0.015]])     # n' = 0: nothing to do
    off = np.array([0, 1, 101, 101], np.int64)
    r = oracle.reconstruct(K, w, mu, S, off, tg, D, 1, seed=1)
    skip = oracle.STATUS["LEMONS_SKIPPED"]
    assert r["status"][0] == skip and r["status"][1] == skip and r["status"][2] == 0


def test_sampling_statistics():
    """One cell, three well-separated components, n' = 200k."""
    D = 3
    n = 200_000
    w = np.array([[0.5, 0.3, 0.2]])
    mu = np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]])
    rng = np.random.default_rng(4)
    Ss = []
    for k in range(3):
        A = rng.normal(size=(D, D)) * 0.03
        Ss.append(A @ A.T + 0.002 * np.eye(D))
    S = np.array([[_pack(s) for s in Ss]])
    tg = _mix_targets(1.0, w[0], mu[0], np.array(Ss))[None]
    off = np.array([0, n], np.int64)
    r = oracle.reconstruct(np.array([3], np.int32), w, mu, S, off, tg, D, 1, seed=77, stats=True)
    v = r["v"]
    # assign each sample to the nearest mean (components are > 10 sigma apart)
    lab = np.argmin(((v[:, None, :] - mu[0][None]) ** 2).sum(-1), axis=1)
    cnt = np.bincount(lab, minlength=3)
    chi2 = ((cnt - n * w[0]) ** 2 / (n * w[0])).sum()
    assert chi2 < 18.4  # 2 dof, p = 1e-4
    for k in range(3):
        vk = v[lab == k]
        nk = len(vk)
        se = np.sqrt(np.diag(Ss[k]) / nk)
        assert np.all(np.abs(vk.mean(0) - mu[0, k]) < 5 * se + 1e-12)
        C = np.cov(vk.T)
        seC = np.sqrt((Ss[k] ** 2 + np.outer(np.diag(Ss[k]), np.diag(Ss[k]))) / nk)
        assert np.all(np.abs(C - Ss[k]) < 6 * seC)
        # whitened marginals are standard normal
        Lk = np.linalg.cholesky(Ss[k])
        z = np.linalg.solve(Lk, (vk - mu[0, k]).T).T
        for i in range(D):
            assert stats.kstest(z[:, i], "norm").pvalue > 1e-3
    assert abs(r["stats"][0, 0] - 1.0) < 0.01  # the projection is a small correction
    assert stats.kstest(r["x"][:, 0], "uniform").pvalue > 1e-3


def test_deterministic_and_thread_independent():
    D = 3
    K = np.array([2, 1], np.int32)
    w = np.array([[0.6, 0.4], [1.0, 0.0]])
    mu = np.zeros((2, 2, D))
    mu[0, 1] = 0.3
    S = np.tile(_pack(0.01 * np.eye(D)), (2, 2, 1))
    tg = np.array([[1.0, 0.1, 0, 0, 0.05], [2.0, 0, 0, 0, 0.03]])
    off = np.array([0, 500, 900], np.int64)
    a = oracle.reconstruct(K, w, mu, S, off, tg, D, 2, seed=5, nthreads=1)
    b = oracle.reconstruct(K, w, mu, S, off, tg, D, 2, seed=5, nthreads=2)
    c = oracle.reconstruct(K, w, mu, S, off, tg, D, 2, seed=6, nthreads=2)
    assert np.array_equal(a["v"], b["v"]) and np.array_equal(a["x"], b["x"])
    assert not np.array_equal(a["v"], c["v"])


def test_round_trip_preserves_particle_moments():
    d = synth.make("weibel_3v")
    off = d["cell_off"]
    nc, D = 6, 3
    r = oracle.compress(d["v"][:off[nc]], d["alpha"][:off[nc]], off[:nc + 1], kmax=16, seed=2003, max_sweeps=40)
    tg = oracle.targets_from_moments(r["moments"], D)
    counts = np.diff(off[:nc + 1])
    rec = oracle.reconstruct(r["K"], r["omega"], r["mu"], r["sigma"], off[:nc + 1], tg, D, 1, seed=3003)
    assert np.all(rec["status"] == 0)
    for c in range(nc):
        sl = slice(off[c], off[c + 1])
        a = d["alpha"][sl]
        v = d["v"][sl]
        W, P, E = _sample_moments(rec["v"][sl], rec["w"][sl])
        scale = np.sqrt(2 * W * E)
        assert W == pytest.approx(a.sum(), rel=1e-13)
        assert np.abs(P - (a[:, None] * v).sum(0)).max() / scale < 1e-12
        assert E == pytest.approx(0.5 * (a * (v * v).sum(1)).sum(), rel=1e-12)
        assert counts[c] == sl.stop - sl.start


def _tensor_case(D, nc=12, seed=61):
    d = synth.random_cells(seed, nc, D, 60, 400, k_lo=1, k_hi=4)
    mix = oracle.compress(d["v"], d["alpha"], d["cell_off"], kmax=8, seed=3, max_sweeps=40)
    off = d["cell_off"]
    return d, mix, off


@pytest.mark.parametrize("D", [1, 3])
def test_tensor_projection_matches_full_second_moment(D):
    """The full-second-moment projection leaves every cell's sample with the
    record's W, P and the whole tensor S (not only its trace) to rounding."""
    d, mix, off = _tensor_case(D)
    r = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off, mix["moments"], D, 1, seed=7)
    assert (r["status"] & oracle.STATUS["LEMONS_SKIPPED"] == 0).all()
    iu = np.triu_indices(D)
    for c in range(len(off) - 1):
        sl = slice(off[c], off[c + 1])
        v, w = r["v"][sl], r["w"][sl]
        m = mix["moments"][c]
        W, P, S = m[0], m[1:1 + D], m[1 + D:]
        scale = np.abs(S).max()
        assert abs(w.sum() - W) <= 1e-13 * W
        assert np.abs((w[:, None] * v).sum(0) - P).max() <= 1e-12 * np.sqrt(W * scale)
        Sv = (w[:, None, None] * v[:, :, None] * v[:, None, :]).sum(0)[iu]
        assert np.abs(Sv - S).max() <= 1e-12 * scale


def test_tensor_projection_is_lemons_in_one_dimension():
    """In 1V the second moment is the energy, and the affine map matching
    mean and variance is unique: the tensor projection equals eqs. alpha,
    beta particle by particle."""
    d, mix, off = _tensor_case(1, seed=62)
    tg = oracle.targets_from_moments(mix["moments"], 1)
    a = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off, tg, 1, 1, seed=9)
    b = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], off, mix["moments"], 1, 1, seed=9)
    np.testing.assert_array_equal(a["status"], b["status"])
    scale = np.sqrt(tg[:, 2] / tg[:, 0])
    cell_of = np.repeat(np.arange(len(off) - 1), np.diff(off))
    assert (np.abs(a["v"][:, 0] - b["v"][:, 0]) / scale[cell_of]).max() < 1e-12
    np.testing.assert_array_equal(a["x"], b["x"])


def test_tensor_projection_differs_from_scalar_in_3v_and_skips_degenerate():
    """In 3V the scalar projection matches only tr(S); the tensor one also
    the off-diagonal entries.  A one-particle cell has no sample covariance:
    left as drawn and flagged."""
    d, mix, off = _tensor_case(3, seed=63)
    tg = oracle.targets_from_moments(mix["moments"], 3)
    counts = np.diff(off).copy()
    counts[0] = 1
    o2 = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    a = oracle.reconstruct(mix["K"], mix["omega"], mix["mu"], mix["sigma"], o2, tg, 3, 0, seed=5)
    b = oracle.reconstruct_tensor(mix["K"], mix["omega"], mix["mu"], mix["sigma"], o2, mix["moments"], 3, 0, seed=5)
    assert b["status"][0] == oracle.STATUS["LEMONS_SKIPPED"]
    iu = np.triu_indices(3)
    off_diag = [1, 2, 4]
    worse = 0
    for c in range(1, len(o2) - 1):
        sl = slice(o2[c], o2[c + 1])
        S = mix["moments"][c][4:]
        Sa = (a["w"][sl, None, None] * a["v"][sl, :, None] * a["v"][sl, None, :]).sum(0)[iu]
        Sb = (b["w"][sl, None, None] * b["v"][sl, :, None] * b["v"][sl, None, :]).sum(0)[iu]
        assert np.abs(Sb - S).max() <= 1e-12 * np.abs(S).max()
        assert abs(Sa[[0, 3, 5]].sum() - S[[0, 3, 5]].sum()) <= 1e-12 * np.abs(S).max()
        worse += np.abs(Sa[off_diag] - S[off_diag]).max() > 1e-6 * np.abs(S).max()
    assert worse >= (len(o2) - 2) // 2
