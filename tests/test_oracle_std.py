"""Pins of the oracle's standard (non-adaptive) EM with K-means start and
Anderson acceleration (Sec. 3.4), independent of the oracle's own code:

* the Anderson least-squares step against numpy's lstsq, and its
  detection of a dependent column;
* K-means against scikit-learn's Lloyd KMeans from the same centres
  (labels, centres), and the hard-assignment mixture against its closed
  form;
* plain standard EM against scikit-learn's GaussianMixture from the same
  start (weights, means, covariances after the same number of steps);
* Anderson-accelerated EM on separated clusters: the same maximum as plain
  EM (a fixed point of the EM map), exact moments after the finish.
"""
import numpy as np
import pytest

import oracle


def _cells(seed, n_cells, n, sep, D=3):
    rng = np.random.default_rng(seed)
    vs = []
    for c in range(n_cells):
        centres = rng.normal(size=(3, D)) * sep
        lab = rng.integers(0, 3, size=n)
        vs.append(centres[lab] + rng.normal(size=(n, D)) * rng.uniform(0.05, 0.15, size=D))
    off = np.arange(n_cells + 1, dtype=np.int64) * n
    return np.concatenate(vs), off


def test_anderson_least_squares_matches_lstsq():
    rng = np.random.default_rng(0)
    for mk in (1, 3, 5):
        A = rng.normal(size=(60, mk))
        f = rng.normal(size=60)
        np.testing.assert_allclose(oracle.aa_solve(A, f), np.linalg.lstsq(A, f, rcond=None)[0], rtol=1e-12,
                                   atol=1e-14)
    A = rng.normal(size=(40, 3))
    A[:, 2] = A[:, 0] - 2.0 * A[:, 1]
    assert oracle.aa_solve(A, rng.normal(size=40)) is None


def test_kmeans_matches_sklearn():
    from sklearn.cluster import KMeans
    v, off = _cells(3, 1, 900, 1.0)
    x = v - v.mean(0)
    a = np.ones(len(x))
    idx = np.array([5, 300, 777], np.int32)
    w, mu, S, asg, passes = oracle.kmeans(x, a, 3, idx)
    km = KMeans(n_clusters=3, init=x[idx], n_init=1, algorithm="lloyd", max_iter=100, tol=0.0).fit(x)
    assert np.array_equal(asg, km.labels_)
    np.testing.assert_allclose(mu, km.cluster_centers_, rtol=1e-12, atol=1e-14)
    assert 1 < passes <= 100
    iu = np.triu_indices(3)
    for k in range(3):
        xk = x[asg == k]
        assert w[k] == pytest.approx(len(xk) / len(x), rel=1e-14)
        np.testing.assert_allclose(S[k], np.cov(xk.T, bias=True)[iu], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("steps", [1, 7])
def test_plain_standard_em_matches_sklearn(steps):
    """max_iter = s evaluations of G, then the finish's EM step: s + 1 EM
    steps from the cold start, as scikit-learn takes from the same start."""
    from sklearn.mixture import GaussianMixture
    v, off = _cells(4, 1, 700, 0.6)
    K = 3
    r = oracle.compress_std(v, np.ones(len(v)), off, K, seed=11, max_iter=steps, tol=0.0)
    idx = oracle.init_indices(len(v), K, 11, 0)
    C = np.cov(v.T, bias=True)
    gm = GaussianMixture(n_components=K, covariance_type="full", reg_covar=0.0, tol=0.0, max_iter=steps + 1,
                         weights_init=np.full(K, 1.0 / K), means_init=v[idx], precisions_init=np.stack(
                             [np.linalg.inv(C)] * K))
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(v)
    iu = np.triu_indices(3)
    np.testing.assert_allclose(r["omega"][0, :K], gm.weights_, rtol=1e-8)
    np.testing.assert_allclose(r["mu"][0, :K], gm.means_, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(r["sigma"][0, :K], gm.covariances_[:, iu[0], iu[1]], rtol=1e-7, atol=1e-10)


def test_anderson_lands_on_the_plain_maximum():
    v, off = _cells(5, 12, 800, 0.8)
    a = np.ones(len(v))
    p = oracle.compress_std(v, a, off, 3, seed=2, max_iter=3000, tol=1e-11)
    q = oracle.compress_std(v, a, off, 3, seed=2, aa_m=5, max_iter=3000, tol=1e-11)
    k = oracle.compress_std(v, a, off, 3, seed=2, aa_m=5, kmeans=True, max_iter=3000, tol=1e-11)
    same = np.abs(q["ll"] - p["ll"]) <= 1e-7 * np.abs(p["ll"])
    print("plain iterations", p["iters"].tolist(), "\nAnderson", q["iters"].tolist(), "\nK-means + Anderson",
          k["iters"].tolist())
    # a converged Anderson iteration is a fixed point of the EM map: where
    # it found the same maximum, the same parameters
    assert same.mean() >= 0.75
    for c in np.nonzero(same)[0]:
        o = np.argsort(p["mu"][c, :3, 0])
        o2 = np.argsort(q["mu"][c, :3, 0])
        np.testing.assert_allclose(q["mu"][c, o2], p["mu"][c, o], rtol=0, atol=1e-5)
        np.testing.assert_allclose(q["omega"][c, o2], p["omega"][c, o], rtol=0, atol=1e-5)
    assert (q["resets"] >= 0).all() and (p["resets"] == 0).all()
    # exact moments after the finish
    iu = np.triu_indices(3)
    for r in (p, q, k):
        for c in range(12):
            K = r["K"][c]
            w, mu, sg = r["omega"][c, :K], r["mu"][c, :K], r["sigma"][c, :K]
            m = r["moments"][c]
            W = m[0]
            assert np.abs(W * (w[:, None] * mu).sum(0) - m[1:4]).max() <= 1e-11 * np.abs(m[4:]).max() ** 0.5 * W ** 0.5
            S = W * (w[:, None] * (sg + (mu[:, :, None] * mu[:, None, :])[:, iu[0], iu[1]])).sum(0)
            assert np.abs(S - m[4:]).max() <= 1e-11 * np.abs(m[4:]).max()


def test_standard_em_stop_rule_resolution():
    """What the stop rule (relative change of the log-likelihood below 1e-7)
    fixes for the standard EM with more components than the data needs:
    the log-likelihood to about 1e-6 relative, the parameters only to about
    1e-3 (median) - the scale of the GPU's converged-mode parameter bars."""
    from paper_2007_12273_amd import synth
    from gpu_util import mixture_errors
    d = synth.make("weibel_3v", n_cells=16)
    off = d["cell_off"]
    a = oracle.compress_std(d["v"], d["alpha"], off, 8, seed=2003, kmax=16, aa_m=5, tol=1e-7)
    b = oracle.compress_std(d["v"], d["alpha"], off, 8, seed=2003, kmax=16, aa_m=5, tol=1e-9, max_iter=5000)
    same = [c for c in range(16) if a["K"][c] == b["K"][c] and abs(a["ll"][c] - b["ll"][c]) <= 1e-5 * abs(b["ll"][c])]
    eL = np.array([abs(a["ll"][c] - b["ll"][c]) / abs(b["ll"][c]) for c in same])
    ep = np.array([max(mixture_errors(a, b, c, 3)) for c in same])
    print("same maximum in %d / 16; L moved by median %.1e, parameters by median %.1e (max %.1e)"
          % (len(same), np.median(eL), np.median(ep), ep.max()))
    assert len(same) >= 8  # tighter mixing can also settle on another maximum
    assert np.median(eL) < 1e-6
    assert np.median(ep) > 1e-4 and ep.max() < 0.1
