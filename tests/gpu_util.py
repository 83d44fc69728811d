"""Helpers shared by the GPU tests: device transfer and comparison metrics."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_gpu(d):
    g = dev()
    v = torch.from_numpy(np.ascontiguousarray(d["v"], dtype=np.float64)).to(g)
    a = torch.from_numpy(np.ascontiguousarray(d["alpha"], dtype=np.float64)).to(g)
    off = torch.from_numpy(np.ascontiguousarray(d["cell_off"], dtype=np.int64)).to(g)
    return v, a, off


def host(r):
    return {k: (t.cpu().numpy() if t is not None else None) for k, t in r.items()}


def unpack(D, s):
    S = np.zeros((D, D))
    t = 0
    for i in range(D):
        for j in range(i, D):
            S[i, j] = S[j, i] = s[t]
            t += 1
    return S


def mixture_errors(g, o, c, D):
    """Per-cell parameter errors between two records with identical K and
    slot order: |d omega| absolute, |d mu| / sqrt(tr C / D), |d Sigma|_F / |Sigma|_F."""
    K = int(o["K"][c])
    mom = o["moments"][c]
    W = mom[0]
    S = unpack(D, mom[1 + D:])
    m = mom[1:1 + D] / W
    C = S / W - np.outer(m, m)
    scale = np.sqrt(max(np.trace(C) / D, 1e-300))
    ew = np.abs(g["omega"][c, :K] - o["omega"][c, :K]).max()
    em = np.abs(g["mu"][c, :K] - o["mu"][c, :K]).max() / scale
    es = max(np.linalg.norm(unpack(D, g["sigma"][c, k]) - unpack(D, o["sigma"][c, k])) /
             np.linalg.norm(unpack(D, o["sigma"][c, k])) for k in range(K))
    return ew, em, es


def conservation(rec, c, D):
    """Relative residuals of mass, momentum, second moment of a record."""
    K = int(rec["K"][c])
    mom = rec["moments"][c]
    W = mom[0]
    P = mom[1:1 + D]
    S = unpack(D, mom[1 + D:])
    w = rec["omega"][c, :K]
    mu = rec["mu"][c, :K]
    Pm = W * (w[:, None] * mu).sum(0)
    Sm = W * sum(w[k] * (unpack(D, rec["sigma"][c, k]) + np.outer(mu[k], mu[k])) for k in range(K))
    scale = np.sqrt(W * np.trace(S))
    return abs(w.sum() - 1.0), np.abs(Pm - P).max() / scale, np.abs(Sm - S).max() / np.trace(S)
