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


def spline2(s):
    """Quadratic B-spline, written out for property checks of GPU outputs."""
    a = np.abs(s)
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def deposit_at(x, w, off, dx, nx, cells):
    """Charge sum_p w_p S2(X_i - X_p) on the given mesh cells of the periodic
    unit mesh, by brute force over the particles of the neighbouring cells
    (the definition; a property check of outputs, not a reference)."""
    n_cells = len(off) - 1
    ny = n_cells // nx if dx == 2 else 1
    nxx = nx if dx == 2 else n_cells
    out = []
    for i in cells:
        ix, iy = (i % nxx, i // nxx) if dx == 2 else (i, 0)
        tot = 0.0
        for oy in ((-1, 0, 1) if dx == 2 else (0,)):
            for ox in (-1, 0, 1):
                j = (((iy + oy) % ny) * nxx + (ix + ox) % nxx) if dx == 2 else (ix + ox) % nxx
                sl = slice(off[j], off[j + 1])
                xs = np.asarray(x[sl]).reshape(-1, dx)
                s = spline2(0.5 - ox - xs[:, 0])
                if dx == 2:
                    s = s * spline2(0.5 - oy - xs[:, 1])
                tot += float((np.asarray(w[sl]) * s).sum())
        out.append(tot)
    return np.array(out)


def take_cells(d, cells):
    """The batch made of the given cells of d, in that order (renumbered)."""
    off = d["cell_off"]
    cells = np.asarray(cells)
    counts = np.array([off[c + 1] - off[c] for c in cells], dtype=np.int64)
    so = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    v = np.concatenate([d["v"][off[c]:off[c + 1]] for c in cells])
    a = np.concatenate([d["alpha"][off[c]:off[c + 1]] for c in cells])
    return dict(v=v, alpha=a, cell_off=so)
