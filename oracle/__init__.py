"""FP64 CPU oracle for the Gaussian-mixture checkpoint-restart hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library and its Python
binding never do.  The arithmetic lives in ``gm_oracle.c`` (plain loops,
FP64, written from the paper); this module only marshals numpy arrays.

Parity status (see each test module): compress, finish, reconstruct and
Philox are pinned (closed forms, library special cases, invariants,
known-answer values); the choice among local maxima on general data is
"parity unpinned" beyond the shared initialisation rule.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GM_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload the ASan runtime;
# tests/test_oracle_sanitizers.py runs it in a subprocess)
_SANITIZE = os.environ.get("GM_ORACLE_SANITIZE") == "1"
_SO = os.path.join(_HERE, "libgmoracle_san.so" if _SANITIZE else "libgmoracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("gm_oracle.c", "gm_oracle_mlp.c") if os.path.exists(os.path.join(_HERE, f))]

STATUS = {
    "SMALL_CELL_K1": 1 << 0, "K0_CAPPED": 1 << 1, "COV_FLOOR": 1 << 2, "MAXSWEEPS": 1 << 3,
    "NEAR_TIE": 1 << 4, "WARM_FALLBACK": 1 << 5, "NONFINITE_INPUT": 1 << 6,
    "LEMONS_SKIPPED": 1 << 7, "DEGENERATE": 1 << 8,
}
MODE_STANDARD_EM = 1
MODE_NO_FINISH = 2
MODE_OUTER_K = 4
MODE_ROUND32 = 8


def build(force=False):
    """Compile the oracle with gcc (-O2, plain C, pthreads)."""
    if not force and os.path.exists(_SO) and all(os.path.getmtime(_SO) >= os.path.getmtime(s) for s in _SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] \
        if _SANITIZE else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=gnu11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                           "-o", tmp] + _SRC + ["-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I32, I64, F64, U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64


def _declare(L):
    L.orc_philox4x64_10.argtypes = [P, P, P]
    L.orc_philox4x64_10.restype = None
    L.orc_compress.argtypes = [P, P, P, I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, F64, U64,
                               ctypes.c_int, F64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
    L.orc_compress.restype = ctypes.c_int
    L.orc_init_indices.argtypes = [ctypes.c_int, ctypes.c_int, U64, U64, P]
    L.orc_init_indices.restype = None
    L.orc_mle_finish.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
    L.orc_mle_finish.restype = ctypes.c_int
    L.orc_penalised_L.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, F64]
    L.orc_penalised_L.restype = F64
    L.orc_reconstruct.argtypes = [P, P, P, P, ctypes.c_int, P, P, I64, ctypes.c_int, ctypes.c_int, U64,
                                  P, P, P, P, P, ctypes.c_int]
    L.orc_reconstruct_tensor.argtypes = [P, P, P, P, ctypes.c_int, P, P, I64, ctypes.c_int, ctypes.c_int, U64,
                                         P, P, P, P, ctypes.c_int]
    L.orc_reconstruct_tensor.restype = ctypes.c_int
    L.orc_project.argtypes = [P, P, P, P, I64, ctypes.c_int, ctypes.c_int, P]
    L.orc_project.restype = ctypes.c_int
    C = ctypes.c_int
    L.orc_compress_std.argtypes = [P, P, P, I64, C, C, C, C, C, F64, U64, C, C, P, P, P, P, P, P, P, P, P, P, P, P, C]
    L.orc_compress_std.restype = C
    L.orc_aa_solve.argtypes = [C, C, P, P, P]
    L.orc_aa_solve.restype = C
    L.orc_kmeans.argtypes = [P, P, C, C, C, P, P, P, P, P]
    L.orc_kmeans.restype = C
    L.orc_reconstruct.restype = ctypes.c_int
    if hasattr(L, "orc_features"):
        _declare_mlp(L)


def _declare_mlp(L):
    L.orc_features.argtypes = [P, P, P, I64, P, P]
    L.orc_features.restype = ctypes.c_int
    L.orc_mlp_forward.argtypes = [P, ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, P, P, P]
    L.orc_mlp_forward.restype = ctypes.c_int
    L.orc_mlp_loss_backward.argtypes = [P, ctypes.c_int, P, P, P, P, P, P, P, F64, ctypes.c_int,
                                        P, P, P, P, P, P, P]
    L.orc_mlp_loss_backward.restype = F64
    L.orc_warm_decode.argtypes = [P, P, P, I64, ctypes.c_int, P, P, P, P]
    L.orc_warm_decode.restype = ctypes.c_int
    L.orc_warm_targets.argtypes = [P, P, P, P, P, I64, ctypes.c_int, P]
    L.orc_warm_targets.restype = ctypes.c_int


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def default_threads():
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def ntri(D):
    return D * (D + 1) // 2


def philox4x64_10(ctr, key):
    c = _c(ctr, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def init_indices(n, K0, seed, cell):
    perm = np.zeros(n, dtype=np.int32)
    lib().orc_init_indices(n, K0, seed, cell, _p(perm))
    return perm[:K0].copy()


def compress(v, alpha, cell_off, kmax, seed, D=None, n_min=10, max_sweeps=1000, fixed_sweeps=None, tol=1e-7,
             mode=0, T=-1.0, init=None, trace=False, nthreads=None):
    """Adaptive EM-GM compress of every cell (FP64).  Returns a dict of arrays.

    ``init`` (optional): dict with K [n_cells], omega [n_cells, kmax],
    mu [n_cells, kmax, D] (original coordinates), sigma [n_cells, kmax, ntri(D)];
    cells with K > 0 start from it instead of the random cold start.
    """
    v = _c(v, np.float64)
    if v.ndim == 1:
        v = v[:, None]
    D = v.shape[1] if D is None else D
    alpha = _c(alpha, np.float64)
    off = _c(cell_off, np.int64)
    n_cells = len(off) - 1
    nt = ntri(D)
    out = {
        "K": np.zeros(n_cells, np.int32), "omega": np.zeros((n_cells, kmax)),
        "mu": np.zeros((n_cells, kmax, D)), "sigma": np.zeros((n_cells, kmax, nt)),
        "moments": np.zeros((n_cells, 1 + D + nt)), "L_pen": np.zeros(n_cells), "L_final": np.zeros(n_cells),
        "sweeps": np.zeros(n_cells, np.int32), "status": np.zeros(n_cells, np.int32),
        "visits": np.zeros(n_cells, np.int64), "margin": np.zeros(n_cells),
    }
    fs = None if fixed_sweeps is None else _c(np.broadcast_to(fixed_sweeps, (n_cells,)), np.int32)
    Lt = Kt = None
    if trace:
        Lt = np.full((n_cells, max_sweeps), np.nan)
        Kt = np.zeros((n_cells, max_sweeps), np.int32)
    iK = iw = imu = iS = None
    if init is not None:
        iK = _c(init["K"], np.int32)
        iw = _c(init["omega"], np.float64)
        imu = _c(init["mu"], np.float64)
        iS = _c(init["sigma"], np.float64)
    rc = lib().orc_compress(_p(v), _p(alpha), _p(off), n_cells, D, kmax, n_min, max_sweeps, _p(fs), tol, seed, mode,
                            float(T), _p(iK), _p(iw), _p(imu), _p(iS), _p(out["K"]), _p(out["omega"]),
                            _p(out["mu"]), _p(out["sigma"]), _p(out["moments"]), _p(out["L_pen"]),
                            _p(out["L_final"]), _p(out["sweeps"]), _p(out["status"]), _p(out["visits"]), _p(Lt),
                            _p(Kt), _p(out["margin"]), nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_compress rejected its arguments")
    if trace:
        out["L_trace"] = Lt
        out["K_trace"] = Kt
    return out


def mle_finish(v, alpha, omega, mu, sigma):
    """One unpenalised joint EM step on one cell from an arbitrary mixture."""
    v = _c(v, np.float64)
    if v.ndim == 1:
        v = v[:, None]
    n, D = v.shape
    w = _c(omega, np.float64).copy()
    m = _c(mu, np.float64).copy()
    S = _c(sigma, np.float64).copy()
    rc = lib().orc_mle_finish(_p(v), _p(_c(alpha, np.float64)), n, D, len(w), _p(w), _p(m), _p(S))
    if rc != 0:
        raise ValueError("mle_finish: a covariance is not positive definite")
    return w, m, S


def penalised_L(v, alpha, omega, mu, sigma, T=-1.0):
    v = _c(v, np.float64)
    if v.ndim == 1:
        v = v[:, None]
    n, D = v.shape
    return lib().orc_penalised_L(_p(v), _p(_c(alpha, np.float64)), n, D, len(omega), _p(_c(omega, np.float64)),
                                 _p(_c(mu, np.float64)), _p(_c(sigma, np.float64)), float(T))


def compress_std(v, alpha, cell_off, K, seed, kmax=None, kmeans=False, aa_m=0, n_min=10, max_iter=1000, tol=1e-7,
                 trace=False, nthreads=None):
    """Standard (non-adaptive) EM of every cell (Sec. 3.4): K components,
    random or K-means start, Anderson memory aa_m (0: plain EM), then the
    unpenalised finish.  Returns a dict of arrays; ``ll`` is the
    log-likelihood at the last iterate, ``resets`` the Anderson resets."""
    v = _c(v, np.float64)
    if v.ndim == 1:
        v = v[:, None]
    D = v.shape[1]
    kmax = K if kmax is None else kmax
    alpha = _c(alpha, np.float64)
    off = _c(cell_off, np.int64)
    n_cells = len(off) - 1
    nt = ntri(D)
    out = {
        "K": np.zeros(n_cells, np.int32), "omega": np.zeros((n_cells, kmax)),
        "mu": np.zeros((n_cells, kmax, D)), "sigma": np.zeros((n_cells, kmax, nt)),
        "moments": np.zeros((n_cells, 1 + D + nt)), "ll": np.zeros(n_cells), "L_final": np.zeros(n_cells),
        "iters": np.zeros(n_cells, np.int32), "status": np.zeros(n_cells, np.int32),
        "resets": np.zeros(n_cells, np.int32), "kmeans_passes": np.zeros(n_cells, np.int32),
    }
    lt = np.full((n_cells, max_iter), np.nan) if trace else None
    rc = lib().orc_compress_std(_p(v), _p(alpha), _p(off), n_cells, D, kmax, K, n_min, max_iter, tol, seed,
                                int(kmeans), aa_m, _p(out["K"]), _p(out["omega"]), _p(out["mu"]), _p(out["sigma"]),
                                _p(out["moments"]), _p(out["ll"]), _p(out["L_final"]), _p(out["iters"]),
                                _p(out["status"]), _p(out["resets"]), _p(out["kmeans_passes"]), _p(lt),
                                nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_compress_std rejected its arguments")
    if trace:
        out["ll_trace"] = lt
    return out


def kmeans(x, a, K, idx):
    """K-means (Lloyd) of the standard-EM start on centred particles x with
    weights a from the particles idx; returns (w, mu, sigma packed, assign,
    passes) where w sums the assigned weights divided by their total."""
    x = _c(x, np.float64)
    n, D = x.shape
    w = np.zeros(K)
    mu = np.zeros((K, D))
    S = np.zeros((K, ntri(D)))
    asg = np.zeros(n, np.int32)
    passes = lib().orc_kmeans(_p(x), _p(_c(a, np.float64)), n, D, K, _p(_c(idx, np.int32)), _p(w), _p(mu), _p(S),
                              _p(asg))
    if passes < 0:
        raise ValueError("orc_kmeans rejected its arguments")
    return w, mu, S, asg, passes


def aa_solve(dF, f):
    """The Anderson least-squares step: gamma = argmin |f - dF gamma| by
    modified Gram-Schmidt (dF: len x mk).  None when a column is dependent."""
    dF = np.asarray(dF, dtype=np.float64)
    cols = _c(dF.T, np.float64)
    g = np.zeros(dF.shape[1])
    rc = lib().orc_aa_solve(dF.shape[0], dF.shape[1], _p(cols), _p(_c(f, np.float64)), _p(g))
    if rc == -2:
        raise ValueError("orc_aa_solve rejected its arguments")
    return None if rc != 0 else g


def reconstruct(K, omega, mu, sigma, out_off, target, D, dx, seed, stats=False, nthreads=None):
    K = _c(K, np.int32)
    omega = _c(omega, np.float64)
    kmax = omega.shape[1]
    mu = _c(mu, np.float64)
    sigma = _c(sigma, np.float64)
    off = _c(out_off, np.int64)
    target = _c(target, np.float64)
    n_cells = len(off) - 1
    n = int(off[-1])
    v = np.zeros((n, D))
    w = np.zeros(n)
    x = np.zeros((n, dx)) if dx > 0 else None
    st = np.zeros(n_cells, np.int32)
    sb = np.zeros((n_cells, 4)) if stats else None
    rc = lib().orc_reconstruct(_p(K), _p(omega), _p(mu), _p(sigma), kmax, _p(off), _p(target), n_cells, D, dx, seed,
                               _p(v), _p(w), _p(x), _p(st), _p(sb), nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_reconstruct rejected its arguments")
    out = {"v": v, "w": w, "x": x, "status": st}
    if stats:
        out["stats"] = sb
    return out


def reconstruct_tensor(K, omega, mu, sigma, out_off, moments, D, dx, seed, nthreads=None):
    """Sampling as reconstruct(); projection matching W, P and the full
    second moment S of the moments record (W, P, S packed per cell)."""
    K = _c(K, np.int32)
    omega = _c(omega, np.float64)
    kmax = omega.shape[1]
    off = _c(out_off, np.int64)
    mom = _c(moments, np.float64)
    n_cells = len(off) - 1
    n = int(off[-1])
    v = np.zeros((n, D))
    w = np.zeros(n)
    x = np.zeros((n, dx)) if dx > 0 else None
    st = np.zeros(n_cells, np.int32)
    rc = lib().orc_reconstruct_tensor(_p(K), _p(omega), _p(_c(mu, np.float64)), _p(_c(sigma, np.float64)), kmax,
                                      _p(off), _p(mom), n_cells, D, dx, seed, _p(v), _p(w), _p(x), _p(st),
                                      nthreads or default_threads())
    if rc != 0:
        raise ValueError("orc_reconstruct_tensor rejected its arguments")
    return {"v": v, "w": w, "x": x, "status": st}


def project(v, w, cell_off, moments, D, tensor=False):
    """Projection of given particles (copies of v, w) towards the moments
    record: Lemons' scalar form or the full second moment.  Returns
    (v', status)."""
    v = np.array(v, dtype=np.float64, order="C").reshape(-1, D)
    w = np.ascontiguousarray(w, dtype=np.float64)
    off = _c(cell_off, np.int64)
    n_cells = len(off) - 1
    st = np.zeros(n_cells, np.int32)
    rc = lib().orc_project(_p(v), _p(w), _p(off), _p(_c(moments, np.float64)), n_cells, D, int(tensor), _p(st))
    if rc != 0:
        raise ValueError("orc_project rejected its arguments")
    return v, st


def targets_from_moments(moments, D):
    """Reconstruction targets (W, P, E = tr(S)/2) from the compress moments record."""
    mom = np.asarray(moments)
    W = mom[:, 0]
    P = mom[:, 1:1 + D]
    diag = [1 + D + i * D - i * (i - 1) // 2 for i in range(D)]
    E = 0.5 * sum(mom[:, j] for j in diag)
    return np.concatenate([W[:, None], P, E[:, None]], axis=1)


# ---------------------------------------------------------------- warm start
NF, NH, NO = 105, 256, 160


def features(v, alpha, cell_off):
    """105 features and the whitening frame (m, L_C packed lower) per 3V cell."""
    v = _c(v, np.float64)
    off = _c(cell_off, np.int64)
    n_cells = len(off) - 1
    f = np.zeros((n_cells, NF))
    fr = np.zeros((n_cells, 9))
    lib().orc_features(_p(v), _p(_c(alpha, np.float64)), _p(off), n_cells, _p(f), _p(fr))
    return f, fr


def mlp_forward(X, params, bf16=False):
    X = _c(X, np.float64)
    B = X.shape[0]
    W1, b1, W2, b2, W3, b3 = [_c(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    H1 = np.zeros((B, NH))
    H2 = np.zeros((B, NH))
    Y = np.zeros((B, NO))
    lib().orc_mlp_forward(_p(X), B, _p(W1), _p(b1), _p(W2), _p(b2), _p(W3), _p(b3), int(bf16), _p(H1), _p(H2),
                          _p(Y))
    return H1, H2, Y


def mlp_loss_backward(X, params, targets, lam=1.0, bf16=False):
    """Loss (mean over rows) and gradients {W1, b1, ..., b3, dY}."""
    X = _c(X, np.float64)
    B = X.shape[0]
    Wn = [_c(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    g = {k: np.zeros_like(w) for k, w in zip(("W1", "b1", "W2", "b2", "W3", "b3"), Wn)}
    g["dY"] = np.zeros((B, NO))
    Tg = _c(targets, np.float64)
    L = lib().orc_mlp_loss_backward(_p(X), B, *[_p(w) for w in Wn], _p(Tg), float(lam), int(bf16),
                                    _p(g["W1"]), _p(g["b1"]), _p(g["W2"]), _p(g["b2"]), _p(g["W3"]), _p(g["b3"]),
                                    _p(g["dY"]))
    return L, g


def warm_decode(Y, frame, cell_off, kmax):
    Y = _c(Y, np.float64)
    fr = _c(frame, np.float64)
    off = _c(cell_off, np.int64)
    n_cells = len(off) - 1
    K = np.zeros(n_cells, np.int32)
    w = np.zeros((n_cells, kmax))
    mu = np.zeros((n_cells, kmax, 3))
    S = np.zeros((n_cells, kmax, 6))
    lib().orc_warm_decode(_p(Y), _p(fr), _p(off), n_cells, kmax, _p(K), _p(w), _p(mu), _p(S))
    return {"K": K, "omega": w, "mu": mu, "sigma": S}


def warm_targets(mix, frame):
    K = _c(mix["K"], np.int32)
    w = _c(mix["omega"], np.float64)
    kmax = w.shape[1]
    fr = _c(frame, np.float64)
    n_cells = len(K)
    Tg = np.zeros((n_cells, NO))
    lib().orc_warm_targets(_p(K), _p(w), _p(_c(mix["mu"], np.float64)), _p(_c(mix["sigma"], np.float64)), _p(fr),
                           n_cells, kmax, _p(Tg))
    return Tg
