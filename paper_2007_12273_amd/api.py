"""Python binding of libgmcr: argument marshalling only.

Tensors must already live on the GPU (torch, ROCm build).  Every step of
the computation runs in the HIP kernels behind the C ABI; this module only
allocates outputs, packs pointers and passes torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import _lib
from ._lib import GmInit, GmMix, GmOpts, check


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def ntri(D):
    return D * (D + 1) // 2


def _need(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def make_opts(D, kmax, n_min=10, max_sweeps=1000, tol=1e-7, seed=0, fp64=False, outer_k=False):
    o = GmOpts()
    _lib.load().gm_opts_default(ctypes.byref(o), D, kmax)
    o.n_min = n_min
    o.max_sweeps = max_sweeps
    o.tol_rel = tol
    o.seed = seed
    o.estep_fp64 = 1 if fp64 else 0
    o.outer_k = 1 if outer_k else 0
    return o


class MixtureBuffers:
    """Output record of gm_compress for n_cells cells (caller-owned memory)."""

    def __init__(self, n_cells, D, kmax, device):
        f64 = dict(dtype=torch.float64, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.D, self.kmax, self.n_cells = D, kmax, n_cells
        self.K = torch.zeros(n_cells, **i32)
        self.omega = torch.zeros(n_cells, kmax, **f64)
        self.mu = torch.zeros(n_cells, kmax, D, **f64)
        self.sigma = torch.zeros(n_cells, kmax, ntri(D), **f64)
        self.moments = torch.zeros(n_cells, 1 + D + ntri(D), **f64)
        self.L_pen = torch.zeros(n_cells, **f64)
        self.L_final = torch.zeros(n_cells, **f64)
        self.sweeps = torch.zeros(n_cells, **i32)
        self.status = torch.zeros(n_cells, **i32)
        self.visits = torch.zeros(n_cells, dtype=torch.int64, device=device)

    def struct(self):
        m = GmMix()
        for name in ("K", "omega", "mu", "sigma", "moments", "L_pen", "L_final", "sweeps", "status", "visits"):
            setattr(m, name, getattr(self, name).data_ptr())
        return m

    def as_dict(self):
        return {k: getattr(self, k) for k in ("K", "omega", "mu", "sigma", "moments", "L_pen", "L_final", "sweeps",
                                              "status", "visits")}


class Compressor:
    """Reusable compress call for a fixed (n_cells, D, kmax): owns the output
    record and the workspace so that repeated calls allocate nothing."""

    def __init__(self, n_cells, D, kmax, device="cuda", **opt):
        self.opts = make_opts(D, kmax, **opt)
        self.out = MixtureBuffers(n_cells, D, kmax, device)
        L = _lib.load()
        nbytes = L.gm_compress_workspace(n_cells, ctypes.byref(self.opts))
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        self.n_cells = n_cells
        self._mix = self.out.struct()

    def __call__(self, v, alpha, cell_off, fixed_sweeps=None, init=None, stream=None):
        D = self.opts.D
        _need(v, torch.float64, "v")
        _need(alpha, torch.float64, "alpha")
        _need(cell_off, torch.int64, "cell_off")
        if cell_off.numel() != self.n_cells + 1:
            raise ValueError("cell_off must have n_cells + 1 entries")
        if v.numel() != alpha.numel() * D:
            raise ValueError("v must be [n, D] with n = len(alpha)")
        fs = None
        if fixed_sweeps is not None:
            _need(fixed_sweeps, torch.int32, "fixed_sweeps")
            fs = _ptr(fixed_sweeps)
        ini = None
        if init is not None:
            ini = GmInit()
            for name in ("K", "omega", "mu", "sigma"):
                t = init[name]
                _need(t, torch.int32 if name == "K" else torch.float64, "init." + name)
                setattr(ini, name, t.data_ptr())
            ini = ctypes.byref(ini)
        rc = _lib.load().gm_compress(_ptr(v), _ptr(alpha), _ptr(cell_off), self.n_cells, ctypes.byref(self.opts), fs,
                                     ini, ctypes.byref(self._mix), _ptr(self.ws), self.ws.numel(), _stream(stream))
        check(rc, "gm_compress")
        return self.out

    def autotune(self, v, alpha, cell_off, init=None, stream=None):
        """Tune the EM launch plan on this batch (gm_autotune); returns the
        report as a dict and leaves a complete result in self.out."""
        _need(v, torch.float64, "v")
        _need(alpha, torch.float64, "alpha")
        _need(cell_off, torch.int64, "cell_off")
        if cell_off.numel() != self.n_cells + 1:
            raise ValueError("cell_off must have n_cells + 1 entries")
        ini = None
        if init is not None:
            ini = GmInit()
            for name in ("K", "omega", "mu", "sigma"):
                t = init[name]
                _need(t, torch.int32 if name == "K" else torch.float64, "init." + name)
                setattr(ini, name, t.data_ptr())
            ini = ctypes.byref(ini)
        rep = (ctypes.c_double * _lib.GM_TUNE_REPORT_LEN)()
        rc = _lib.load().gm_autotune(_ptr(v), _ptr(alpha), _ptr(cell_off), self.n_cells, ctypes.byref(self.opts), ini,
                                     ctypes.byref(self._mix), _ptr(self.ws), self.ws.numel(), _stream(stream), rep,
                                     _lib.GM_TUNE_REPORT_LEN)
        check(rc, "gm_autotune")
        r = list(rep)
        nb = 12
        return {"builtin_em_ms": r[0], "tuned_em_ms": r[1], "bucket_ms": r[2:2 + nb],
                "variant": [int(x) for x in r[2 + nb:2 + 2 * nb]], "lane": [int(x) for x in r[2 + 2 * nb:2 + 3 * nb]]}


class WarmCompressor:
    """Reusable gm_compress_warm call (learned warm start and compress in
    one library call) for a fixed (n_cells, kmax) and model: owns the output
    record and the workspace."""

    def __init__(self, n_cells, model, device="cuda", **opt):
        self.opts = make_opts(3, model.kmax, **opt)
        self.out = MixtureBuffers(n_cells, 3, model.kmax, device)
        L = _lib.load()
        nbytes = L.gm_compress_warm_workspace(n_cells, ctypes.byref(self.opts))
        if nbytes == 0:
            raise ValueError("invalid options")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.n_cells, self.model = n_cells, model
        self._mix = self.out.struct()

    def __call__(self, v, alpha, cell_off, stream=None):
        _need(v, torch.float64, "v")
        _need(alpha, torch.float64, "alpha")
        _need(cell_off, torch.int64, "cell_off")
        if cell_off.numel() != self.n_cells + 1:
            raise ValueError("cell_off must have n_cells + 1 entries")
        if v.numel() != alpha.numel() * 3:
            raise ValueError("v must be [n, 3] with n = len(alpha)")
        rc = _lib.load().gm_compress_warm(_ptr(v), _ptr(alpha), _ptr(cell_off), self.n_cells, ctypes.byref(self.opts),
                                          self.model._h, ctypes.byref(self._mix), _ptr(self.ws), self.ws.numel(),
                                          _stream(stream))
        check(rc, "gm_compress_warm")
        return self.out


class StandardEM:
    """Reusable standard-EM call (gm_compress_standard) for a fixed batch
    shape: owns the output record, the diagnostics and the workspace."""

    def __init__(self, n_cells, n_tot, D, kmax, device="cuda", trace=False, **opt):
        self.opts = make_opts(D, kmax, **opt)
        self.out = MixtureBuffers(n_cells, D, kmax, device)
        self.n_cells, self.n_tot = n_cells, n_tot
        L = _lib.load()
        nbytes = L.gm_compress_standard_workspace(n_cells, n_tot, ctypes.byref(self.opts))
        if nbytes == 0:
            raise ValueError("invalid options")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.resets = torch.zeros(n_cells, dtype=torch.int32, device=device)
        self.kmeans_passes = torch.zeros(n_cells, dtype=torch.int32, device=device)
        self.ll_trace = (torch.full((n_cells, self.opts.max_sweeps), float("nan"), dtype=torch.float64,
                                    device=device) if trace else None)
        self._mix = self.out.struct()

    def __call__(self, v, alpha, cell_off, K, kmeans=False, aa_memory=0, stream=None):
        _need(v, torch.float64, "v")
        _need(alpha, torch.float64, "alpha")
        _need(cell_off, torch.int64, "cell_off")
        if cell_off.numel() != self.n_cells + 1 or alpha.numel() != self.n_tot:
            raise ValueError("batch does not match the shape this call was made for")
        rc = _lib.load().gm_compress_standard(_ptr(v), _ptr(alpha), _ptr(cell_off), self.n_cells, self.n_tot,
                                              ctypes.byref(self.opts), int(K), 1 if kmeans else 0, int(aa_memory),
                                              ctypes.byref(self._mix), _ptr(self.resets),
                                              _ptr(self.kmeans_passes), _ptr(self.ll_trace), _ptr(self.ws),
                                              self.ws.numel(), _stream(stream))
        check(rc, "gm_compress_standard")
        return self.out


def compress(v, alpha, cell_off, kmax, n_min=10, max_sweeps=1000, tol=1e-7, seed=0, fp64=False, fixed_sweeps=None,
             init=None, stream=None, outer_k=False):
    """Adaptive EM-GM compress of every cell.  Returns a dict of GPU tensors
    (K, omega, mu, sigma, moments, L_pen, L_final, sweeps, status, visits).
    outer_k: outer search over K (gm_opts.outer_k)."""
    D = 1 if v.dim() == 1 else v.shape[1]
    n_cells = cell_off.numel() - 1
    c = Compressor(n_cells, D, kmax, device=v.device, n_min=n_min, max_sweeps=max_sweeps, tol=tol, seed=seed,
                   fp64=fp64, outer_k=outer_k)
    return c(v.contiguous(), alpha, cell_off, fixed_sweeps=fixed_sweeps, init=init, stream=stream).as_dict()


def compress_noalloc(v, alpha, cell_off, out, opts, fixed_sweeps=None, init=None, stream=None):
    """gm_compress_noalloc: the compress of `compress` into the caller's
    MixtureBuffers `out` with the library's fixed scratch instead of a
    workspace (at most GM_NOALLOC_MAX_CELLS cells).  `opts` from make_opts.
    Allocates nothing on the device."""
    _need(v, torch.float64, "v")
    _need(alpha, torch.float64, "alpha")
    _need(cell_off, torch.int64, "cell_off")
    n_cells = cell_off.numel() - 1
    if n_cells != out.n_cells or out.D != opts.D or out.kmax != opts.kmax:
        raise ValueError("output buffers do not match the batch and options")
    if v.numel() != alpha.numel() * opts.D:
        raise ValueError("v must be [n, D] with n = len(alpha)")
    fs = None
    if fixed_sweeps is not None:
        _need(fixed_sweeps, torch.int32, "fixed_sweeps")
        fs = _ptr(fixed_sweeps)
    ini = None
    if init is not None:
        ini = GmInit()
        for name in ("K", "omega", "mu", "sigma"):
            t = init[name]
            _need(t, torch.int32 if name == "K" else torch.float64, "init." + name)
            setattr(ini, name, t.data_ptr())
        ini = ctypes.byref(ini)
    mix = out.struct()
    rc = _lib.load().gm_compress_noalloc(_ptr(v), _ptr(alpha), _ptr(cell_off), n_cells, ctypes.byref(opts), fs, ini,
                                         ctypes.byref(mix), _stream(stream))
    check(rc, "gm_compress_noalloc")
    return out


class Reconstructor:
    """Reusable reconstruct call: owns the output particle arrays."""

    def __init__(self, out_off, D, dx, device="cuda", projection="scalar"):
        if projection not in ("scalar", "tensor"):
            raise ValueError("projection must be 'scalar' (Lemons) or 'tensor' (full second moment)")
        self.projection = projection
        self.D, self.dx = D, dx
        self.out_off = out_off
        n = int(out_off[-1].item())
        self.n_cells = out_off.numel() - 1
        f64 = dict(dtype=torch.float64, device=device)
        self.v = torch.empty(n, D, **f64)
        self.w = torch.empty(n, **f64)
        self.x = torch.empty(n, dx, **f64) if dx > 0 else None
        self.status = torch.empty(self.n_cells, dtype=torch.int32, device=device)

    def __call__(self, K, omega, mu, sigma, target, seed, stream=None):
        _need(K, torch.int32, "K")
        for t, name in ((omega, "omega"), (mu, "mu"), (sigma, "sigma"), (target, "target")):
            _need(t, torch.float64, name)
        _need(self.out_off, torch.int64, "out_off")
        kmax = omega.shape[-1]
        if K.numel() != self.n_cells or target.numel() != self.n_cells * (1 + self.D + ntri(self.D)):
            raise ValueError("mixture / target arrays do not match out_off")
        L = _lib.load()
        fn = L.gm_reconstruct_tensor if self.projection == "tensor" else L.gm_reconstruct
        rc = fn(_ptr(K), _ptr(omega), _ptr(mu), _ptr(sigma), kmax, _ptr(self.out_off), _ptr(target), self.n_cells,
                self.D, self.dx, seed, _ptr(self.v), _ptr(self.w), _ptr(self.x), _ptr(self.status), None, 0,
                _stream(stream))
        check(rc, "gm_reconstruct_tensor" if self.projection == "tensor" else "gm_reconstruct")
        return {"v": self.v, "w": self.w, "x": self.x, "status": self.status}


def reconstruct(K, omega, mu, sigma, out_off, target, D, dx, seed, stream=None, projection="scalar"):
    r = Reconstructor(out_off, D, dx, device=omega.device, projection=projection)
    return r(K, omega, mu, sigma, target, seed, stream=stream)


def project(v, w, cell_off, moments, tensor=False, out=None, stream=None):
    """Projection of given particles (v [n, D], w [n]) towards each cell's
    moments record, with the mass N' = sum w (gm_project).  Returns
    (v', status); out may be v (in place)."""
    _need(v, torch.float64, "v")
    _need(w, torch.float64, "w")
    _need(cell_off, torch.int64, "cell_off")
    _need(moments, torch.float64, "moments")
    D = v.shape[1]
    n_cells = cell_off.numel() - 1
    if w.numel() != v.shape[0] or moments.numel() != n_cells * (1 + D + ntri(D)):
        raise ValueError("v, w, moments do not match cell_off")
    out = out if out is not None else torch.empty_like(v)
    _need(out, torch.float64, "out")
    status = torch.empty(n_cells, dtype=torch.int32, device=v.device)
    check(_lib.load().gm_project(_ptr(v), _ptr(w), _ptr(cell_off), _ptr(moments), n_cells, D, 1 if tensor else 0,
                                 _ptr(out), _ptr(status), _stream(stream)), "gm_project")
    return out, status


class GaussLaw:
    """Gauss'-law weight correction on a periodic mesh (dx = 1: n_cells in a
    row; dx = 2: nx * (n_cells / nx)); owns the solver workspace."""

    def __init__(self, n_cells, dx, nx=None, device="cuda"):
        self.n_cells, self.dx = n_cells, dx
        self.nx = nx if nx is not None else n_cells
        nb = _lib.load().gm_gauss_workspace(n_cells, dx)
        if nb == 0:
            raise ValueError("bad mesh: n_cells=%d dx=%d" % (n_cells, dx))
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)

    def _check(self, x, w, cell_off):
        _need(x, torch.float64, "x")
        _need(w, torch.float64, "w")
        _need(cell_off, torch.int64, "cell_off")
        if cell_off.numel() != self.n_cells + 1 or x.numel() != w.numel() * self.dx:
            raise ValueError("x, w do not match the mesh")

    def deposit(self, x, w, cell_off, out=None, stream=None):
        """Charge D_i = sum_p w_p S2(X_i - X_p) on every mesh cell."""
        self._check(x, w, cell_off)
        out = out if out is not None else torch.empty(self.n_cells, dtype=torch.float64, device=w.device)
        _need(out, torch.float64, "out")
        check(_lib.load().gm_deposit(_ptr(x), _ptr(w), _ptr(cell_off), self.n_cells, self.dx, self.nx, _ptr(out),
                                     _ptr(self.ws), self.ws.numel(), _stream(stream)), "gm_deposit")
        return out

    def correct(self, x, w, cell_off, target, tol=1e-13, max_iter=200, stream=None):
        """Correct w in place so that deposit(x, w) = target; returns
        (iterations, relative residual).  Raises if the solve stalls."""
        self._check(x, w, cell_off)
        _need(target, torch.float64, "target")
        if target.numel() != self.n_cells:
            raise ValueError("target must hold one value per mesh cell")
        it, res = ctypes.c_int32(0), ctypes.c_double(0.0)
        rc = _lib.load().gm_gauss_correct(_ptr(x), _ptr(w), _ptr(cell_off), self.n_cells, self.dx, self.nx,
                                          _ptr(target), tol, max_iter, _ptr(self.ws), self.ws.numel(), _stream(stream),
                                          ctypes.byref(it), ctypes.byref(res))
        check(rc, "gm_gauss_correct")
        return it.value, res.value


def autotune_set(D, kmax, variant, lane=None, fp64=False, warm=False):
    """Install an EM launch plan by hand (codes as in the autotune report)."""
    va = (ctypes.c_int32 * 12)(*[int(x) for x in variant])
    la = (ctypes.c_int32 * 12)(*[int(x) for x in lane]) if lane is not None else None
    check(_lib.load().gm_autotune_set(D, kmax, 1 if fp64 else 0, 1 if warm else 0, va, la), "gm_autotune_set")


def autotune_reset():
    """Forget every tuned EM launch plan."""
    check(_lib.load().gm_autotune_reset(), "gm_autotune_reset")


def autotune_get(D, kmax, fp64=False, warm=False):
    """The EM launch plan gm_compress uses for (D, kmax class, fp64, warm) on
    the current device: dict of variant codes, lanes and launch order per
    bucket, and whether it is a tuned (or hand-set, or loaded) plan."""
    va, la, oa = (ctypes.c_int32 * 12)(), (ctypes.c_int32 * 12)(), (ctypes.c_int32 * 12)()
    rc = _lib.load().gm_autotune_get(D, kmax, 1 if fp64 else 0, 1 if warm else 0, va, la, oa)
    check(min(rc, 0), "gm_autotune_get")
    return {"variant": list(va), "lane": list(la), "order": list(oa), "tuned": rc == 1}


def autotune_save(path):
    """Write the current device's tuned EM launch plans to a plan file (lines
    of other devices in an existing file are kept)."""
    check(_lib.load().gm_autotune_save(os.fsencode(path)), "gm_autotune_save")


def autotune_load(path):
    """Install the plans of a plan file that were tuned on a device like the
    current one (same architecture and CU count); returns how many."""
    rc = _lib.load().gm_autotune_load(os.fsencode(path))
    check(min(rc, 0), "gm_autotune_load")
    return rc


def profile_enable(on=True):
    _lib.load().gm_profile_enable(1 if on else 0)


def profile_read():
    """Durations (ms) of the last compress phases and reconstruct:
    {'plan', 'em', 'finish', 'reconstruct'} (waits for the recorded events)."""
    buf = (ctypes.c_double * 4)()
    check(_lib.load().gm_profile_read(buf, 4), "gm_profile_read")
    return dict(zip(("plan", "em", "finish", "reconstruct"), list(buf)))


# ---------------------------------------------------------------------------
# learned warm start
# ---------------------------------------------------------------------------
NFEAT_ROW, NOUT = 128, 160
PARAM_SHAPES = (("W1", (128, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)), ("W3", (256, 160)),
                ("b3", (160,)))


def warm_features(v, alpha, cell_off, feats=None, frame=None, stream=None):
    """Features [n_cells, 128] (int16 tensor holding BF16 bit patterns) and
    frames [n_cells, 9] FP64 of 3V cells (into feats / frame when given)."""
    _need(v, torch.float64, "v")
    _need(alpha, torch.float64, "alpha")
    _need(cell_off, torch.int64, "cell_off")
    n_cells = cell_off.numel() - 1
    if feats is None:
        feats = torch.empty(n_cells, NFEAT_ROW, dtype=torch.int16, device=v.device)
    if frame is None:
        frame = torch.empty(n_cells, 9, dtype=torch.float64, device=v.device)
    _need(feats, torch.int16, "feats")
    _need(frame, torch.float64, "frame")
    if feats.shape != (n_cells, NFEAT_ROW) or frame.shape != (n_cells, 9):
        raise ValueError("feats must be [n_cells, 128] and frame [n_cells, 9]")
    rc = _lib.load().gm_warm_features(_ptr(v), _ptr(alpha), _ptr(cell_off), n_cells, 3, _ptr(feats), _ptr(frame),
                                      _stream(stream))
    check(rc, "gm_warm_features")
    return feats, frame


def warm_targets(mix, frame, stream=None):
    """Training targets [n_cells, 160] FP32 from a compress record."""
    K, omega, mu, sigma = mix["K"], mix["omega"], mix["mu"], mix["sigma"]
    _need(K, torch.int32, "K")
    for t, name in ((omega, "omega"), (mu, "mu"), (sigma, "sigma"), (frame, "frame")):
        _need(t, torch.float64, name)
    n_cells, kmax = omega.shape
    T = torch.empty(n_cells, NOUT, dtype=torch.float32, device=omega.device)
    rc = _lib.load().gm_warm_targets(_ptr(K), _ptr(omega), _ptr(mu), _ptr(sigma), kmax, _ptr(frame), n_cells,
                                     _ptr(T), _stream(stream))
    check(rc, "gm_warm_targets")
    return T


def warm_decode(Y, frame, cell_off, kmax, out=None, stream=None):
    """Initial mixtures (gm_init layout) from network outputs."""
    _need(Y, torch.float32, "Y")
    _need(frame, torch.float64, "frame")
    _need(cell_off, torch.int64, "cell_off")
    n_cells = cell_off.numel() - 1
    if Y.shape != (n_cells, NOUT) or frame.shape != (n_cells, 9):
        raise ValueError("Y must be [n_cells, 160] and frame [n_cells, 9]")
    dev = Y.device
    if out is None:
        out = {"K": torch.empty(n_cells, dtype=torch.int32, device=dev),
               "omega": torch.empty(n_cells, kmax, dtype=torch.float64, device=dev),
               "mu": torch.empty(n_cells, kmax, 3, dtype=torch.float64, device=dev),
               "sigma": torch.empty(n_cells, kmax, 6, dtype=torch.float64, device=dev)}
    rc = _lib.load().gm_warm_decode(_ptr(Y), _ptr(frame), _ptr(cell_off), n_cells, kmax, _ptr(out["K"]),
                                    _ptr(out["omega"]), _ptr(out["mu"]), _ptr(out["sigma"]), _stream(stream))
    check(rc, "gm_warm_decode")
    return out


class WarmStart:
    """Handle of a gm_warm model (the perceptron and its training state)."""

    def __init__(self, kmax, batch=1024, seed=0, device="cuda", path=None):
        """A fresh model (seeded weights), or, with `path`, the model that
        gm_warm_save wrote there (gm_warm_load; kmax is taken from the file)."""
        L = _lib.load()
        self.batch, self.device = batch, torch.device(device)
        self.n_param = int(L.gm_warm_param_count())
        h = ctypes.c_void_p()
        if path is None:
            check(L.gm_warm_create(ctypes.byref(h), 3, kmax, batch, seed, _stream(None)), "gm_warm_create")
            self.kmax = kmax
        else:
            check(L.gm_warm_load(ctypes.byref(h), os.fsencode(path), batch, _stream(None)), "gm_warm_load")
            with open(path, "rb") as f:
                self.kmax = int.from_bytes(f.read(16)[12:16], "little", signed=True)
        self._h = h
        self._ws = None

    @classmethod
    def load(cls, path, batch=1024, device="cuda"):
        return cls(None, batch=batch, device=device, path=path)

    def save(self, path):
        """Write the parameters to `path` (gm_warm_save)."""
        check(_lib.load().gm_warm_save(self._h, os.fsencode(path)), "gm_warm_save")

    def close(self):
        if self._h:
            _lib.load().gm_warm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        """Parameters as a flat float32 numpy array (host copy)."""
        import numpy as np
        buf = np.empty(self.n_param, dtype=np.float32)
        check(_lib.load().gm_warm_get_params(self._h, buf.ctypes.data), "gm_warm_get_params")
        return buf

    def set_params(self, flat):
        import numpy as np
        buf = np.ascontiguousarray(flat, dtype=np.float32)
        if buf.size != self.n_param:
            raise ValueError("expected %d parameters" % self.n_param)
        check(_lib.load().gm_warm_set_params(self._h, buf.ctypes.data), "gm_warm_set_params")

    def gradients(self):
        import numpy as np
        buf = np.empty(self.n_param, dtype=np.float32)
        check(_lib.load().gm_warm_gradients(self._h, buf.ctypes.data), "gm_warm_gradients")
        return buf

    def forward(self, feats, Y=None, stream=None):
        _need(feats, torch.int16, "feats")
        n = feats.shape[0]
        if feats.shape[1] != NFEAT_ROW:
            raise ValueError("features must be [n, 128]")
        if Y is not None:
            _need(Y, torch.float32, "Y")
            if Y.shape != (n, NOUT):
                raise ValueError("Y must be [n, 160]")
        L = _lib.load()
        self.forward_workspace(n)
        if Y is None:
            Y = torch.empty(n, NOUT, dtype=torch.float32, device=feats.device)
        check(L.gm_warm_forward(self._h, _ptr(feats), n, _ptr(Y), _ptr(self._ws), self._ws.numel(), _stream(stream)),
              "gm_warm_forward")
        return Y

    def train_step(self, feats, targets, idx, lr=1e-3, lam=1.0, loss_rows=None, stream=None):
        _need(feats, torch.int16, "feats")
        _need(targets, torch.float32, "targets")
        _need(idx, torch.int32, "idx")
        if idx.numel() != self.batch:
            raise ValueError("idx must hold exactly batch = %d rows" % self.batch)
        if feats.shape[1] != NFEAT_ROW or targets.shape != (feats.shape[0], NOUT):
            raise ValueError("features must be [n, 128] and targets [n, 160]")
        if loss_rows is not None:
            _need(loss_rows, torch.float32, "loss_rows")
            if loss_rows.numel() < self.batch:
                raise ValueError("loss_rows must hold batch = %d values" % self.batch)
        check(_lib.load().gm_warm_train_step(self._h, _ptr(feats), _ptr(targets), feats.shape[0], _ptr(idx), lr, lam,
                                             _ptr(loss_rows), _stream(stream)), "gm_warm_train_step")

    def train(self, feats, targets, epochs, lr=1e-3, lam=1.0, seed=0, stream=None):
        """gm_warm_train: `epochs` shuffled passes of Adam steps; returns the
        per-epoch mean row losses (a list of floats)."""
        import numpy as np
        _need(feats, torch.int16, "feats")
        _need(targets, torch.float32, "targets")
        if feats.shape[1] != NFEAT_ROW or targets.shape != (feats.shape[0], NOUT):
            raise ValueError("features must be [n, 128] and targets [n, 160]")
        L = _lib.load()
        n = feats.shape[0]
        need = int(L.gm_warm_train_workspace(n, self.batch))
        if need == 0:
            raise ValueError("need at least one full batch of %d rows, have %d" % (self.batch, n))
        ws = torch.empty(need, dtype=torch.uint8, device=feats.device)
        loss = np.zeros(epochs, dtype=np.float32)
        check(L.gm_warm_train(self._h, _ptr(feats), _ptr(targets), n, epochs, lr, lam, seed, _ptr(ws), need,
                              loss.ctypes.data, _stream(stream)), "gm_warm_train")
        return [float(x) for x in loss]

    def infer(self, feats, frame, cell_off, out, stream=None):
        """Network and decode fused (gm_warm_infer) into `out` (a gm_init
        dict of device tensors, kmax slots)."""
        _need(feats, torch.int16, "feats")
        n = feats.shape[0]
        if feats.shape[1] != NFEAT_ROW or frame.shape != (n, 9) or cell_off.numel() != n + 1:
            raise ValueError("features [n, 128], frame [n, 9] and cell_off [n + 1] expected")
        rc = _lib.load().gm_warm_infer(self._h, _ptr(feats), _ptr(frame), _ptr(cell_off), n, self.kmax,
                                       _ptr(out["K"]), _ptr(out["omega"]), _ptr(out["mu"]), _ptr(out["sigma"]),
                                       _stream(stream))
        check(rc, "gm_warm_infer")
        return out

    def initial_mixtures(self, v, alpha, cell_off, bufs=None, stream=None):
        """features -> network and decode (fused): a gm_init record for
        compress.  `bufs` (from init_buffers) makes repeated calls
        allocation-free."""
        n_cells = cell_off.numel() - 1
        if bufs is None:
            bufs = self.init_buffers(n_cells)
        warm_features(v, alpha, cell_off, feats=bufs["feats"], frame=bufs["frame"], stream=stream)
        return self.infer(bufs["feats"], bufs["frame"], cell_off, bufs["init"], stream=stream)

    def init_buffers(self, n_cells):
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.forward_workspace(n_cells)
        return {"feats": torch.empty(n_cells, NFEAT_ROW, dtype=torch.int16, device=dev),
                "frame": torch.empty(n_cells, 9, **f64),
                "Y": torch.empty(n_cells, NOUT, dtype=torch.float32, device=dev),
                "init": {"K": torch.empty(n_cells, dtype=torch.int32, device=dev),
                         "omega": torch.empty(n_cells, self.kmax, **f64),
                         "mu": torch.empty(n_cells, self.kmax, 3, **f64),
                         "sigma": torch.empty(n_cells, self.kmax, 6, **f64)}}

    def forward_workspace(self, n):
        need = int(_lib.load().gm_warm_forward_workspace(n))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)


def params_to_flat(P):
    """Oracle-layout parameters (W1 [105, 256], ...) -> flat float32 vector
    of the library's layout (W1 padded to 128 rows)."""
    import numpy as np
    parts = []
    for name, shape in PARAM_SHAPES:
        a = np.asarray(P[name], dtype=np.float64)
        if name == "W1":
            z = np.zeros(shape)
            z[:a.shape[0]] = a
            a = z
        parts.append(a.reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def flat_to_params(flat):
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = 1
        for s in shape:
            n *= s
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out
