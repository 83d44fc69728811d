"""Python binding of libgmcr: argument marshalling only.

Tensors must already live on the GPU (torch, ROCm build).  Every step of
the computation runs in the HIP kernels behind the C ABI; this module only
allocates outputs, packs pointers and passes torch's current stream.
"""
from __future__ import annotations

import ctypes

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


def make_opts(D, kmax, n_min=10, max_sweeps=1000, tol=1e-7, seed=0, fp64=False):
    o = GmOpts()
    _lib.load().gm_opts_default(ctypes.byref(o), D, kmax)
    o.n_min = n_min
    o.max_sweeps = max_sweeps
    o.tol_rel = tol
    o.seed = seed
    o.estep_fp64 = 1 if fp64 else 0
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


def compress(v, alpha, cell_off, kmax, n_min=10, max_sweeps=1000, tol=1e-7, seed=0, fp64=False, fixed_sweeps=None,
             init=None, stream=None):
    """Adaptive EM-GM compress of every cell.  Returns a dict of GPU tensors
    (K, omega, mu, sigma, moments, L_pen, L_final, sweeps, status, visits)."""
    D = 1 if v.dim() == 1 else v.shape[1]
    n_cells = cell_off.numel() - 1
    c = Compressor(n_cells, D, kmax, device=v.device, n_min=n_min, max_sweeps=max_sweeps, tol=tol, seed=seed,
                   fp64=fp64)
    return c(v.contiguous(), alpha, cell_off, fixed_sweeps=fixed_sweeps, init=init, stream=stream).as_dict()


class Reconstructor:
    """Reusable reconstruct call: owns the output particle arrays."""

    def __init__(self, out_off, D, dx, device="cuda"):
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
        rc = _lib.load().gm_reconstruct(_ptr(K), _ptr(omega), _ptr(mu), _ptr(sigma), kmax, _ptr(self.out_off),
                                        _ptr(target), self.n_cells, self.D, self.dx, seed, _ptr(self.v), _ptr(self.w),
                                        _ptr(self.x), _ptr(self.status), None, 0, _stream(stream))
        check(rc, "gm_reconstruct")
        return {"v": self.v, "w": self.w, "x": self.x, "status": self.status}


def reconstruct(K, omega, mu, sigma, out_off, target, D, dx, seed, stream=None):
    r = Reconstructor(out_off, D, dx, device=omega.device)
    return r(K, omega, mu, sigma, target, seed, stream=stream)


def profile_enable(on=True):
    _lib.load().gm_profile_enable(1 if on else 0)


def profile_read():
    """Durations (ms) of the last compress phases and reconstruct:
    {'plan', 'em', 'finish', 'reconstruct'} (waits for the recorded events)."""
    buf = (ctypes.c_double * 4)()
    check(_lib.load().gm_profile_read(buf, 4), "gm_profile_read")
    return dict(zip(("plan", "em", "finish", "reconstruct"), list(buf)))
