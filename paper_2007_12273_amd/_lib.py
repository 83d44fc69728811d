"""ctypes view of libgmcr.so (the C ABI in include/gmcr.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation behind these bindings.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmcr.so")

GM_OK, GM_EINVAL, GM_EHIP, GM_ENOMEM, GM_ENOTIMPL, GM_ENOCONV, GM_EIO, GM_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7
GM_NOALLOC_MAX_CELLS = 65536
GM_TUNE_REPORT_LEN = 38

STATUS = {
    "SMALL_CELL_K1": 1 << 0, "K0_CAPPED": 1 << 1, "COV_FLOOR": 1 << 2, "MAXSWEEPS": 1 << 3,
    "NEAR_TIE": 1 << 4, "WARM_FALLBACK": 1 << 5, "NONFINITE_INPUT": 1 << 6,
    "LEMONS_SKIPPED": 1 << 7, "DEGENERATE": 1 << 8,
}

P = ctypes.c_void_p


class GmOpts(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32), ("kmax", ctypes.c_int32), ("n_min", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32), ("tol_rel", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("estep_fp64", ctypes.c_int32), ("outer_k", ctypes.c_int32),
    ]


class GmMix(ctypes.Structure):
    _fields_ = [(n, P) for n in ("K", "omega", "mu", "sigma", "moments", "L_pen", "L_final", "sweeps", "status",
                                 "visits")]


class GmInit(ctypes.Structure):
    _fields_ = [(n, P) for n in ("K", "omega", "mu", "sigma")]


EXPORTS = ("gm_opts_default", "gm_compress_workspace", "gm_compress", "gm_compress_noalloc", "gm_compress_warm",
           "gm_compress_warm_workspace", "gm_warm_model_kmax", "gm_warm_infer", "gm_autotune", "gm_autotune_set", "gm_autotune_reset",
           "gm_autotune_get", "gm_autotune_save", "gm_autotune_load",
           "gm_reconstruct_workspace", "gm_reconstruct_tensor", "gm_project", "gm_gauss_workspace", "gm_deposit",
           "gm_gauss_correct", "gm_compress_standard_workspace", "gm_compress_standard",
           "gm_reconstruct", "gm_warm_param_count", "gm_warm_create", "gm_warm_destroy", "gm_warm_get_params",
           "gm_warm_set_params", "gm_warm_gradients", "gm_warm_save", "gm_warm_load", "gm_warm_features", "gm_warm_forward_workspace",
           "gm_warm_forward", "gm_warm_decode", "gm_warm_targets", "gm_warm_train_step", "gm_warm_train_workspace",
           "gm_warm_train", "gm_profile_enable",
           "gm_profile_read", "gm_strerror", "gm_version")

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load libgmcr.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing("libgmcr.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    L.gm_opts_default.argtypes = [ctypes.POINTER(GmOpts), ctypes.c_int32, ctypes.c_int32]
    L.gm_opts_default.restype = None
    L.gm_compress_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(GmOpts)]
    L.gm_compress_workspace.restype = ctypes.c_size_t
    L.gm_compress.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(GmOpts), P, ctypes.POINTER(GmInit),
                              ctypes.POINTER(GmMix), P, ctypes.c_size_t, P]
    L.gm_compress.restype = ctypes.c_int
    L.gm_compress_noalloc.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(GmOpts), P, ctypes.POINTER(GmInit),
                                      ctypes.POINTER(GmMix), P]
    L.gm_compress_noalloc.restype = ctypes.c_int
    L.gm_compress_warm_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(GmOpts)]
    L.gm_compress_warm_workspace.restype = ctypes.c_size_t
    L.gm_compress_warm.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(GmOpts), P, ctypes.POINTER(GmMix), P,
                                   ctypes.c_size_t, P]
    L.gm_compress_warm.restype = ctypes.c_int
    L.gm_warm_infer.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, P, P, P]
    L.gm_warm_infer.restype = ctypes.c_int
    L.gm_warm_model_kmax.argtypes = [P]
    L.gm_warm_model_kmax.restype = ctypes.c_int
    L.gm_autotune.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(GmOpts), ctypes.POINTER(GmInit),
                              ctypes.POINTER(GmMix), P, ctypes.c_size_t, P, P, ctypes.c_int32]
    L.gm_autotune.restype = ctypes.c_int
    L.gm_autotune_set.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]
    L.gm_autotune_set.restype = ctypes.c_int
    L.gm_autotune_reset.argtypes = []
    L.gm_autotune_reset.restype = ctypes.c_int
    L.gm_autotune_get.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    L.gm_autotune_get.restype = ctypes.c_int
    L.gm_autotune_save.argtypes = [ctypes.c_char_p]
    L.gm_autotune_save.restype = ctypes.c_int
    L.gm_autotune_load.argtypes = [ctypes.c_char_p]
    L.gm_autotune_load.restype = ctypes.c_int
    L.gm_reconstruct_workspace.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.gm_reconstruct_workspace.restype = ctypes.c_size_t
    L.gm_reconstruct.argtypes = [P, P, P, P, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_uint64, P, P, P, P, P, ctypes.c_size_t, P]
    L.gm_reconstruct.restype = ctypes.c_int
    L.gm_reconstruct_tensor.argtypes = L.gm_reconstruct.argtypes
    L.gm_reconstruct_tensor.restype = ctypes.c_int
    L.gm_project.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P]
    L.gm_project.restype = ctypes.c_int
    L.gm_gauss_workspace.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.gm_gauss_workspace.restype = ctypes.c_size_t
    L.gm_deposit.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_size_t, P]
    L.gm_deposit.restype = ctypes.c_int
    L.gm_gauss_correct.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_double,
                                   ctypes.c_int32, P, ctypes.c_size_t, P, P, P]
    L.gm_gauss_correct.restype = ctypes.c_int
    L.gm_compress_standard_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, P]
    L.gm_compress_standard_workspace.restype = ctypes.c_size_t
    L.gm_compress_standard.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, P, P, P, P, P, ctypes.c_size_t, P]
    L.gm_compress_standard.restype = ctypes.c_int
    I32, I64, SZ, U64, F32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_float
    L.gm_warm_param_count.argtypes = []
    L.gm_warm_param_count.restype = SZ
    L.gm_warm_create.argtypes = [ctypes.POINTER(P), I32, I32, I32, U64, P]
    L.gm_warm_create.restype = ctypes.c_int
    L.gm_warm_destroy.argtypes = [P]
    L.gm_warm_destroy.restype = None
    for name in ("gm_warm_get_params", "gm_warm_set_params", "gm_warm_gradients"):
        getattr(L, name).argtypes = [P, P]
        getattr(L, name).restype = ctypes.c_int
    L.gm_warm_train_workspace.argtypes = [I64, I32]
    L.gm_warm_train_workspace.restype = SZ
    L.gm_warm_train.argtypes = [P, P, P, I64, I32, F32, F32, U64, P, SZ, P, P]
    L.gm_warm_train.restype = ctypes.c_int
    L.gm_warm_save.argtypes = [P, ctypes.c_char_p]
    L.gm_warm_save.restype = ctypes.c_int
    L.gm_warm_load.argtypes = [ctypes.POINTER(P), ctypes.c_char_p, I32, P]
    L.gm_warm_load.restype = ctypes.c_int
    L.gm_warm_features.argtypes = [P, P, P, I64, I32, P, P, P]
    L.gm_warm_features.restype = ctypes.c_int
    L.gm_warm_forward_workspace.argtypes = [I64]
    L.gm_warm_forward_workspace.restype = SZ
    L.gm_warm_forward.argtypes = [P, P, I64, P, P, SZ, P]
    L.gm_warm_forward.restype = ctypes.c_int
    L.gm_warm_decode.argtypes = [P, P, P, I64, I32, P, P, P, P, P]
    L.gm_warm_decode.restype = ctypes.c_int
    L.gm_warm_targets.argtypes = [P, P, P, P, I32, P, I64, P, P]
    L.gm_warm_targets.restype = ctypes.c_int
    L.gm_warm_train_step.argtypes = [P, P, P, I64, P, F32, F32, P, P]
    L.gm_warm_train_step.restype = ctypes.c_int
    L.gm_profile_enable.argtypes = [ctypes.c_int]
    L.gm_profile_enable.restype = None
    L.gm_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.gm_profile_read.restype = ctypes.c_int
    L.gm_strerror.argtypes = [ctypes.c_int]
    L.gm_strerror.restype = ctypes.c_char_p
    L.gm_version.argtypes = []
    L.gm_version.restype = ctypes.c_int
    _lib = L
    return L


def check(rc, what):
    if rc != GM_OK:
        msg = load().gm_strerror(rc).decode()
        raise RuntimeError("%s failed: %s (%d)" % (what, msg, rc))
