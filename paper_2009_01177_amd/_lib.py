"""ctypes loader for libtor_hip.so (argument marshalling only).

The library is built in-tree by paper_2009_01177_amd.build.  There is no
fallback: if the shared library is missing or fails to load, every call
raises, so no result can silently come from anywhere but the HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# The regular in-tree build.  TOR_LIBRARY, read when the library is first
# loaded, selects another build of it (the phase-clock build,
# libtor_hip_phase.so).
LIB_PATH = os.path.join(HERE, "libtor_hip.so")
TOR_NPHASE = 7

TOR_OK, TOR_EINVAL, TOR_ENOTPD, TOR_EHIP, TOR_ENOMEM, TOR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
TOR_EINPUT = -6
TOR_FP64, TOR_DD, TOR_QD, TOR_AUTO = 0, 1, 2, -1
TOR_ALGO_AUTO, TOR_ALGO_BORDER, TOR_ALGO_SCHUR = 0, 1, 2
TOR_NMAX = 50
TOR_FLAG_TIME_KERNEL = 1
TOR_FLAG_GRAPH = 2
TOR_FLAG_CHECK_INPUT = 4
TOR_NOALLOC_SCRATCH_BYTES = 256 << 20

# Every symbol include/tor.h declares.
EXPORTS = (
    "tor_version", "tor_strerror", "tor_init", "tor_shutdown", "tor_eval", "tor_eval_batched",
    "tor_mcmc", "tor_eval_part", "tor_combine_parts",
    "tor_debug_level_sums", "tor_debug_sampled_terms", "tor_last_kernel_ms",
    "tor_next_mask", "tor_kth_mask", "tor_plan_items",
    "tor_features", "tor_mlp_forward", "tor_mlp_grad", "tor_mlp_adam",
    "tor_selector_set", "tor_selector_get", "tor_selector_save", "tor_selector_load",
    "tor_fallback_bits", "tor_select_tiers", "tor_last_select_stats",
    "tor_autotune", "tor_autotune_save", "tor_autotune_load", "tor_workspace_bytes",
    "tor_batch_workspace_bytes", "tor_eval_noalloc", "tor_noalloc_nmax",
    "tor_mlp_grad_quantile", "tor_selector_label", "tor_selector_train", "tor_debug_level_sums_schur",
    "tor_debug_phase_clocks",
)

TOR_NFEAT = 20
TOR_MLP_PARAMS = 1761
TOR_TARGET_KAPPA, TOR_TARGET_ERR64 = 0, 1
TOR_LOSS_ASYM_SQUARED, TOR_LOSS_QUANTILE = 0, 1


class TorResultC(ctypes.Structure):
    _fields_ = [
        ("tor", ctypes.c_double * 4),
        ("abs_sum", ctypes.c_double * 2),
        ("err_bound", ctypes.c_double),
        ("tier_used", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class TorOptionsC(ctypes.Structure):
    _fields_ = [
        ("algo", ctypes.c_int32),
        ("split_depth", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("bottom_modes", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class TorSelectorC(ctypes.Structure):
    _fields_ = [
        ("theta", ctypes.c_double * TOR_MLP_PARAMS),
        ("mean", ctypes.c_double * TOR_NFEAT),
        ("std", ctypes.c_double * TOR_NFEAT),
        ("fmin", ctypes.c_double * TOR_NFEAT),
        ("fmax", ctypes.c_double * TOR_NFEAT),
        ("log10_c", ctypes.c_double * 3),
        ("slope", ctypes.c_double * 3),
        ("margin", ctypes.c_double),
        ("nmin", ctypes.c_int32),
        ("nmax", ctypes.c_int32),
        ("trained", ctypes.c_int32),
        ("target", ctypes.c_int32),
    ]


class TorTrainOptionsC(ctypes.Structure):
    _fields_ = [
        ("target", ctypes.c_int32),
        ("loss", ctypes.c_int32),
        ("epochs", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("lr", ctypes.c_double),
        ("beta1", ctypes.c_double),
        ("beta2", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("under", ctypes.c_double),
        ("over", ctypes.c_double),
        ("quantile", ctypes.c_double),
        ("slack", ctypes.c_double),
        ("margin", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class TorSelectStatsC(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("n_fp64", "n_dd", "n_qd", "n_fallback", "n_spot", "n_violations", "n_escalated",
                 "reserved")]


class TorError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _strerror(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


_lib = None


def _strerror(code: int) -> str:
    try:
        return lib().tor_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "error %d" % code


def _torch_gpu_first():
    """Initialise PyTorch's GPU runtime before the library's.  The library is
    linked against the system HIP runtime and PyTorch carries its own; when
    the library's initialises the device first, PyTorch then finds no GPU in
    that process.  Counting devices does not initialise anything, so a host
    without a GPU is left alone."""
    try:
        import torch
    except ImportError:  # pragma: no cover - torch is a dependency
        return
    if torch.cuda.device_count() > 0:
        torch.cuda.init()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("TOR_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is not built (run `python -m paper_2009_01177_amd.build` "
            "or __graft_entry__.build())")
    _torch_gpu_first()
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    dp = ctypes.POINTER(ctypes.c_double)
    L.tor_version.restype = ctypes.c_char_p
    L.tor_strerror.restype = ctypes.c_char_p
    L.tor_strerror.argtypes = [ctypes.c_int]
    L.tor_init.restype = ctypes.c_int
    L.tor_shutdown.restype = ctypes.c_int
    L.tor_eval.restype = ctypes.c_int
    L.tor_eval.argtypes = [vp, i32, i64, i32, ctypes.POINTER(TorOptionsC), vp,
                           ctypes.POINTER(TorResultC)]
    L.tor_eval_batched.restype = ctypes.c_int
    L.tor_eval_batched.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), i32,
                                   ctypes.POINTER(i32), ctypes.c_double, ctypes.POINTER(TorOptionsC),
                                   vp, vp]
    L.tor_eval_part.restype = ctypes.c_int
    L.tor_eval_part.argtypes = [vp, i32, i64, i32, ctypes.POINTER(TorOptionsC), vp, i32, i32,
                                ctypes.POINTER(TorResultC)]
    L.tor_combine_parts.restype = ctypes.c_int
    L.tor_combine_parts.argtypes = [i32, i32, ctypes.POINTER(TorResultC), i32, ctypes.POINTER(TorResultC)]
    L.tor_mcmc.restype = ctypes.c_int
    L.tor_mcmc.argtypes = [vp, i32, i64, i32, i32, i32, vp, vp, i32, ctypes.c_double,
                           ctypes.POINTER(TorOptionsC), vp, vp, vp]
    L.tor_debug_level_sums.restype = ctypes.c_int
    L.tor_debug_level_sums.argtypes = [vp, i32, i64, i32, vp, dp, ctypes.POINTER(TorResultC)]
    L.tor_debug_level_sums_schur.restype = ctypes.c_int
    L.tor_debug_level_sums_schur.argtypes = [vp, i32, i64, i32, vp, dp, ctypes.POINTER(TorResultC)]
    L.tor_debug_phase_clocks.restype = ctypes.c_int
    L.tor_debug_phase_clocks.argtypes = [i32, ctypes.POINTER(u64)]
    L.tor_debug_sampled_terms.restype = ctypes.c_int
    L.tor_debug_sampled_terms.argtypes = [vp, i32, i64, i32, vp, i64, vp, vp]
    L.tor_last_kernel_ms.restype = ctypes.c_double
    L.tor_last_kernel_ms.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    pd = ctypes.POINTER(ctypes.c_double)
    L.tor_features.restype = ctypes.c_int
    L.tor_features.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), i32, vp, vp]
    L.tor_mlp_forward.restype = ctypes.c_int
    L.tor_mlp_forward.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    L.tor_mlp_grad.restype = ctypes.c_int
    L.tor_mlp_grad.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    L.tor_mlp_grad_quantile.restype = ctypes.c_int
    L.tor_mlp_grad_quantile.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_double, vp, vp, vp]
    L.tor_selector_label.restype = ctypes.c_int
    L.tor_selector_label.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), i32, i32,
                                     vp, ctypes.POINTER(ctypes.c_double)]
    L.tor_selector_train.restype = ctypes.c_int
    L.tor_selector_train.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int32), i32, ctypes.POINTER(TorTrainOptionsC), vp,
                                     ctypes.POINTER(TorSelectorC), ctypes.POINTER(ctypes.c_double)]
    L.tor_mlp_adam.restype = ctypes.c_int
    L.tor_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, i32, vp]
    L.tor_selector_set.restype = ctypes.c_int
    L.tor_selector_set.argtypes = [ctypes.POINTER(TorSelectorC)]
    L.tor_selector_get.restype = ctypes.c_int
    L.tor_selector_get.argtypes = [ctypes.POINTER(TorSelectorC)]
    L.tor_selector_save.restype = ctypes.c_int
    L.tor_selector_save.argtypes = [ctypes.c_char_p]
    L.tor_selector_load.restype = ctypes.c_int
    L.tor_selector_load.argtypes = [ctypes.c_char_p]
    L.tor_fallback_bits.restype = ctypes.c_double
    L.tor_fallback_bits.argtypes = [pd, ctypes.c_double]
    L.tor_select_tiers.restype = ctypes.c_int
    L.tor_select_tiers.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), i32, ctypes.c_double, vp,
                                   ctypes.POINTER(i32), pd, ctypes.POINTER(i32)]
    L.tor_last_select_stats.restype = ctypes.c_int
    L.tor_last_select_stats.argtypes = [ctypes.POINTER(TorSelectStatsC)]
    L.tor_autotune.restype = ctypes.c_int
    L.tor_autotune.argtypes = [i32, i32, vp, ctypes.POINTER(i32), pd]
    L.tor_autotune_save.restype = ctypes.c_int
    L.tor_autotune_save.argtypes = [ctypes.c_char_p]
    L.tor_autotune_load.restype = ctypes.c_int
    L.tor_autotune_load.argtypes = [ctypes.c_char_p]
    L.tor_next_mask.restype = u64
    L.tor_next_mask.argtypes = [u64]
    L.tor_kth_mask.restype = u64
    L.tor_kth_mask.argtypes = [i32, i32, u64]
    L.tor_plan_items.restype = ctypes.c_int
    L.tor_plan_items.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.tor_workspace_bytes.restype = ctypes.c_int
    L.tor_workspace_bytes.argtypes = [i32, i32, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.tor_batch_workspace_bytes.restype = ctypes.c_int
    L.tor_batch_workspace_bytes.argtypes = [i32, i32, i32, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.tor_eval_noalloc.restype = ctypes.c_int
    L.tor_eval_noalloc.argtypes = [vp, i32, i64, i32, vp, vp]
    L.tor_noalloc_nmax.restype = i32
    L.tor_noalloc_nmax.argtypes = [i32]
    _lib = L
    return L


def check(code: int, what: str = "") -> int:
    if code != TOR_OK:
        raise TorError(code, what)
    return code
