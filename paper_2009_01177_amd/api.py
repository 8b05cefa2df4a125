"""Python binding of the C ABI (include/tor.h), same names, argument
marshalling only.  PyTorch provides device memory and the current stream;
every step of the evaluation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

from . import _lib
from ._lib import TorError, check, lib

_TIERS = {"fp64": _lib.TOR_FP64, "dd": _lib.TOR_DD, "qd": _lib.TOR_QD, "auto": _lib.TOR_AUTO}
_ALGOS = {"auto": _lib.TOR_ALGO_AUTO, "border": _lib.TOR_ALGO_BORDER, "schur": _lib.TOR_ALGO_SCHUR}


def tier_id(tier) -> int:
    if isinstance(tier, str):
        return _TIERS[tier.lower()]
    return int(tier)


def algo_id(algo) -> int:
    if isinstance(algo, str):
        return _ALGOS[algo.lower()]
    return int(algo)


@dataclass
class TorResult:
    expansion: tuple          # Tor as (hi, lo, ...) non-overlapping doubles
    abs_sum: tuple            # S_abs as double-double
    err_bound: float
    tier_used: int
    status: int
    value: float = field(init=False)

    def __post_init__(self):
        finite = all(np.isfinite(self.expansion))
        self.value = float(sum(Fraction(x) for x in self.expansion)) if finite else float("nan")

    @property
    def exact(self) -> Fraction:
        """The returned expansion summed exactly."""
        return sum((Fraction(x) for x in self.expansion), Fraction(0))

    @property
    def abs_exact(self) -> Fraction:
        return sum((Fraction(x) for x in self.abs_sum), Fraction(0))

    @property
    def kappa(self) -> float:
        t = self.exact
        return float(self.abs_exact / abs(t)) if t != 0 else float("inf")


def _res(r: _lib.TorResultC) -> TorResult:
    return TorResult(tuple(r.tor), tuple(r.abs_sum), r.err_bound, r.tier_used, r.status)


def _torch():
    import torch
    return torch


def _device_o(O):
    """complex128 device tensor (contiguous rows) and n, ld."""
    torch = _torch()
    if isinstance(O, np.ndarray):
        O = torch.from_numpy(np.ascontiguousarray(O, dtype=np.complex128))
    if not isinstance(O, torch.Tensor):
        raise TypeError("O must be a numpy array or a torch tensor")
    if O.dtype != torch.complex128:
        O = O.to(torch.complex128)
    if not O.is_cuda:
        O = O.to("cuda")
    if O.dim() != 2 or O.shape[0] != O.shape[1] or O.shape[0] % 2:
        raise ValueError("O must be 2n x 2n")
    if O.stride(1) != 1:
        O = O.contiguous()
    n = O.shape[0] // 2
    ld = O.stride(0) if n > 0 else 0
    return O, n, max(ld, 2 * n)


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def tor_version() -> str:
    return lib().tor_version().decode()


def tor_init():
    check(lib().tor_init(), "tor_init")


def tor_shutdown():
    check(lib().tor_shutdown(), "tor_shutdown")


def tor_eval(O, tier="dd", algo="auto", split_depth: int = -1, grid: int = 0,
             stream=None, raise_on_error: bool = True, time_kernel: bool = False,
             bottom_modes: int = 0, check_input: bool = False) -> TorResult:
    """Tor(O) of one instance (synchronous); check_input: TOR_FLAG_CHECK_INPUT."""
    Od, n, ld = _device_o(O)
    flags = (_lib.TOR_FLAG_TIME_KERNEL if time_kernel else 0) | (_lib.TOR_FLAG_CHECK_INPUT if check_input else 0)
    opt = _lib.TorOptionsC(algo_id(algo), int(split_depth), int(grid), flags, int(bottom_modes))
    out = _lib.TorResultC()
    rc = lib().tor_eval(ctypes.c_void_p(Od.data_ptr()), n, ld, tier_id(tier), ctypes.byref(opt),
                        _stream_ptr(stream), ctypes.byref(out))
    if rc != _lib.TOR_OK and raise_on_error:
        raise TorError(rc, "tor_eval")
    return _res(out)


def tor_eval_part(O, part: int, nparts: int, tier="dd", stream=None, bottom_modes: int = 0,
                  raise_on_error: bool = True, check_input: bool = False) -> TorResult:
    """Share `part` of `nparts` of Tor(O) (include/tor.h, tor_eval_part)."""
    Od, n, ld = _device_o(O)
    opt = _lib.TorOptionsC(_lib.TOR_ALGO_AUTO, -1, 0, _lib.TOR_FLAG_CHECK_INPUT if check_input else 0,
                           int(bottom_modes))
    out = _lib.TorResultC()
    rc = lib().tor_eval_part(ctypes.c_void_p(Od.data_ptr()), n, ld, tier_id(tier), ctypes.byref(opt),
                             _stream_ptr(stream), int(part), int(nparts), ctypes.byref(out))
    if rc != _lib.TOR_OK and raise_on_error:
        raise TorError(rc, "tor_eval_part")
    return _res(out)


def tor_combine_parts(tier, n: int, parts) -> TorResult:
    """Tor from the TorResults of all parts, in part order (host only)."""
    arr = (_lib.TorResultC * max(len(parts), 1))()
    for i, r in enumerate(parts):
        arr[i].tor[:] = (list(r.expansion) + [0.0] * 4)[:4]
        arr[i].abs_sum[:] = list(r.abs_sum)[:2]
        arr[i].err_bound = r.err_bound
        arr[i].tier_used = r.tier_used
        arr[i].status = r.status
    out = _lib.TorResultC()
    check(lib().tor_combine_parts(tier_id(tier), int(n), arr, len(parts), ctypes.byref(out)),
          "tor_combine_parts")
    return _res(out)


class Batch:
    """A packed batch on the device: instance k's O (2n_k x 2n_k, leading
    dimension 2n_k) at offsets[k] complex elements into one buffer."""

    def __init__(self, Os, device="cuda"):
        torch = _torch()
        self.n = np.array([o.shape[0] // 2 for o in Os], dtype=np.int32)
        sizes = np.array([o.shape[0] * o.shape[0] for o in Os], dtype=np.int64)
        self.offsets = np.zeros(len(Os), dtype=np.int64)
        if len(Os):
            self.offsets[1:] = np.cumsum(sizes)[:-1]
        flat = np.concatenate([np.ascontiguousarray(o, dtype=np.complex128).ravel() for o in Os]) \
            if len(Os) else np.zeros(1, dtype=np.complex128)
        self.O = torch.from_numpy(flat).to(device)
        self.batch = len(Os)
        self.out = torch.zeros((max(self.batch, 1), 8), dtype=torch.float64, device=device)


def _results_from(buf):
    """Decode a (batch, 8) float64 view of tor_result_t records."""
    raw = np.ascontiguousarray(buf).view(np.uint8)
    res = []
    for i in range(buf.shape[0]):
        r = _lib.TorResultC.from_buffer_copy(raw[i].tobytes())
        res.append(_res(r))
    return res


def tor_eval_batched(batch: "Batch", tiers=None, tau: float = 1e-3, graph: bool = False,
                     stream=None, bottom_modes: int = 0, sync: bool = True, check_input: bool = False):
    """Torontonians of a packed batch; returns a list of TorResult when
    sync is True (else None: the results are in batch.out on the device)."""
    torch = _torch()
    B = batch.batch
    if tiers is None:
        tptr = None
    else:
        if isinstance(tiers, (str, int)):
            tiers = [tiers] * B
        t = np.ascontiguousarray([tier_id(x) for x in tiers], dtype=np.int32)
        tptr = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    flags = (_lib.TOR_FLAG_GRAPH if graph else 0) | (_lib.TOR_FLAG_CHECK_INPUT if check_input else 0)
    opt = _lib.TorOptionsC(_lib.TOR_ALGO_AUTO, -1, 0, flags, int(bottom_modes))
    rc = lib().tor_eval_batched(ctypes.c_void_p(batch.O.data_ptr()),
                                batch.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                batch.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), B, tptr,
                                float(tau), ctypes.byref(opt), _stream_ptr(stream),
                                ctypes.c_void_p(batch.out.data_ptr()))
    check(rc, "tor_eval_batched")
    if not sync:
        return None
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    return _results_from(batch.out[:B].cpu().numpy())


def tor_mcmc(O_full, proposals, uniforms, tier="dd", tau: float = 1e-3, stream=None,
             bottom_modes: int = 0):
    """Markov chains over N-click patterns (include/tor.h, tor_mcmc).

    O_full     2M x 2M complex O of the state (numpy or torch)
    proposals  steps x chains x N int32 candidate modes, rows ascending
    uniforms   steps x chains acceptance variates in [0, 1]
    Returns (state_step, cand): device tensors, int32 [steps, chains] and
    float64 [steps, chains, 8] holding one tor_result_t per candidate
    (results_of() decodes them).  Synchronous."""
    torch = _torch()
    Od, M, ld = _device_o(O_full)
    dev = Od.device
    P = torch.as_tensor(proposals)
    P = P.to(device=dev, dtype=torch.int32).contiguous()
    U = torch.as_tensor(uniforms).to(device=dev, dtype=torch.float64).contiguous()
    if P.dim() != 3 or U.dim() != 2 or tuple(P.shape[:2]) != tuple(U.shape):
        raise ValueError("proposals must be steps x chains x N and uniforms steps x chains")
    steps, chains, N = (int(x) for x in P.shape)
    cand = torch.zeros((steps, chains, 8), dtype=torch.float64, device=dev)
    state = torch.zeros((steps, chains), dtype=torch.int32, device=dev)
    opt = _lib.TorOptionsC(_lib.TOR_ALGO_AUTO, -1, 0, 0, int(bottom_modes))
    rc = lib().tor_mcmc(ctypes.c_void_p(Od.data_ptr()), M, ld, N, chains, steps,
                        ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(U.data_ptr()), tier_id(tier),
                        float(tau), ctypes.byref(opt), _stream_ptr(stream),
                        ctypes.c_void_p(cand.data_ptr()), ctypes.c_void_p(state.data_ptr()))
    check(rc, "tor_mcmc")
    return state, cand


def results_of(cand) -> list:
    """Decode tor_result_t records (a [..., 8] float64 tensor or array) into
    a flat list of TorResult."""
    if hasattr(cand, "cpu"):
        cand = cand.cpu().numpy()
    return _results_from(np.asarray(cand).reshape(-1, 8))


def tor_autotune(n: int, tier="dd", stream=None):
    """(best s_b, times in ms for s_b = 1..6, -1 where not run)."""
    best = ctypes.c_int32(0)
    ms = np.zeros(6, dtype=np.float64)
    check(lib().tor_autotune(int(n), tier_id(tier), _stream_ptr(stream), ctypes.byref(best),
                             ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tor_autotune")
    return int(best.value), ms


def tor_autotune_save(path: str):
    check(lib().tor_autotune_save(str(path).encode()), "tor_autotune_save")


def tor_autotune_load(path: str):
    check(lib().tor_autotune_load(str(path).encode()), "tor_autotune_load")


# ---- precision selector ----------------------------------------------------

def _dptr_t(t):
    return ctypes.c_void_p(t.data_ptr())


def tor_features(batch: "Batch", stream=None):
    """(B, TOR_NFEAT) float64 device tensor of the instances' selector features."""
    torch = _torch()
    f = torch.zeros((batch.batch, _lib.TOR_NFEAT), dtype=torch.float64, device=batch.O.device)
    rc = lib().tor_features(_dptr_t(batch.O),
                            batch.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            batch.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), batch.batch,
                            _stream_ptr(stream), _dptr_t(f))
    check(rc, "tor_features")
    return f


def tor_mlp_forward(theta, mean, std, X, stream=None):
    torch = _torch()
    Y = torch.zeros(X.shape[0], dtype=torch.float64, device=X.device)
    check(lib().tor_mlp_forward(_dptr_t(theta), _dptr_t(mean), _dptr_t(std), _dptr_t(X), X.shape[0],
                                _stream_ptr(stream), _dptr_t(Y)), "tor_mlp_forward")
    return Y


def tor_mlp_grad(theta, mean, std, X, y, under=4.0, over=1.0, stream=None):
    """(grad, loss) device tensors."""
    torch = _torch()
    grad = torch.zeros(_lib.TOR_MLP_PARAMS, dtype=torch.float64, device=X.device)
    loss = torch.zeros(1, dtype=torch.float64, device=X.device)
    check(lib().tor_mlp_grad(_dptr_t(theta), _dptr_t(mean), _dptr_t(std), _dptr_t(X), _dptr_t(y),
                             X.shape[0], float(under), float(over), _stream_ptr(stream), _dptr_t(grad),
                             _dptr_t(loss)), "tor_mlp_grad")
    return grad, loss


def tor_mlp_grad_quantile(theta, mean, std, X, y, q=0.9, stream=None):
    """(grad, loss) device tensors of the quantile loss at level q."""
    torch = _torch()
    grad = torch.zeros(_lib.TOR_MLP_PARAMS, dtype=torch.float64, device=X.device)
    loss = torch.zeros(1, dtype=torch.float64, device=X.device)
    check(lib().tor_mlp_grad_quantile(_dptr_t(theta), _dptr_t(mean), _dptr_t(std), _dptr_t(X), _dptr_t(y),
                                      X.shape[0], float(q), _stream_ptr(stream), _dptr_t(grad), _dptr_t(loss)),
          "tor_mlp_grad_quantile")
    return grad, loss


def tor_selector_label(batch: "Batch", ref_tier="qd", stream=None) -> np.ndarray:
    """(B, 4) host array of labels: log10 kappa and log10 of the FP64 and DD
    relative forward errors against the reference tier (include/tor.h)."""
    out = np.full((batch.batch, 4), np.nan, dtype=np.float64)
    check(lib().tor_selector_label(_dptr_t(batch.O), batch.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   batch.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), batch.batch,
                                   tier_id(ref_tier), _stream_ptr(stream),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tor_selector_label")
    return out


def train_options(target="err64", loss="quantile", epochs=400, batch_size=512, lr=3e-3, beta1=0.9,
                  beta2=0.999, eps=1e-8, under=4.0, over=1.0, quantile=0.9, slack=0.3, margin=0.0,
                  seed=0) -> "_lib.TorTrainOptionsC":
    o = _lib.TorTrainOptionsC()
    o.target = {"kappa": _lib.TOR_TARGET_KAPPA, "err64": _lib.TOR_TARGET_ERR64}[target]
    o.loss = {"asym_squared": _lib.TOR_LOSS_ASYM_SQUARED, "quantile": _lib.TOR_LOSS_QUANTILE}[loss]
    o.epochs, o.batch_size = int(epochs), int(batch_size)
    o.lr, o.beta1, o.beta2, o.eps = float(lr), float(beta1), float(beta2), float(eps)
    o.under, o.over, o.quantile = float(under), float(over), float(quantile)
    o.slack, o.margin, o.seed = float(slack), float(margin), int(seed)
    return o


def tor_selector_train(feats, labels, n, opt: "_lib.TorTrainOptionsC", stream=None):
    """Train and calibrate a selector (include/tor.h); returns (TorSelectorC,
    per-epoch mean losses).  feats (B, TOR_NFEAT), labels (B, 4), n (B,):
    host arrays; the selector is not installed."""
    X = np.ascontiguousarray(feats, dtype=np.float64)
    L = np.ascontiguousarray(labels, dtype=np.float64)
    nn = np.ascontiguousarray(n, dtype=np.int32)
    if X.ndim != 2 or X.shape[1] != _lib.TOR_NFEAT or L.shape != (X.shape[0], 4) or nn.shape != (X.shape[0],):
        raise ValueError("feats (B, TOR_NFEAT), labels (B, 4) and n (B,) expected")
    sel = _lib.TorSelectorC()
    losses = np.zeros(opt.epochs, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().tor_selector_train(X.ctypes.data_as(dp), L.ctypes.data_as(dp),
                                   nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), X.shape[0],
                                   ctypes.byref(opt), _stream_ptr(stream), ctypes.byref(sel),
                                   losses.ctypes.data_as(dp)), "tor_selector_train")
    return sel, losses


def tor_mlp_adam(theta, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().tor_mlp_adam(_dptr_t(theta), _dptr_t(grad), _dptr_t(m), _dptr_t(v), float(lr),
                             float(beta1), float(beta2), float(eps), int(step), _stream_ptr(stream)),
          "tor_mlp_adam")


def tor_selector_set(sel: "_lib.TorSelectorC | None"):
    check(lib().tor_selector_set(ctypes.byref(sel) if sel is not None else None), "tor_selector_set")


def tor_selector_get() -> "_lib.TorSelectorC":
    sel = _lib.TorSelectorC()
    check(lib().tor_selector_get(ctypes.byref(sel)), "tor_selector_get")
    return sel


def tor_selector_save(path: str):
    check(lib().tor_selector_save(str(path).encode()), "tor_selector_save")


def tor_selector_load(path: str):
    check(lib().tor_selector_load(str(path).encode()), "tor_selector_load")


def tor_fallback_bits(feats, tau: float) -> float:
    f = np.ascontiguousarray(np.asarray(feats, dtype=np.float64))
    return float(lib().tor_fallback_bits(f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(tau)))


def tor_select_tiers(batch: "Batch", tau: float, stream=None):
    """(tiers, log10_kappa_pred, source) per instance (numpy)."""
    B = batch.batch
    t = np.zeros(B, dtype=np.int32)
    k = np.zeros(B, dtype=np.float64)
    src = np.zeros(B, dtype=np.int32)
    rc = lib().tor_select_tiers(_dptr_t(batch.O),
                                batch.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                batch.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), B, float(tau),
                                _stream_ptr(stream), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    check(rc, "tor_select_tiers")
    return t, k, src


def tor_last_select_stats() -> dict:
    st = _lib.TorSelectStatsC()
    check(lib().tor_last_select_stats(ctypes.byref(st)), "tor_last_select_stats")
    return {name: int(getattr(st, name)) for name, _ in st._fields_ if name != "reserved"}


def tor_debug_level_sums(O, tier="dd", stream=None, algo="border"):
    """(levels, result): levels[m] is L_m = sum over |Z| = m of det^(-1/2),
    each as a Fraction of the returned expansion; algo "border" (the
    bordered kernel) or "schur" (the Schur path's kernels in their level-sum
    mode)."""
    Od, n, ld = _device_o(O)
    lv = np.zeros(4 * (n + 1), dtype=np.float64)
    out = _lib.TorResultC()
    fn = {"border": lib().tor_debug_level_sums, "schur": lib().tor_debug_level_sums_schur}[algo]
    rc = fn(ctypes.c_void_p(Od.data_ptr()), n, ld, tier_id(tier), _stream_ptr(stream),
            lv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(out))
    check(rc, "tor_debug_level_sums")
    levels = [sum((Fraction(x) for x in lv[4 * m:4 * m + 4]), Fraction(0)) for m in range(n + 1)]
    return levels, _res(out)


PHASES = ("expand", "last_level", "wait_after_expand", "bottom", "totals", "wait_after_bottom", "other")


def tor_debug_phase_clocks(reset: bool = False) -> dict:
    """Shader-clock cycles of the middle + bottom kernel per phase, summed
    over its wavefronts (include/tor.h, tor_debug_phase_clocks); needs the
    phase-clock build (TOR_LIBRARY=.../libtor_hip_phase.so)."""
    out = (ctypes.c_uint64 * _lib.TOR_NPHASE)()
    check(lib().tor_debug_phase_clocks(1 if reset else 0, out), "tor_debug_phase_clocks")
    return {name: int(out[k]) for k, name in enumerate(PHASES)}


def tor_debug_sampled_terms(O, masks, tier="dd", stream=None) -> np.ndarray:
    """Signed terms of the given subsets: array (k, 4) of expansions."""
    torch = _torch()
    Od, n, ld = _device_o(O)
    m = torch.as_tensor(np.ascontiguousarray(np.asarray(masks, dtype=np.uint64)).view(np.int64),
                        device=Od.device)
    k = m.numel()
    out = torch.zeros((k, 4), dtype=torch.float64, device=Od.device)
    rc = lib().tor_debug_sampled_terms(ctypes.c_void_p(Od.data_ptr()), n, ld, tier_id(tier),
                                       ctypes.c_void_p(m.data_ptr()), k, _stream_ptr(stream),
                                       ctypes.c_void_p(out.data_ptr()))
    check(rc, "tor_debug_sampled_terms")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return out.cpu().numpy()


def tor_last_kernel_ms():
    """(ms, split_depth, grid, launches) of the dominant kernel in the last
    timed evaluation; ms is the sum over its launches."""
    d = ctypes.c_int32(-1)
    gr = ctypes.c_int32(-1)
    nl = ctypes.c_int32(0)
    ms = lib().tor_last_kernel_ms(ctypes.byref(d), ctypes.byref(gr), ctypes.byref(nl))
    return float(ms), int(d.value), int(gr.value), int(nl.value)


# ---- host scheduling helpers (no GPU) -------------------------------------

def tor_next_mask(mask: int) -> int:
    return int(lib().tor_next_mask(int(mask)))


def tor_kth_mask(N: int, c: int, k: int) -> int:
    return int(lib().tor_kth_mask(int(N), int(c), int(k)))


def tor_workspace_bytes(n: int, tier="dd", bottom_modes: int = 0) -> int:
    """Device bytes one evaluation of an n-mode instance allocates (host only)."""
    b = ctypes.c_uint64(0)
    check(lib().tor_workspace_bytes(int(n), tier_id(tier), int(bottom_modes), ctypes.byref(b)),
          "tor_workspace_bytes")
    return int(b.value)


def tor_batch_workspace_bytes(n: int, count: int, tier="dd", bottom_modes: int = 0) -> int:
    """Device bytes the batched path needs for `count` instances of n modes
    in one tier (host only)."""
    b = ctypes.c_uint64(0)
    check(lib().tor_batch_workspace_bytes(int(n), tier_id(tier), int(count), int(bottom_modes),
                                          ctypes.byref(b)), "tor_batch_workspace_bytes")
    return int(b.value)


def tor_noalloc_nmax(tier="dd") -> int:
    """Largest n tor_eval_noalloc accepts in `tier` (host only)."""
    v = int(lib().tor_noalloc_nmax(tier_id(tier)))
    if v < 0:
        check(v, "tor_noalloc_nmax")
    return v


def tor_eval_noalloc(O, tier="dd", stream=None, out=None):
    """Tor(O) into the device tensor `out` (float64 [8], one tor_result_t;
    allocated here when None) without any allocation inside the library;
    enqueued on the stream, returns `out` without waiting."""
    torch = _torch()
    Od, n, ld = _device_o(O)
    if out is None:
        out = torch.zeros(8, dtype=torch.float64, device=Od.device)
    if out.dtype != torch.float64 or out.numel() < 8 or not out.is_contiguous() or out.device != Od.device:
        raise ValueError("out must be a contiguous float64 device tensor of at least 8 elements")
    check(lib().tor_eval_noalloc(ctypes.c_void_p(Od.data_ptr()), n, ld, tier_id(tier), _stream_ptr(stream),
                                 ctypes.c_void_p(out.data_ptr())), "tor_eval_noalloc")
    return out


def tor_plan_items(n: int, d: int) -> np.ndarray:
    out = np.zeros(1 << d, dtype=np.uint64)
    check(lib().tor_plan_items(int(n), int(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
          "tor_plan_items")
    return out
