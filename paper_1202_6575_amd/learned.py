"""Learned cross ranks: Python binding of the rank-model entry points of
libstablemerge.so (argument marshalling only; every step runs in the
library's HIP kernels).

A 1 -> 32 (ReLU) -> 1 FP32 network models the cumulative distribution of a
sorted array; a bounded exponential search from its prediction finds the
exact cross rank, falling back to the plain binary search of Steps 1-2 when
the walk would leave the window.  Parameters: 97 device floats
(W1[0:32], b1[32:64], w2[64:96], b2[96]).
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib, _check, _dtype_code, _ptr, _stream_ptr, _require_device, SMError

NPARAM = 97
HIST_BINS = 65
HIST_CENTER = 32

_vp, _i64, _i32, _sz, _f32, _u64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t,
                                    ctypes.c_float, ctypes.c_uint64)
_lib.sm_mlp_grad_workspace_bytes.restype = _sz
_lib.sm_mlp_grad_workspace_bytes.argtypes = [_i64]
_lib.sm_mlp_grad.restype = _i32
_lib.sm_mlp_grad.argtypes = [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.sm_mlp_adam.restype = _i32
_lib.sm_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _vp]
_lib.sm_mlp_init.restype = _i32
_lib.sm_mlp_init.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp]
_lib.sm_mlp_predict.restype = _i32
_lib.sm_mlp_predict.argtypes = [_vp, _vp, _i64, _i32, _i64, _vp, _vp]
_lib.sm_rank_model_workspace_bytes.restype = _sz
_lib.sm_rank_model_workspace_bytes.argtypes = [_i64, _i32]
_lib.stable_merge_sort_learned.restype = _i32
_lib.stable_merge_sort_learned.argtypes = [_vp, _vp, _i64, _vp, _vp, _i32, _vp, _f32, _vp, _vp,
                                           _sz, _vp, _vp]
_lib.sm_rank_model_train.restype = _i32
_lib.sm_rank_model_train.argtypes = [_vp, _i64, _vp, _i64, _i32, _i32, _i64, _i64, _f32, _u64,
                                     _vp, _vp, _vp, _sz, _vp]
_lib.stable_merge_rank_search.restype = _i32
_lib.stable_merge_rank_search.argtypes = [_vp, _i64, _vp, _i64, _i32, _i32, _vp, _i64, _i64, _vp,
                                          _vp, _vp, _vp]
_lib.stable_merge_partition_learned.restype = _i32
_lib.stable_merge_partition_learned.argtypes = [_vp, _i64, _i64, _i64, _i64, _i32, _vp, _vp, _i64,
                                                _i64, _i64, _vp, _vp, _vp, _vp, _vp]
_lib.stable_merge_learned.restype = _i32
_lib.stable_merge_learned.argtypes = [_vp, _vp, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _i64,
                                      _i64, _i64, _vp, _vp, _vp, _sz, _vp]
_lib.stable_merge_learned_workspace_bytes.restype = _sz
_lib.stable_merge_learned_workspace_bytes.argtypes = [_i64, _i64, _i64, _i32, _i32]
_pp = ctypes.POINTER(ctypes.c_void_p)
_lib.sm_predictor_create.restype = _i32
_lib.sm_predictor_create.argtypes = [_pp, _i32, _i32]
_lib.sm_predictor_destroy.restype = _i32
_lib.sm_predictor_destroy.argtypes = [_vp]
_lib.sm_predictor_train.restype = _i32
_lib.sm_predictor_train.argtypes = [_vp, _vp, _i64, _vp, _i64, _i64, _i64, _f32, _u64, _vp, _sz,
                                    _vp]
_lib.sm_predictor_params.restype = _vp
_lib.sm_predictor_params.argtypes = [_vp]
_lib.sm_predictor_info.restype = _i32
_lib.sm_predictor_info.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                   ctypes.POINTER(_i64), ctypes.POINTER(_f32)]
_lib.sm_predictor_save.restype = _i32
_lib.sm_predictor_save.argtypes = [_vp, _vp, _sz]
_lib.sm_predictor_load.restype = _i32
_lib.sm_predictor_load.argtypes = [_pp, _vp, _sz]
BLOB_BYTES = 432


def _f32_params(p):
    if p.dtype != torch.float32 or p.numel() != NPARAM or not p.is_cuda or not p.is_contiguous():
        raise SMError(-1, "params must be a contiguous device float32 tensor of 97 entries")


def _model_ptr(model):
    """Device address of a model: a Predictor handle or a tensor of 97
    device floats."""
    if isinstance(model, Predictor):
        return model.ptr()
    _f32_params(model)
    return _ptr(model)


def mlp_grad(params, keys, target, *, stream=None):
    """(grad[97], loss) of the mean squared normalised-rank error (device tensors)."""
    _f32_params(params)
    _require_device(keys, target)
    S = keys.numel()
    grad = torch.empty(NPARAM, dtype=torch.float32, device=keys.device)
    loss = torch.empty(1, dtype=torch.float32, device=keys.device)
    ws = torch.empty(max(int(_lib.sm_mlp_grad_workspace_bytes(S)), 16), dtype=torch.uint8,
                     device=keys.device)
    _check(_lib.sm_mlp_grad(_ptr(params), _ptr(keys), _ptr(target), S, _dtype_code(keys),
                            _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return grad, loss


def mlp_adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, *, stream=None):
    """One Adam step, in place on params, m and v."""
    for t in (params, m, v, grad):
        _f32_params(t)
    _check(_lib.sm_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr),
                            float(beta1), float(beta2), float(eps), _stream_ptr(stream)))


def mlp_init(sorted_keys, target, *, stream=None):
    """Interpolating knot initialisation from a sorted sample and its targets."""
    _require_device(sorted_keys, target)
    p = torch.empty(NPARAM, dtype=torch.float32, device=sorted_keys.device)
    _check(_lib.sm_mlp_init(_ptr(sorted_keys), _ptr(target), sorted_keys.numel(),
                            _dtype_code(sorted_keys), _ptr(p), _stream_ptr(stream)))
    return p


def mlp_predict(params, keys, length, *, stream=None):
    _f32_params(params)
    _require_device(keys)
    out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    _check(_lib.sm_mlp_predict(_ptr(params), _ptr(keys), keys.numel(), _dtype_code(keys),
                               int(length), _ptr(out), _stream_ptr(stream)))
    return out


def train_rank_model(X, Q, is_high, samples=1 << 20, steps=1000, lr=3e-3, seed=0, *,
                     params=None, workspace=None, stream=None):
    """Trains a model of sorted X for sorted queries Q.  Returns (params,
    loss tensor[1]); sqrt(loss) * len(X) is the RMS rank error on the sample."""
    _require_device(X, Q, params, workspace)
    code = _dtype_code(X)
    if params is None:
        params = torch.empty(NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    if workspace is None:
        need = int(_lib.sm_rank_model_workspace_bytes(samples, code))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=X.device)
    _check(_lib.sm_rank_model_train(_ptr(X), X.numel(), _ptr(Q), Q.numel(), code, int(is_high),
                                    int(samples), int(steps), float(lr), int(seed) & (2 ** 64 - 1),
                                    _ptr(params), _ptr(loss), _ptr(workspace), workspace.numel(),
                                    _stream_ptr(stream)))
    return params, loss


def step0_from_loss(loss: float, length: int) -> int:
    """Initial search step: the largest power of two not above the RMS rank error."""
    rms = math.sqrt(max(float(loss), 0.0)) * length
    return 1 << max(0, int(math.floor(math.log2(rms)))) if rms >= 1.0 else 1


def rank_search(X, queries, guess, is_high, step0=1, window=256, *, stream=None):
    """(ranks int64, probes int32, fallback int32) of queries in sorted X."""
    _require_device(X, queries, guess)
    q = queries.numel()
    dev = queries.device
    ranks = torch.empty(q, dtype=torch.int64, device=dev)
    probes = torch.empty(q, dtype=torch.int32, device=dev)
    fb = torch.empty(q, dtype=torch.int32, device=dev)
    _check(_lib.stable_merge_rank_search(_ptr(X), X.numel(), _ptr(queries), q, _dtype_code(X),
                                         int(is_high), _ptr(guess), int(step0), int(window),
                                         _ptr(ranks), _ptr(probes), _ptr(fb), _stream_ptr(stream)))
    return ranks, probes, fb


def partition_learned(keys, n, m, p_a, p_b, model_b, model_a, step0_a=1, step0_b=1, window=256,
                      *, xbar=None, ybar=None, hist=None, counters=None, stream=None):
    """Steps 1-2 from learned starting points.  Returns (xbar, ybar, hist,
    counters) with counters = [searches, fallbacks, probes]; hist and
    counters are accumulated into when given."""
    mb, ma = _model_ptr(model_b), _model_ptr(model_a)
    _require_device(keys, xbar, ybar, hist, counters)
    dev = keys.device
    if xbar is None:
        xbar = torch.empty(p_a + 1, dtype=torch.int64, device=dev)
    if ybar is None:
        ybar = torch.empty(p_b + 1, dtype=torch.int64, device=dev)
    if hist is None:
        hist = torch.zeros(HIST_BINS, dtype=torch.uint64, device=dev)
    if counters is None:
        counters = torch.zeros(4, dtype=torch.uint64, device=dev)
    _check(_lib.stable_merge_partition_learned(_ptr(keys), n, m, p_a, p_b, _dtype_code(keys),
                                               mb, ma, int(step0_a),
                                               int(step0_b), int(window), _ptr(xbar), _ptr(ybar),
                                               _ptr(hist), _ptr(counters), _stream_ptr(stream)))
    return xbar, ybar, hist, counters


def merge_learned(keys, n, m, model_b, model_a, step0_a=1, step0_b=1, block=16, window=256,
                  payloads=None, *, out_keys=None, out_payloads=None, hist=None, counters=None,
                  workspace=None, stream=None):
    """The whole stable merge of keys = A (n) ‖ B (m) with learned cross
    ranks at blocks of `block` elements per side.  Returns (out_keys,
    out_payloads, hist, counters); the output is the unique stable merge
    whatever the models predict."""
    mb, ma = _model_ptr(model_b), _model_ptr(model_a)
    _require_device(keys, payloads, out_keys, out_payloads, hist, counters, workspace)
    dev = keys.device
    code = _dtype_code(keys)
    if workspace is None:
        need = int(_lib.stable_merge_learned_workspace_bytes(n, m, int(block), code,
                                                             int(payloads is not None)))
        if need == 0:
            raise SMError(-1, "stable_merge_learned: unsupported sizes or block")
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if out_keys is None:
        out_keys = torch.empty(n + m, dtype=keys.dtype, device=dev)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(n + m, dtype=torch.uint32, device=dev)
    if hist is None:
        hist = torch.zeros(HIST_BINS, dtype=torch.uint64, device=dev)
    if counters is None:
        counters = torch.zeros(4, dtype=torch.uint64, device=dev)
    _check(_lib.stable_merge_learned(_ptr(keys), _ptr(payloads), n, m, _ptr(out_keys),
                                     _ptr(out_payloads), code, mb, ma,
                                     int(step0_a), int(step0_b), int(block), int(window),
                                     _ptr(hist), _ptr(counters), _ptr(workspace),
                                     workspace.numel(), _stream_ptr(stream)))
    return out_keys, out_payloads, hist, counters


def train_sort_model(keys, sample=1 << 20, samples=1 << 18, steps=1000, lr=3e-3, seed=0, *,
                     stream=None):
    """A model of the keys' distribution for sort_learned: the first `sample`
    keys, sorted by the library's own sort, are the modelled array (an
    unbiased sample when the input order carries no information; any model
    gives the same sort).  Returns (params, step_frac) with step_frac the
    RMS rank error relative to the array length."""
    from . import sort as _sort
    _require_device(keys)
    k = min(int(sample), keys.numel())
    if k < 2:
        raise SMError(-1, "train_sort_model: need at least two keys")
    X, _ = _sort(keys[:k].contiguous(), stream=stream)
    params, loss = train_rank_model(X, X, False, samples=min(int(samples), k), steps=steps, lr=lr,
                                    seed=seed, stream=stream)
    return params, math.sqrt(max(float(loss.item()), 0.0))


def sort_learned(keys, model, step_frac, payloads=None, *, out_keys=None, out_payloads=None,
                 run: int = 0, tile: int = 0, counters=None, workspace=None, stream=None):
    """stable_merge_sort with learned cross ranks in every merge pass.
    Returns (out_keys, out_payloads, counters) with counters = [searches,
    probes] accumulated over the passes; the output equals sort()'s."""
    from . import _opts
    mp = _model_ptr(model)
    _require_device(keys, payloads, out_keys, out_payloads, counters, workspace)
    N = keys.numel()
    code = _dtype_code(keys)
    dev = keys.device
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(N, dtype=torch.uint32, device=dev)
    if counters is None:
        counters = torch.zeros(2, dtype=torch.uint64, device=dev)
    o = _opts(0, 0, tile, False, run)
    if workspace is None:
        need = int(_lib.stable_merge_sort_workspace_bytes(N, code, int(payloads is not None),
                                                          ctypes.byref(o)))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=dev)
    _check(_lib.stable_merge_sort_learned(_ptr(keys), _ptr(payloads), N, _ptr(out_keys),
                                          _ptr(out_payloads), code, mp,
                                          float(step_frac), _ptr(counters), _ptr(workspace),
                                          workspace.numel(), ctypes.byref(o),
                                          _stream_ptr(stream)))
    return out_keys, out_payloads, counters


class Predictor:
    """A rank-model handle of the library (sm_predictor_*): the network with
    its key type and rank kind, trainable, savable to SM_PREDICTOR_BLOB_BYTES
    host bytes and loadable from them.  ``params()`` is a device tensor view
    of its 97 parameters for the calls that take a model."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def create(cls, dtype, is_high: bool) -> "Predictor":
        h = ctypes.c_void_p()
        code = _dtype_code(torch.empty(0, dtype=dtype))
        _check(_lib.sm_predictor_create(ctypes.byref(h), code, int(bool(is_high))))
        return cls(h)

    @classmethod
    def load(cls, blob: bytes) -> "Predictor":
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = ctypes.c_void_p()
        _check(_lib.sm_predictor_load(ctypes.byref(h), buf, len(blob)))
        return cls(h)

    def train(self, X, Q, samples=1 << 20, steps=1000, lr=3e-3, seed=0, *, workspace=None,
              stream=None) -> "Predictor":
        _require_device(X, Q, workspace)
        if workspace is None:
            need = int(_lib.sm_rank_model_workspace_bytes(samples, _dtype_code(X)))
            workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=X.device)
        _check(_lib.sm_predictor_train(self._h, _ptr(X), X.numel(), _ptr(Q), Q.numel(),
                                       int(samples), int(steps), float(lr),
                                       int(seed) & (2 ** 64 - 1), _ptr(workspace),
                                       workspace.numel(), _stream_ptr(stream)))
        return self

    def info(self):
        """(dtype code, is_high, trained array length, last loss)."""
        d, h, n, loss = _i32(), _i32(), _i64(), _f32()
        _check(_lib.sm_predictor_info(self._h, ctypes.byref(d), ctypes.byref(h), ctypes.byref(n),
                                      ctypes.byref(loss)))
        return d.value, bool(h.value), n.value, loss.value

    def save(self) -> bytes:
        buf = ctypes.create_string_buffer(BLOB_BYTES)
        _check(_lib.sm_predictor_save(self._h, buf, BLOB_BYTES))
        return buf.raw

    def params(self) -> torch.Tensor:
        """A copy of the handle's 97 parameters as a device float32 tensor
        (the calls that take a model also accept the Predictor itself)."""
        import numpy as np
        p = np.frombuffer(self.save(), dtype="<f4", count=NPARAM, offset=40)
        return torch.from_numpy(p.copy()).to(torch.device("cuda", torch.cuda.current_device()))

    def ptr(self) -> ctypes.c_void_p:
        """Device address of the handle's parameters."""
        ptr = _lib.sm_predictor_params(self._h) if self._h else None
        if not ptr:
            raise SMError(-1, "invalid predictor handle")
        return ctypes.c_void_p(ptr)

    def close(self):
        if self._h:
            _check(_lib.sm_predictor_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
