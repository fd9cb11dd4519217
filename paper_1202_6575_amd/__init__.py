"""Stable parallel merge for AMD MI355X (gfx950).

Python binding of ``libstablemerge.so`` (C ABI in ``include/stablemerge.h``),
after J. L. Traeff, "Simplified, stable parallel merging" (arXiv:1202.6575).

This module only marshals arguments: it takes torch device tensors, passes
their device pointers and the current HIP stream to the library, and turns
negative status codes into exceptions.  Every step of the merge runs in the
library's HIP kernels; there is no fallback path.  If the library is not
built, importing this package raises.

Keys layout: A = keys[0:n], B = keys[n:n+m] in one contiguous buffer.
Supported key dtypes: torch.int32 and torch.int64 (signed order), torch.uint32,
torch.uint64, torch.float32 and torch.float64 (IEEE 754 totalOrder: -NaN < -inf
< ... < -0 < +0 < ... < +inf < +NaN).
Payloads: optional torch.uint32 tensor with the same layout.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["merge", "merge_noalloc", "partition", "merge_pieces", "merge_batched", "sort",
           "sort_runs", "segmented_sort", "workspace_bytes", "pieces_workspace_bytes", "batched_workspace_bytes",
           "sort_workspace_bytes", "segmented_sort_workspace_bytes", "SMError", "LIB_PATH",
           "DTYPES"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstablemerge.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950) first")

_lib = ctypes.CDLL(LIB_PATH)

SM_INT32, SM_UINT32, SM_UINT64, SM_INT64, SM_FLOAT32, SM_FLOAT64 = 0, 1, 2, 3, 4, 5
DTYPES = {torch.int32: SM_INT32, torch.uint32: SM_UINT32, torch.uint64: SM_UINT64,
          torch.int64: SM_INT64, torch.float32: SM_FLOAT32, torch.float64: SM_FLOAT64}
STATUS = {0: "SM_OK", -1: "SM_ERR_ARG", -2: "SM_ERR_DTYPE", -3: "SM_ERR_ALIAS",
          -4: "SM_ERR_WORKSPACE", -5: "SM_ERR_HIP", -6: "SM_ERR_UNSORTED"}


class SMError(RuntimeError):
    """A negative status from libstablemerge; ``code`` holds it."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("p_a", ctypes.c_int64), ("p_b", ctypes.c_int64), ("tile", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("run", ctypes.c_int32),
                ("descending", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
_lib.sm_last_error.restype = ctypes.c_char_p
_lib.sm_last_error.argtypes = []
_lib.sm_version.restype = _i32
_lib.stable_merge_workspace_bytes.restype = _sz
_lib.stable_merge_workspace_bytes.argtypes = [_i64, _i64, _i32, _i32, ctypes.POINTER(Options)]
_lib.stable_merge.restype = _i32
_lib.stable_merge.argtypes = [_vp, _vp, _i64, _i64, _vp, _vp, _i32, _vp, _sz,
                              ctypes.POINTER(Options), _vp]
_lib.stable_merge_noalloc.restype = _i32
_lib.stable_merge_noalloc.argtypes = [_vp, _vp, _i64, _i64, _vp, _vp, _i32,
                                      ctypes.POINTER(Options), _vp]
_lib.stable_merge_pieces.restype = _i32
_lib.stable_merge_pieces.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _i32,
                                     _vp, _sz, _vp]
_lib.stable_merge_pieces_workspace_bytes.restype = _sz
_lib.stable_merge_pieces_workspace_bytes.argtypes = [_i64, _i64, _i64, _i64, _i32, _i32]
_lib.stable_merge_batched.restype = _i32
_lib.stable_merge_batched.argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _i32, _vp, _sz,
                                      ctypes.POINTER(Options), _vp]
_lib.stable_merge_batched_workspace_bytes.restype = _sz
_lib.stable_merge_batched_workspace_bytes.argtypes = [_i64, _i64, _i32, _i32,
                                                      ctypes.POINTER(Options)]
_lib.stable_merge_sort.restype = _i32
_lib.stable_merge_sort.argtypes = [_vp, _vp, _i64, _vp, _vp, _i32, _vp, _sz,
                                   ctypes.POINTER(Options), _vp]
_lib.stable_merge_sort_runs.restype = _i32
_lib.stable_merge_sort_runs.argtypes = [_vp, _vp, _i64, _vp, _vp, _i32, _i32, _vp]
_lib.stable_merge_sort_workspace_bytes.restype = _sz
_lib.stable_merge_sort_workspace_bytes.argtypes = [_i64, _i32, _i32, ctypes.POINTER(Options)]
_lib.stable_merge_segmented_sort.restype = _i32
_lib.stable_merge_segmented_sort.argtypes = [_vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _i32, _vp,
                                             _sz, ctypes.POINTER(Options), _vp]
_lib.stable_merge_segmented_sort_workspace_bytes.restype = _sz
_lib.stable_merge_segmented_sort_workspace_bytes.argtypes = [_i64, _i64, _i64, _i32, _i32,
                                                             ctypes.POINTER(Options)]
_lib.stable_merge_partition.restype = _i32
_lib.stable_merge_partition.argtypes = [_vp, _i64, _i64, _i64, _i64, _i32, _vp, _vp, _vp]


def _check(rc: int):
    if rc != 0:
        raise SMError(rc, _lib.sm_last_error().decode())


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return DTYPES[t.dtype]
    except KeyError:
        raise SMError(-2, f"unsupported key dtype {t.dtype}") from None


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _opts(p_a=0, p_b=0, tile=0, validate=False, run=0, descending=False) -> Options:
    return Options(int(p_a), int(p_b), int(tile), int(bool(validate)), int(run),
                   int(bool(descending)))


def workspace_bytes(n: int, m: int, dtype: torch.dtype, has_payload: bool = False,
                    p_a: int = 0, p_b: int = 0, tile: int = 0, descending: bool = False) -> int:
    """Device workspace bytes stable_merge needs (0 on bad arguments)."""
    o = _opts(p_a, p_b, tile, descending=descending)
    return int(_lib.stable_merge_workspace_bytes(n, m, DTYPES[dtype], int(has_payload),
                                                 ctypes.byref(o)))


def pieces_workspace_bytes(n: int, m: int, p_a: int, p_b: int, dtype: torch.dtype,
                           has_payload: bool = False) -> int:
    """Device workspace bytes stable_merge_pieces needs (0 on bad arguments)."""
    return int(_lib.stable_merge_pieces_workspace_bytes(n, m, p_a, p_b, DTYPES[dtype],
                                                        int(has_payload)))


def batched_workspace_bytes(count: int, total: int, dtype: torch.dtype,
                            has_payload: bool = False, tile: int = 0,
                            descending: bool = False) -> int:
    """Device workspace bytes stable_merge_batched needs (0 on bad arguments)."""
    o = _opts(0, 0, tile, descending=descending)
    return int(_lib.stable_merge_batched_workspace_bytes(count, total, DTYPES[dtype],
                                                         int(has_payload), ctypes.byref(o)))


def sort_workspace_bytes(N: int, dtype: torch.dtype, has_payload: bool = False, run: int = 0,
                         tile: int = 0) -> int:
    """Device workspace bytes stable_merge_sort needs (0 on bad arguments)."""
    o = _opts(0, 0, tile, False, run)
    return int(_lib.stable_merge_sort_workspace_bytes(N, DTYPES[dtype], int(has_payload),
                                                      ctypes.byref(o)))


def _tuned(op: str, keys: torch.Tensor, has_payload: bool, size: int) -> int:
    """The block length cached by the autotuner for this call's class, else
    0 (the library's default)."""
    from . import autotune
    got = autotune.lookup(op, keys.dtype, has_payload, size, device=keys.device)
    return got if got is not None else 0


def _require_device(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise SMError(-1, "tensors must be contiguous device tensors")


def merge(keys: torch.Tensor, n: int, m: int | None = None, payloads: torch.Tensor | None = None,
          *, out_keys: torch.Tensor | None = None, out_payloads: torch.Tensor | None = None,
          p_a: int = 0, p_b: int = 0, tile: int = 0, validate: bool = False,
          descending: bool = False, workspace: torch.Tensor | None = None, stream=None):
    """Stable merge of A = keys[:n] and B = keys[n:n+m] (Section 2, Steps 1-4).

    Returns (out_keys, out_payloads); out_payloads is None without payloads.
    Equal keys keep A before B; each source keeps its order.  With
    descending=True both inputs and the output run from largest to smallest.
    With tile, p_a and p_b all 0 and no workspace given, the autotuner's
    cached block length for this size class is used, if there is one."""
    if m is None:
        m = keys.numel() - n
    if keys.numel() < n + m:
        raise SMError(-1, "keys holds fewer than n + m elements")
    _require_device(keys, payloads, out_keys, out_payloads, workspace)
    code = _dtype_code(keys)
    if out_keys is None:
        out_keys = torch.empty(n + m, dtype=keys.dtype, device=keys.device)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(n + m, dtype=torch.uint32, device=keys.device)
    if tile == 0 and p_a == 0 and p_b == 0 and workspace is None:
        tile = _tuned("merge", keys, payloads is not None, n + m)
    o = _opts(p_a, p_b, tile, validate, descending=descending)
    need = int(_lib.stable_merge_workspace_bytes(n, m, code, int(payloads is not None),
                                                 ctypes.byref(o)))
    if workspace is None:
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=keys.device)
    _check(_lib.stable_merge(_ptr(keys), _ptr(payloads), n, m, _ptr(out_keys), _ptr(out_payloads),
                             code, _ptr(workspace), workspace.numel(), ctypes.byref(o),
                             _stream_ptr(stream)))
    return out_keys, out_payloads


NOALLOC_SCRATCH_BYTES = 16 << 20


def merge_noalloc(keys: torch.Tensor, n: int, m: int | None, payloads: torch.Tensor | None,
                  out_keys: torch.Tensor, out_payloads: torch.Tensor | None = None, *,
                  p_a: int = 0, p_b: int = 0, tile: int = 0, descending: bool = False,
                  stream=None):
    """stable_merge_noalloc: the merge of ``merge`` into caller-given outputs,
    with the library's per-device scratch array in place of a workspace (for
    callers that cannot allocate).  Calls that overlap on one device race on
    that array."""
    if m is None:
        m = keys.numel() - n
    if keys.numel() < n + m or out_keys.numel() < n + m:
        raise SMError(-1, "keys and out_keys must hold n + m elements")
    _require_device(keys, payloads, out_keys, out_payloads)
    o = _opts(p_a, p_b, tile, False, descending=descending)
    _check(_lib.stable_merge_noalloc(_ptr(keys), _ptr(payloads), n, m, _ptr(out_keys),
                                     _ptr(out_payloads), _dtype_code(keys), ctypes.byref(o),
                                     _stream_ptr(stream)))
    return out_keys, out_payloads


def partition(keys: torch.Tensor, n: int, m: int, p_a: int, p_b: int | None = None, *,
              xbar: torch.Tensor | None = None, ybar: torch.Tensor | None = None, stream=None):
    """Steps 1-2: (xbar[p_a+1], ybar[p_b+1]) as device int64 tensors."""
    p_b = p_a if p_b is None else p_b
    _require_device(keys, xbar, ybar)
    if xbar is None:
        xbar = torch.empty(p_a + 1, dtype=torch.int64, device=keys.device)
    if ybar is None:
        ybar = torch.empty(p_b + 1, dtype=torch.int64, device=keys.device)
    if xbar.numel() < p_a + 1 or ybar.numel() < p_b + 1 or xbar.dtype != torch.int64 \
            or ybar.dtype != torch.int64:
        raise SMError(-1, "xbar / ybar must be int64 with p_a + 1 / p_b + 1 entries")
    _check(_lib.stable_merge_partition(_ptr(keys), n, m, p_a, p_b, _dtype_code(keys), _ptr(xbar),
                                       _ptr(ybar), _stream_ptr(stream)))
    return xbar, ybar


def merge_pieces(keys: torch.Tensor, n: int, m: int, p_a: int, p_b: int, xbar: torch.Tensor,
                 ybar: torch.Tensor, payloads: torch.Tensor | None = None, *,
                 out_keys: torch.Tensor | None = None, out_payloads: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None, stream=None):
    """Steps 3-4 given the cross ranks of ``partition`` for the same p_a, p_b."""
    _require_device(keys, payloads, out_keys, out_payloads, xbar, ybar, workspace)
    code = _dtype_code(keys)
    if workspace is None:
        need = int(_lib.stable_merge_pieces_workspace_bytes(n, m, p_a, p_b, code,
                                                            int(payloads is not None)))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=keys.device)
    if out_keys is None:
        out_keys = torch.empty(n + m, dtype=keys.dtype, device=keys.device)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(n + m, dtype=torch.uint32, device=keys.device)
    _check(_lib.stable_merge_pieces(_ptr(keys), _ptr(payloads), n, m, p_a, p_b, _ptr(xbar),
                                    _ptr(ybar), _ptr(out_keys), _ptr(out_payloads), code,
                                    _ptr(workspace), workspace.numel(), _stream_ptr(stream)))
    return out_keys, out_payloads


def merge_batched(keys: torch.Tensor, offsets: torch.Tensor, n_a: torch.Tensor,
                  payloads: torch.Tensor | None = None, *, out_keys: torch.Tensor | None = None,
                  out_payloads: torch.Tensor | None = None, tile: int = 0,
                  validate: bool = False, descending: bool = False,
                  workspace: torch.Tensor | None = None, stream=None):
    """Independent stable merges of many pairs in one launch sequence.

    Pair k is keys[offsets[k]:offsets[k+1]] with its first n_a[k] elements as
    A; its merge lands in the same range of out_keys.  offsets (count + 1) and
    n_a (count) are device int64 tensors.  Returns (out_keys, out_payloads).
    With tile 0 and no workspace given, the autotuner's cached block length
    for this size class is used, if there is one."""
    _require_device(keys, offsets, n_a, payloads, out_keys, out_payloads, workspace)
    if offsets.dtype != torch.int64 or n_a.dtype != torch.int64:
        raise SMError(-1, "offsets and n_a must be int64")
    count = n_a.numel()
    if offsets.numel() != count + 1:
        raise SMError(-1, "offsets must hold count + 1 entries")
    total = keys.numel()
    code = _dtype_code(keys)
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(total, dtype=torch.uint32, device=keys.device)
    if tile == 0 and workspace is None:
        tile = _tuned("batched", keys, payloads is not None, total)
    o = _opts(0, 0, tile, validate, descending=descending)
    if workspace is None:
        need = int(_lib.stable_merge_batched_workspace_bytes(count, total, code,
                                                             int(payloads is not None),
                                                             ctypes.byref(o)))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=keys.device)
    _check(_lib.stable_merge_batched(_ptr(keys), _ptr(payloads), _ptr(offsets), _ptr(n_a), count,
                                     total, _ptr(out_keys), _ptr(out_payloads), code,
                                     _ptr(workspace), workspace.numel(), ctypes.byref(o),
                                     _stream_ptr(stream)))
    return out_keys, out_payloads


def sort(keys: torch.Tensor, payloads: torch.Tensor | None = None, *,
         out_keys: torch.Tensor | None = None, out_payloads: torch.Tensor | None = None,
         run: int = 0, tile: int = 0, descending: bool = False,
         workspace: torch.Tensor | None = None, stream=None):
    """Stable merge sort of keys (payloads travel along), smallest first or,
    with descending=True, largest first.  Passing the inputs as out_keys /
    out_payloads sorts in place.  Returns (out_keys, out_payloads)."""
    _require_device(keys, payloads, out_keys, out_payloads, workspace)
    N = keys.numel()
    code = _dtype_code(keys)
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(N, dtype=torch.uint32, device=keys.device)
    o = _opts(0, 0, tile, False, run, descending)
    if workspace is None:
        need = int(_lib.stable_merge_sort_workspace_bytes(N, code, int(payloads is not None),
                                                          ctypes.byref(o)))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=keys.device)
    _check(_lib.stable_merge_sort(_ptr(keys), _ptr(payloads), N, _ptr(out_keys),
                                  _ptr(out_payloads), code, _ptr(workspace), workspace.numel(),
                                  ctypes.byref(o), _stream_ptr(stream)))
    return out_keys, out_payloads


def sort_runs(keys: torch.Tensor, run: int = 512, payloads: torch.Tensor | None = None, *,
              out_keys: torch.Tensor | None = None, out_payloads: torch.Tensor | None = None,
              stream=None):
    """The merge sort's run formation alone: every run of `run` consecutive
    elements stably sorted on its own.  Returns (out_keys, out_payloads)."""
    _require_device(keys, payloads, out_keys, out_payloads)
    N = keys.numel()
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(N, dtype=torch.uint32, device=keys.device)
    _check(_lib.stable_merge_sort_runs(_ptr(keys), _ptr(payloads), N, _ptr(out_keys),
                                       _ptr(out_payloads), _dtype_code(keys), int(run),
                                       _stream_ptr(stream)))
    return out_keys, out_payloads


def segmented_sort_workspace_bytes(count: int, N: int, max_len: int, dtype: torch.dtype,
                                   has_payload: bool = False, run: int = 0, tile: int = 0) -> int:
    """Device workspace bytes stable_merge_segmented_sort needs (0 on bad arguments)."""
    o = _opts(0, 0, tile, False, run)
    return int(_lib.stable_merge_segmented_sort_workspace_bytes(
        count, N, max_len, DTYPES[dtype], int(has_payload), ctypes.byref(o)))


def segmented_sort(keys: torch.Tensor, offsets: torch.Tensor, max_len: int,
                   payloads: torch.Tensor | None = None, *, out_keys: torch.Tensor | None = None,
                   out_payloads: torch.Tensor | None = None, run: int = 0, tile: int = 0,
                   validate: bool = False, descending: bool = False,
                   workspace: torch.Tensor | None = None, stream=None):
    """Stable sort of every segment keys[offsets[s]:offsets[s+1]] on its own.
    offsets is a device int64 tensor of count + 1 entries from 0 to N; max_len
    bounds the segment lengths (host value).  Returns (out_keys, out_payloads)."""
    _require_device(keys, offsets, payloads, out_keys, out_payloads, workspace)
    if offsets.dtype != torch.int64:
        raise SMError(-1, "offsets must be int64")
    N = keys.numel()
    count = offsets.numel() - 1
    code = _dtype_code(keys)
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if payloads is not None and out_payloads is None:
        out_payloads = torch.empty(N, dtype=torch.uint32, device=keys.device)
    o = _opts(0, 0, tile, validate, run, descending)
    if workspace is None:
        need = int(_lib.stable_merge_segmented_sort_workspace_bytes(
            count, N, max_len, code, int(payloads is not None), ctypes.byref(o)))
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=keys.device)
    _check(_lib.stable_merge_segmented_sort(_ptr(keys), _ptr(payloads), _ptr(offsets), count, N,
                                            max_len, _ptr(out_keys), _ptr(out_payloads), code,
                                            _ptr(workspace), workspace.numel(), ctypes.byref(o),
                                            _stream_ptr(stream)))
    return out_keys, out_payloads
