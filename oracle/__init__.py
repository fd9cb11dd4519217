"""CPU oracle for the simplified stable parallel merge (Traeff, arXiv:1202.6575).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only ``tests/``, the
package smoke check (``__graft_entry__.smoke``) and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library and never
imports it.

The arithmetic lives in ``oracle.c`` (plain C, built by ``build_oracle``) and,
for the learned cross-rank predictor, in ``oracle/mlp.py`` (numpy, FP64).
This module only marshals numpy arrays into those C routines.

Key types: ``0`` = int32 (signed order), ``1`` = uint32, ``2`` = uint64,
``3`` = int64, ``4`` = float32, ``5`` = float64 (IEEE 754 totalOrder).  The
routines that order keys take ``descending=True`` for non-increasing order
(``DESCENDING`` added to the key type code): ties still keep A before B and
each source's own order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INT32, UINT32, UINT64, INT64, FLOAT32, FLOAT64 = 0, 1, 2, 3, 4, 5
DESCENDING = 8
NP_DTYPE = {INT32: np.int32, UINT32: np.uint32, UINT64: np.uint64, INT64: np.int64,
            FLOAT32: np.float32, FLOAT64: np.float64}


def build_oracle(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no tuning)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.orc_rank_low.restype = i64
        lib.orc_rank_low.argtypes = [vp, i64, vp, i64, i32]
        lib.orc_rank_high.restype = i64
        lib.orc_rank_high.argtypes = [vp, i64, vp, i64, i32]
        lib.orc_merge.restype = None
        lib.orc_merge.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, i32]
        lib.orc_merge_batched.restype = None
        lib.orc_merge_batched.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, i32]
        lib.orc_merge_scatter.restype = i32
        lib.orc_merge_scatter.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, i32]
        lib.orc_block_start.restype = i64
        lib.orc_block_start.argtypes = [i64, i64, i64]
        lib.orc_block_of.restype = i64
        lib.orc_block_of.argtypes = [i64, i64, i64]
        lib.orc_cross_ranks.restype = None
        lib.orc_cross_ranks.argtypes = [vp, i64, vp, i64, i64, i64, i32, vp, vp]
        lib.orc_pieces.restype = None
        lib.orc_pieces.argtypes = [i64, i64, i64, i64, vp, vp, vp]
        lib.orc_pieces_two_select.restype = None
        lib.orc_pieces_two_select.argtypes = [i64, i64, i64, i64, vp, vp, vp]
        lib.orc_merge_by_pieces.restype = i32
        lib.orc_merge_by_pieces.argtypes = [vp, vp, i64, vp, vp, i64, i64, i64, vp, vp, i32]
        lib.orc_sort.restype = None
        lib.orc_sort.argtypes = [vp, vp, i64, i64, vp, vp, i32]
        lib.orc_gallop.restype = i64
        lib.orc_gallop.argtypes = [vp, i64, vp, i64, i32, i32, i64, i64, i64,
                                   ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int)]
        _lib = lib
    return _lib


def dtype_code(arr: np.ndarray) -> int:
    if arr.dtype == np.int32:
        return INT32
    if arr.dtype == np.uint32:
        return UINT32
    if arr.dtype == np.uint64:
        return UINT64
    if arr.dtype == np.int64:
        return INT64
    if arr.dtype == np.float32:
        return FLOAT32
    if arr.dtype == np.float64:
        return FLOAT64
    raise TypeError(f"unsupported key dtype {arr.dtype}")


def _code(arr: np.ndarray, descending: bool = False) -> int:
    return dtype_code(arr) | (DESCENDING if descending else 0)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype=None):
    if a is None:
        return None
    return np.ascontiguousarray(a if dtype is None else a.astype(dtype, copy=False))


def rank_low(x, X: np.ndarray, descending: bool = False) -> int:
    """rank_low(x, X): number of elements of X strictly before x in the order."""
    X = _c(X)
    xa = np.array([x], dtype=X.dtype)
    return int(_load().orc_rank_low(_ptr(xa), 0, _ptr(X), len(X), _code(X, descending)))


def rank_high(x, X: np.ndarray, descending: bool = False) -> int:
    """rank_high(x, X): number of elements of X before or equal to x in the order."""
    X = _c(X)
    xa = np.array([x], dtype=X.dtype)
    return int(_load().orc_rank_high(_ptr(xa), 0, _ptr(X), len(X), _code(X, descending)))


def merge(A, B, pa=None, pb=None, descending: bool = False):
    """O1: stable two-pointer merge.  Returns (C, pc) (pc is None without payloads)."""
    A, B = _c(A), _c(B)
    assert A.dtype == B.dtype
    has_p = pa is not None
    pa, pb = _c(pa, np.uint32), _c(pb, np.uint32)
    C = np.empty(len(A) + len(B), dtype=A.dtype)
    pc = np.empty(len(C), dtype=np.uint32) if has_p else None
    _load().orc_merge(_ptr(A), _ptr(pa), len(A), _ptr(B), _ptr(pb), len(B),
                      _ptr(C), _ptr(pc), _code(A, descending))
    return C, pc


def merge_batched(keys, offsets, n_a, pay=None, descending: bool = False, pairs=None,
                  out=None, out_pay=None):
    """O5: O1 applied to every pair k = keys[offsets[k]:offsets[k+1]] (first
    n_a[k] elements A, the rest B).  ``pairs`` = (k0, k1) merges only those
    pairs into the given ``out`` / ``out_pay`` (the C routine runs without
    Python's lock, so threads may fill disjoint pair ranges).  Returns
    (out, out_pay)."""
    keys = _c(keys)
    offsets = _c(offsets, np.int64)
    n_a = _c(n_a, np.int64)
    has_p = pay is not None
    pay = _c(pay, np.uint32)
    if out is None:
        out = np.empty_like(keys)
    if has_p and out_pay is None:
        out_pay = np.empty(len(keys), dtype=np.uint32)
    k0, k1 = pairs if pairs is not None else (0, len(n_a))
    _load().orc_merge_batched(_ptr(keys), _ptr(pay), _ptr(offsets), _ptr(n_a), k0, k1,
                              _ptr(out), _ptr(out_pay) if has_p else None,
                              _code(keys, descending))
    return out, out_pay


def merge_scatter(A, B, pa=None, pb=None):
    """O2: closed-form scatter.  Returns (C, pc, ok) with ok True iff the
    positions i + rank_low(A[i], B) and j + rank_high(B[j], A) form a permutation."""
    A, B = _c(A), _c(B)
    has_p = pa is not None
    pa, pb = _c(pa, np.uint32), _c(pb, np.uint32)
    C = np.zeros(len(A) + len(B), dtype=A.dtype)
    pc = np.zeros(len(C), dtype=np.uint32) if has_p else None
    rc = _load().orc_merge_scatter(_ptr(A), _ptr(pa), len(A), _ptr(B), _ptr(pb), len(B),
                                   _ptr(C), _ptr(pc), dtype_code(A))
    return C, pc, rc == 0


def block_start(length: int, p: int, i: int) -> int:
    return int(_load().orc_block_start(length, p, i))


def block_of(length: int, p: int, k: int) -> int:
    return int(_load().orc_block_of(length, p, k))


def cross_ranks(A, B, p_a: int, p_b: int | None = None, descending: bool = False):
    """Steps 1-2: (xbar[p_a+1], ybar[p_b+1]) as int64 arrays."""
    p_b = p_a if p_b is None else p_b
    A, B = _c(A), _c(B)
    xbar = np.empty(p_a + 1, dtype=np.int64)
    ybar = np.empty(p_b + 1, dtype=np.int64)
    _load().orc_cross_ranks(_ptr(A), len(A), _ptr(B), len(B), p_a, p_b, _code(A, descending),
                            _ptr(xbar), _ptr(ybar))
    return xbar, ybar


PIECE_FIELDS = ("a_lo", "a_hi", "b_lo", "b_hi", "c_off", "case")


def pieces(n: int, m: int, p_a: int, p_b: int, xbar, ybar, two_select: bool = False):
    """Steps 3-4: int64 array [p_a+p_b, 6] of (a_lo, a_hi, b_lo, b_hi, c_off, case).
    case is ord('a')..ord('e') for A blocks and ord('A')..ord('E') for B blocks
    (0 in the two-select form)."""
    xbar = _c(xbar, np.int64)
    ybar = _c(ybar, np.int64)
    out = np.empty((p_a + p_b, 6), dtype=np.int64)
    f = _load().orc_pieces_two_select if two_select else _load().orc_pieces
    f(n, m, p_a, p_b, _ptr(xbar), _ptr(ybar), _ptr(out))
    return out


def merge_by_pieces(A, B, p_a: int, p_b: int | None = None, pa=None, pb=None,
                    descending: bool = False):
    """The method run sequentially: Steps 1-4, each subproblem merged with O1."""
    p_b = p_a if p_b is None else p_b
    A, B = _c(A), _c(B)
    has_p = pa is not None
    pa, pb = _c(pa, np.uint32), _c(pb, np.uint32)
    C = np.zeros(len(A) + len(B), dtype=A.dtype)
    pc = np.zeros(len(C), dtype=np.uint32) if has_p else None
    rc = _load().orc_merge_by_pieces(_ptr(A), _ptr(pa), len(A), _ptr(B), _ptr(pb), len(B),
                                     p_a, p_b, _ptr(C), _ptr(pc), _code(A, descending))
    if rc != 0:
        raise AssertionError("a subproblem fell outside C")
    return C, pc


def sort(keys, pay=None, run_len: int = 512, descending: bool = False):
    """O4, method mirror: sort runs of run_len, then pairwise merge rounds."""
    keys = np.array(keys, copy=True)
    pay = None if pay is None else np.array(pay, dtype=np.uint32, copy=True)
    tk = np.empty_like(keys)
    tp = None if pay is None else np.empty_like(pay)
    _load().orc_sort(_ptr(keys), _ptr(pay), len(keys), run_len, _ptr(tk), _ptr(tp),
                     _code(keys, descending))
    return keys, pay


def gallop(x, X, is_high: bool, guess: int, window: int, step0: int = 1):
    """O6: bounded exponential search from guess with steps step0, 2 step0,
    4 step0, ... up to window.  Returns (rank, probes, fallback)."""
    X = _c(X)
    xa = np.array([x], dtype=X.dtype)
    probes = ctypes.c_int64(0)
    fb = ctypes.c_int(0)
    r = _load().orc_gallop(_ptr(xa), 0, _ptr(X), len(X), dtype_code(X), int(is_high),
                           int(guess), int(step0), int(window), ctypes.byref(probes),
                           ctypes.byref(fb))
    return int(r), int(probes.value), bool(fb.value)


HIST_BINS = 65
HIST_CENTER = 32


def error_bin(e: int) -> int:
    """Bin of a signed rank error e = guess - rank: bin 32 holds e = 0; bin
    32 + 1 + k holds e in [2^k, 2^(k+1)); bin 32 - 1 - k holds -e in that
    range (k capped at 31)."""
    if e == 0:
        return HIST_CENTER
    k = min(int(abs(e)).bit_length() - 1, 31)
    return HIST_CENTER + 1 + k if e > 0 else HIST_CENTER - 1 - k
