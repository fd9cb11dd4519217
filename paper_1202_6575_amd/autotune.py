"""Autotuner for the merge launch parameters.

The launch parameter that changes the speed of the merge kernels, and never
the output (a stable merge is unique), is the block length ``tile``: a
subproblem holds up to 2 * tile elements, which one workgroup of 256 lanes
stages in LDS, so the tile sets the items per lane (about 2 * tile / 256)
and how many workgroups share a compute unit.

``tune`` times every candidate tile on the caller's own data (HIP events on
the current stream, median of several runs), returns the fastest and caches
it per (operation, key type, payload, size class, device) in a JSON file
(``SM_AUTOTUNE_CACHE``, default ``~/.cache/paper_1202_6575_amd/autotune.json``).
``lookup`` reads that cache; the package's ``merge`` and ``merge_batched``
consult it whenever the caller leaves ``tile`` at 0 and passes no workspace
(a workspace is sized for one tile), and otherwise use the library's
default.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

TILES = (512, 1024, 1152, 1536, 2048, 2368, 3072, 4096)

_memo: dict = {}


def cache_path() -> str:
    return os.environ.get("SM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1202_6575_amd",
                                       "autotune.json"))


def size_class(size: int) -> int:
    """The power of two of the element count."""
    return int(math.log2(max(int(size), 1)))


def cache_key(op: str, dtype: torch.dtype, has_payload: bool, size: int, device=None) -> str:
    """Key of one cache entry; the device is the current one unless given."""
    dev = torch.cuda.current_device() if device is None else (torch.device(device).index or 0)
    name = torch.cuda.get_device_name(dev).replace(" ", "_")
    return (f"{op}/{str(dtype).replace('torch.', '')}/{'pay' if has_payload else 'keys'}/"
            f"2^{size_class(size)}/{name}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _read_cached(path):
    """The cache file's contents, read again only when the file changed."""
    try:
        st = os.stat(path)
    except OSError:
        return {}
    stamp = (st.st_mtime_ns, st.st_size)
    hit = _memo.get(path)
    if hit and hit[0] == stamp:
        return hit[1]
    data = _load(path)
    _memo[path] = (stamp, data)
    return data


def lookup(op: str, dtype: torch.dtype, has_payload: bool, size: int, device=None,
           path: str | None = None):
    """The cached tile for this operation and size class on this device, or
    None."""
    entry = _read_cached(path or cache_path()).get(cache_key(op, dtype, has_payload, size, device))
    return int(entry["tile"]) if entry else None


def time_ms(fn, reps: int = 5, warmup: int = 1) -> float:
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def tune(op: str, run, dtype: torch.dtype, has_payload: bool, size: int, cands=None,
         valid=None, reps: int = 5, use_cache: bool = True, path: str | None = None):
    """Returns (best tile, {tile: ms}).  run(tile) launches the operation
    once; valid(tile) filters candidates (for example by the library's
    workspace query, which returns 0 for a tile whose subproblems do not fit
    LDS).  With use_cache an entry for this class is returned without timing
    anything, and a new choice is written to the cache file."""
    path = path or cache_path()
    key = cache_key(op, dtype, has_payload, size)
    if use_cache:
        entry = _load(path).get(key)
        if entry:
            return int(entry["tile"]), {int(k): v for k, v in entry["ms"].items()}
    cands = [t for t in (cands or TILES) if valid is None or valid(t)]
    if not cands:
        raise ValueError("no valid tile candidates")
    ms = {t: time_ms(lambda: run(t), reps=reps) for t in cands}
    best = min(ms, key=ms.get)
    if use_cache:
        cache = _load(path)
        cache[key] = {"tile": best, "ms": {str(t): v for t, v in ms.items()}}
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, ms
